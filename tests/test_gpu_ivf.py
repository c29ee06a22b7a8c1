"""The inverted-file approximate kNN (through the C ABI) against the FP64
reference in oracle/ivf.py.

Search parity is checked on the reference's own index (its centroids,
rounded to FP32 as the GPU reads them, and its assignment): the answers must
agree row by row, except where a query sits within FP32 error of the
boundary between two probed / unprobed lists or two neighbours tie within
2e-6 (at most a few rows).  Training parity is checked on a well separated
mixture, where no point is near a tie.  At full size the checks are
properties: recall against the exact graph rising with nprobe, every answer in a
probed list, answers inside the query's cluster.
"""
import numpy as np
import pytest

import oracle
from oracle import ivf
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ivhd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05455_amd as m
    return m


def _mixture(M, N, K, seed, spread=4.0):
    rng = np.random.default_rng(seed)
    centres = rng.normal(0, spread, (K, N))
    return (centres[rng.integers(0, K, M)] + rng.normal(size=(M, N))).astype(np.float32)


def _sqd(X, q, idx):
    d = X[idx].astype(np.float64) - X[q].astype(np.float64)
    return np.einsum("kn,kn->k", d, d)


@pytest.mark.parametrize("M,N,nlist,nprobe,k,seed", [(3000, 20, 30, 4, 5, 0), (2000, 100, 16, 3, 10, 1),
                                                     (999, 7, 40, 7, 2, 2), (1500, 784, 12, 2, 20, 3)])
def test_search_matches_oracle_on_its_index(ivhd, M, N, nlist, nprobe, k, seed):
    X = _mixture(M, N, 8, seed)
    C, a = ivf.ivf_train(X, nlist, 3)
    C32 = C.astype(np.float32)
    want = ivf.ivf_search(X, C32.astype(np.float64), a, X, k, nprobe, self_idx=np.arange(M))
    dX = torch.from_numpy(X).cuda()
    got = ivhd.ivhd_ivf_search(dX, torch.from_numpy(C32).cuda(), torch.from_numpy(a).cuda(), dX, k, nprobe,
                               self_idx=torch.arange(M, dtype=torch.int32).cuda()).cpu().numpy()
    bad = 0
    for q in range(M):
        if np.array_equal(got[q], want[q]):
            continue
        g, w = got[q][got[q] >= 0], want[q][want[q] >= 0]
        if len(g) == len(w) and np.allclose(_sqd(X, q, g), _sqd(X, q, w), rtol=2e-6, atol=0):
            continue
        bad += 1
    assert bad <= max(2, M // 500), bad


def test_search_returns_distances_and_pads_short_lists(ivhd):
    X = _mixture(400, 6, 4, 4)
    C, a = ivf.ivf_train(X, 40, 2)
    dX = torch.from_numpy(X).cuda()
    idx, dist = ivhd.ivhd_ivf_search(dX, torch.from_numpy(C.astype(np.float32)).cuda(),
                                     torch.from_numpy(a).cuda(), dX[:50].contiguous(), 25, 1, with_dist=True)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for q in range(50):
        valid = idx[q] >= 0
        # without exclusion the query itself comes first; -1 only after the valid ones
        assert idx[q, 0] == q and dist[q, 0] == 0.0
        assert np.all(valid[:valid.sum()]) and not np.any(valid[valid.sum():])
        np.testing.assert_allclose(dist[q][valid], _sqd(X, q, idx[q][valid]), rtol=1e-5, atol=1e-6)
    assert (idx < 0).any()        # 40 lists of ~10 points: one probe cannot fill 25


def test_train_matches_oracle_on_separated_clusters(ivhd):
    cfg = synth.CONFIGS["C1"]
    X, labels, _ = synth.make_inputs(cfg)
    C, a = ivf.ivf_train(X, 10, 5)
    Cg, ag = ivhd.ivhd_ivf_train(torch.from_numpy(X).cuda(), 10, 5)
    assert np.array_equal(ag.cpu().numpy(), a)
    np.testing.assert_allclose(Cg.cpu().numpy(), C, rtol=1e-5, atol=1e-5)


def test_probing_all_but_one_list_is_nearly_exact(ivhd):
    X = _mixture(2500, 16, 6, 5)
    dX = torch.from_numpy(X).cuda()
    g = ivhd.ivf_knn_graph(dX, 5, nlist=8, nprobe=7, n_iter=4).cpu().numpy()
    exact = oracle.knn(X, 5)
    assert np.mean([len(np.intersect1d(g[i], exact[i])) for i in range(len(X))]) / 5 > 0.999


def test_full_size_recall_and_probe_membership(ivhd):
    # isotropic 100-D clusters have no local structure, so the recall of an
    # inverted file is modest here; it must grow with nprobe, and every answer
    # must come from a probed list
    cfg = synth.CONFIGS["C3"]
    X, labels, _ = synth.make_inputs(cfg)
    dX = torch.from_numpy(X).cuda()
    nlist = 1024
    C, a = ivhd.ivhd_ivf_train(dX, nlist, 6)
    me = torch.arange(cfg.M, dtype=torch.int32).cuda()
    exact = ivhd.ivhd_knn_build(dX, cfg.nn).cpu().numpy()
    rows = np.random.default_rng(9).choice(cfg.M, 20000, replace=False)
    recalls = []
    for nprobe in (4, 16):
        g = ivhd.ivhd_ivf_search(dX, C, a, dX, cfg.nn, nprobe, self_idx=me).cpu().numpy()
        recalls.append(np.mean([len(np.intersect1d(g[i], exact[i])) for i in rows]) / cfg.nn)
    assert recalls[1] > recalls[0] > 0.2, recalls
    Cn, an = C.cpu().numpy().astype(np.float64), a.cpu().numpy()
    for i in rows[:300]:
        d = ((Cn - X[i]) ** 2).sum(1)
        probed = set(np.argsort(d, kind="stable")[:16].tolist())
        assert all(an[j] in probed for j in g[i] if j >= 0)
    # clusters are well separated: the answers stay in the query's cluster
    assert np.mean(labels[g[rows, 0]] == labels[rows]) > 0.99


def test_bad_arguments(ivhd):
    X = _mixture(300, 4, 3, 6)
    dX = torch.from_numpy(X).cuda()
    C, a = ivhd.ivhd_ivf_train(dX, 8, 1)
    with pytest.raises(ivhd.IvhdError, match="nprobe"):
        ivhd.ivhd_ivf_search(dX, C, a, dX, 3, 8)
    with pytest.raises(ivhd.IvhdError, match="k ="):
        ivhd.ivhd_ivf_search(dX, C, a, dX, 29, 2)
    bad = a.clone()
    bad[5] = 8
    with pytest.raises(ivhd.IvhdError, match="outside"):
        ivhd.ivhd_ivf_search(dX, C, bad, dX, 3, 2)
    with pytest.raises(ivhd.IvhdError, match="nlist"):
        ivhd.ivhd_ivf_train(dX, 1, 1)
