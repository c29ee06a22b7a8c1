"""The MFMA brute-force kNN builder against the FP64 oracle.

The order is unique under (distance, index); FP32 may swap neighbours whose
FP64 distances agree to about 1e-6, so a row that differs from the oracle
must still pick neighbours whose exact distances match the oracle's, rank by
rank, within that relative gap.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ivhd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05455_amd as m
    return m


def _sqd(X, q, idx):
    d = X[idx].astype(np.float64) - X[q].astype(np.float64)
    return np.einsum("kn,kn->k", d, d)


def _check_rows(X, rows, got, want, rel=2e-6):
    bad = 0
    for r, q in enumerate(rows):
        g, w = got[r], want[r]
        assert len(set(g.tolist())) == len(g), f"row {q}: duplicate neighbours"
        assert q not in g, f"row {q}: self returned"
        assert g.min() >= 0
        if np.array_equal(g, w):
            continue
        dg, dw = _sqd(X, q, g), _sqd(X, q, w)
        assert np.allclose(dg, dw, rtol=rel, atol=0), f"row {q}: {g} vs {w}, {dg} vs {dw}"
        bad += 1
    return bad


# padded widths 32, 64, 96, 128 (register-resident queries; with k + 4 > 16
# at 128 the general kernel) and 224, 800 (general kernel), every list length
# (k + 4 <= 8, <= 16, <= 32) on both kernels
@pytest.mark.parametrize("M,N,k,seed", [(3000, 32, 2, 0), (1000, 100, 5, 1), (513, 7, 10, 2),
                                        (200, 784, 20, 3), (777, 2, 3, 4), (40, 16, 28, 5),
                                        (5, 3, 4, 6), (1500, 50, 3, 7), (900, 90, 12, 8),
                                        (600, 120, 25, 9), (700, 60, 28, 10), (500, 90, 20, 11),
                                        (1000, 200, 3, 12), (333, 150, 9, 13)])
def test_knn_build_matches_oracle(ivhd, M, N, k, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(M, N)).astype(np.float32)
    got = ivhd.ivhd_knn_build(torch.from_numpy(X).cuda(), k).cpu().numpy()
    want = oracle.knn(X, k)
    bad = _check_rows(X, np.arange(M), got, want)
    assert bad <= max(1, M // 1000)


def test_knn_on_a_clustered_mixture(ivhd):
    cfg = synth.CONFIGS["C1"]
    X, labels, _ = synth.make_inputs(cfg)
    got = ivhd.ivhd_knn_build(torch.from_numpy(X).cuda(), cfg.nn).cpu().numpy()
    assert _check_rows(X, np.arange(cfg.M), got, oracle.knn(X, cfg.nn)) == 0


def test_knn_ties_go_to_the_lower_index(ivhd):
    # integer points on a line: exact FP32 distances, many ties
    X = np.zeros((64, 4), np.float32)
    X[:, 0] = np.arange(64)
    got = ivhd.ivhd_knn_build(torch.from_numpy(X).cuda(), 4).cpu().numpy()
    assert np.array_equal(got, oracle.knn(X, 4))


@pytest.mark.parametrize("N", [24, 150])
def test_knn_query_with_self_and_distances(ivhd, N):
    rng = np.random.default_rng(7)
    X = rng.normal(size=(2000, N)).astype(np.float32)
    rows = rng.choice(2000, 300, replace=False)
    dX = torch.from_numpy(X).cuda()
    idx, dist = ivhd.ivhd_knn_query(dX, dX[torch.from_numpy(rows).cuda()].contiguous(), 6,
                                    self_idx=torch.from_numpy(rows.astype(np.int32)).cuda(),
                                    with_dist=True)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    want = oracle.knn(X, 6, queries=rows)
    assert _check_rows(X, rows, idx, want) <= 1
    for r, q in enumerate(rows):
        np.testing.assert_allclose(dist[r], _sqd(X, q, idx[r]), rtol=1e-5)
    # without exclusion the query itself comes first at distance 0
    idx0 = ivhd.ivhd_knn_query(dX, dX[:10].contiguous(), 3).cpu().numpy()
    assert np.array_equal(idx0[:, 0], np.arange(10))


def test_knn_at_mnist_shape_on_sampled_rows(ivhd):
    cfg = synth.CONFIGS["C2"]
    X, labels, _ = synth.make_inputs(cfg)
    got = ivhd.ivhd_knn_build(torch.from_numpy(X).cuda(), cfg.nn).cpu().numpy()
    rows = np.random.default_rng(0).choice(cfg.M, 200, replace=False)
    assert _check_rows(X, rows, got[rows], oracle.knn(X, cfg.nn, queries=rows)) <= 2


@pytest.mark.slow
def test_knn_at_full_size_on_sampled_rows(ivhd):
    cfg = synth.CONFIGS["C3"]
    X, labels, _ = synth.make_inputs(cfg)
    got = ivhd.ivhd_knn_build(torch.from_numpy(X).cuda(), cfg.nn).cpu().numpy()
    rows = np.random.default_rng(1).choice(cfg.M, 24, replace=False)
    assert _check_rows(X, rows, got[rows], oracle.knn(X, cfg.nn, queries=rows, chunk=4)) <= 1
    # every vertex's neighbours sit in its own cluster for this well separated mixture
    assert np.mean(labels[got[:, 0]] == labels) > 0.999
