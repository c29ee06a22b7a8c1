"""GPU evaluation of a layout (ivhd_eval_*, paper_2303_05455_amd.evaluate)
against the FP64 oracle's quality metrics: neighbourhoods and ranks by the
(distance, index) order, Q_NX(k), cf_k and T(k), element by element.  Both
sides decide the integer results in FP64, so the neighbour lists and ranks
must be equal, and the scores equal up to the last bit of a division."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05455_amd as p
    from paper_2303_05455_amd import evaluate
    return p, evaluate


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


@pytest.fixture(scope="module")
def c1():
    cfg = synth.CONFIGS["C1"]
    X, labels, Y0 = synth.make_inputs(cfg)
    # a layout with structure: the two leading principal axes
    Xc = X.astype(np.float64) - X.mean(0)
    Y = (Xc @ np.linalg.svd(Xc, full_matrices=False)[2][:2].T).astype(np.float32)
    return X, labels, Y


def test_neighbours_equal_the_rank_definition_on_c1(pkg, c1):
    p, _ = pkg
    X, labels, Y = c1
    M = X.shape[0]
    rows = np.arange(M, dtype=np.int32)
    for Z, k in ((X, 10), (Y, 100), (Y, 128), (X, 1)):
        got = p.ivhd_eval_neighbours(_t(Z), _t(rows, torch.int32), k).cpu().numpy()
        assert np.array_equal(got, oracle.rank_neighbours(Z, k)), (Z.shape, k)


@pytest.mark.parametrize("M,N,k,Q,seed", [(50, 3, 49, 50, 0), (777, 1, 7, 333, 1), (300, 1024, 5, 65, 2),
                                          (129, 2, 128, 1, 3)])
def test_neighbours_edge_sizes(pkg, M, N, k, Q, seed):
    p, _ = pkg
    rng = np.random.default_rng(seed)
    Z = rng.normal(size=(M, N)).astype(np.float32)
    rows = np.sort(rng.choice(M, Q, replace=False)).astype(np.int32)
    got = p.ivhd_eval_neighbours(_t(Z), _t(rows, torch.int32), k).cpu().numpy()
    assert np.array_equal(got, oracle.rank_neighbours(Z, k, rows))


def test_neighbours_and_ranks_break_ties_by_index(pkg):
    p, _ = pkg
    rng = np.random.default_rng(5)
    # integer points on a small grid, many of them repeated: distances tie exactly
    Z = rng.integers(0, 6, size=(400, 2)).astype(np.float32)
    rows = np.arange(400, dtype=np.int32)
    got = p.ivhd_eval_neighbours(_t(Z), _t(rows, torch.int32), 40).cpu().numpy()
    assert np.array_equal(got, oracle.rank_neighbours(Z, 40))
    cand = rng.integers(0, 400, size=(400, 9)).astype(np.int32)
    rk = p.ivhd_eval_ranks(_t(Z), _t(rows, torch.int32), _t(cand, torch.int32)).cpu().numpy()
    full = oracle._ranks_full(Z)
    assert np.array_equal(rk, full[rows[:, None], cand])


def test_ranks_equal_the_rank_definition_on_c1(pkg, c1):
    p, _ = pkg
    X, labels, Y = c1
    M = X.shape[0]
    rows = np.arange(0, M, 3, dtype=np.int32)
    cand = np.random.default_rng(7).integers(0, M, size=(rows.size, 17)).astype(np.int32)
    rk = p.ivhd_eval_ranks(_t(X), _t(rows, torch.int32), _t(cand, torch.int32)).cpu().numpy()
    full = oracle._ranks_full(X)
    assert np.array_equal(rk, full[rows[:, None], cand])


def test_scores_equal_the_oracle_metrics_on_c1_in_full(pkg, c1):
    _, ev = pkg
    X, labels, Y = c1
    M = X.shape[0]
    q = ev.quality(_t(X), _t(Y), np.arange(M), labels=labels, ks=(2, 10, 100), k_qnx=(1, 10, 30),
                   k_trust=(5, 10))
    for k in (1, 10, 30):
        assert q["q_nx"][k] == pytest.approx(oracle.q_nx(X, Y, k), rel=1e-15, abs=0)
    for k in (2, 10, 100):
        assert q["cf"][k] == pytest.approx(oracle.cf_k(Y, labels, k), rel=1e-15, abs=0)
    for k in (5, 10):
        assert q["trust"][k] == pytest.approx(oracle.trustworthiness(X, Y, k), rel=1e-13)
    # far from the random-layout value on this layout, so the comparison discriminates
    assert q["q_nx"][10] > 15 * q["q_nx_random"][10]


def test_scores_on_a_sample_of_the_mnist_shape(pkg):
    _, ev = pkg
    cfg = synth.CONFIGS["C2"]
    X, labels, Y0 = synth.make_inputs(cfg)
    rng = np.random.default_rng(11)
    Y = (X[:, :2] * 0.5 + rng.normal(0, 1.0, size=(cfg.M, 2))).astype(np.float32)
    rows = ev.sample_rows(cfg.M, 40, seed=2)
    dX = _t(X)
    q = ev.quality(dX, _t(Y), rows, labels=labels, ks=(2, 10, 100), k_qnx=(10,), k_trust=(10,))
    assert q["q_nx"][10] == pytest.approx(oracle.q_nx(X, Y, 10, rows), rel=1e-15, abs=0)
    for k in (2, 10, 100):
        assert q["cf"][k] == pytest.approx(oracle.cf_k(Y, labels, k, rows), rel=1e-15, abs=0)
    # the 2-D lists on a wider sample (cheap on the CPU)
    rows2 = ev.sample_rows(cfg.M, 1500, seed=3)
    import paper_2303_05455_amd as p
    got = p.ivhd_eval_neighbours(_t(Y), _t(rows2, torch.int32), 100).cpu().numpy()
    assert np.array_equal(got, oracle.rank_neighbours(Y, 100, rows2))


def test_neighbours_at_the_full_yahoo_shape_on_sampled_rows(pkg):
    p, _ = pkg
    cfg = synth.CONFIGS["C3"]
    X, labels, Y0 = synth.make_inputs(cfg)
    rows = np.array([0, 17, 700_001, cfg.M - 1], dtype=np.int32)
    got = p.ivhd_eval_neighbours(_t(X), _t(rows, torch.int32), 10).cpu().numpy()
    assert np.array_equal(got, oracle.rank_neighbours(X, 10, rows))
    rows2 = np.sort(np.random.default_rng(4).choice(cfg.M, 64, replace=False)).astype(np.int32)
    got = p.ivhd_eval_neighbours(_t(Y0), _t(rows2, torch.int32), 100).cpu().numpy()
    assert np.array_equal(got, oracle.rank_neighbours(Y0, 100, rows2))
