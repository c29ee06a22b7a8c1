"""Whole runs of the loop at the MNIST shape (70,000 x 784, exact kNN) and at
the YAHOO shape (1.4M points, a kNN-shaped stand-in graph) against the FP64
oracle's runs of the same configuration from the same start.

Trajectories of the FP32 loop and the FP64 oracle part ways, so final
layouts are compared by statistics that a faulty loop would move:
* the final stress within 1e-4 relative: a 1e-7 relative nudge of the start
  moves it by 3e-9 (70K) and 4e-7 (1.4M) in the oracle itself, while a 10 %
  error in c moves it by 6 % (70K) and 0.12 % (1.4M);
* the kNN-preservation score Q_NX(10) within 0.01 (70K; the stand-in graph
  has no data space);
* the neighbour hit cf_10 within 0.01.
Statistics are computed by the oracle's metric functions on sampled rows."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ivhd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05455_amd as m
    return m


def f32(x):
    """The value a float parameter takes once it crosses the ABI (float32)."""
    return float(np.float32(x))


def _threads():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _gpu_run(ivhd, nn_idx, Y0, cfg, mode):
    y = torch.from_numpy(Y0.copy()).cuda()
    v = torch.zeros_like(y)
    ctx = ivhd.Context(torch.from_numpy(nn_idx).cuda(), y, v, rn=cfg.rn, a=cfg.a, b=cfg.b, c=cfg.c,
                       seed=cfg.seed, rn_resample_every=cfg.R, mode=mode)
    ctx.step(cfg.T)
    E = ctx.stress()
    rn = ctx.rn_edges().cpu().numpy()
    torch.cuda.synchronize()
    Yg = y.cpu().numpy()
    ctx.close()
    return Yg, rn, E


def _q_nx(v_rows, Y, rows, k=10):
    n = oracle.rank_neighbours(Y, k, rows)
    return float(np.mean([len(np.intersect1d(v_rows[r, :k], n[r])) for r in range(len(rows))]) / k)


@pytest.fixture(scope="module")
def c2():
    cfg = synth.CONFIGS["C2"]
    X, labels, Y0 = synth.make_inputs(cfg)
    knn10 = oracle.knn(X, 10)               # exact, FP64 (its first 5 columns are the 5-NN graph)
    nn_idx = np.ascontiguousarray(knn10[:, :cfg.nn])
    Yo, _, rno = oracle.run(Y0, np.zeros_like(Y0), nn_idx, rn=cfg.rn, a=f32(cfg.a), b=f32(cfg.b), c=f32(cfg.c), seed=cfg.seed,
                            R=cfg.R, T=cfg.T, threads=_threads())
    return cfg, X, labels, Y0, knn10, nn_idx, Yo, rno


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["det", "atomic"])
def test_c2_run_matches_the_oracle_run(ivhd, c2, mode):
    cfg, X, labels, Y0, knn10, nn_idx, Yo, rno = c2
    Yg, rng_, Eg = _gpu_run(ivhd, nn_idx, Y0, cfg, mode)
    assert np.array_equal(rng_, rno)        # the same last random-neighbour draw
    Eo = oracle.stress(Yo, nn_idx, rno, float(np.float32(cfg.c)))
    rows = np.sort(np.random.default_rng(1).choice(cfg.M, 2000, replace=False))
    # positions 1..10 of the data order are the exact 10-NN (no two rows coincide)
    q_g, q_o = _q_nx(knn10[rows], Yg, rows), _q_nx(knn10[rows], Yo, rows)
    cf_g, cf_o = oracle.cf_k(Yg, labels, 10, rows), oracle.cf_k(Yo, labels, 10, rows)
    print(f"C2 {mode}: E gpu={Eg:.6f} oracle={Eo:.6f}; Q_NX(10) {q_g:.4f} / {q_o:.4f} "
          f"(random {10 / (cfg.M - 1):.5f}); cf_10 {cf_g:.4f} / {cf_o:.4f}")
    assert abs(Eg - Eo) <= 1e-4 * Eo
    assert abs(q_g - q_o) <= 0.01
    assert abs(cf_g - cf_o) <= 0.01


@pytest.mark.timeout(900)
def test_c3_shape_run_matches_the_oracle_run(ivhd):
    cfg = synth.CONFIGS["C3"]
    nn_idx, labels, Y0 = synth.standin_graph(cfg, np.random.default_rng([0, 3, 7]))
    Yo, _, rno = oracle.run(Y0, np.zeros_like(Y0), nn_idx, rn=cfg.rn, a=f32(cfg.a), b=f32(cfg.b), c=f32(cfg.c), seed=cfg.seed,
                            R=cfg.R, T=cfg.T, threads=_threads())
    Eo = oracle.stress(Yo, nn_idx, rno, float(np.float32(cfg.c)))
    rows = np.sort(np.random.default_rng(1).choice(cfg.M, 300, replace=False))
    cf_o = oracle.cf_k(Yo, labels, 10, rows)
    for mode in ("det", "atomic"):
        Yg, rng_, Eg = _gpu_run(ivhd, nn_idx, Y0, cfg, mode)
        assert np.array_equal(rng_, rno)
        cf_g = oracle.cf_k(Yg, labels, 10, rows)
        print(f"C3 shape {mode}: E gpu={Eg:.6f} oracle={Eo:.6f}; cf_10 {cf_g:.4f} / {cf_o:.4f}")
        assert abs(Eg - Eo) <= 1e-4 * Eo
        assert abs(cf_g - cf_o) <= 0.01
