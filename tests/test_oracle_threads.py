"""The oracle's threaded loop (used only to time the oracle on every host
core) against its one-thread loop: the per-vertex gather adds the terms of a
vertex in the order the edge-by-edge scatter does, so the two agree bit for
bit, for any thread count, with absent slots, hubs, redraws and variants."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("kw", [dict(), dict(nesterov=True), dict(metric="l1"), dict(R=7)])
def test_threaded_loop_equals_the_one_thread_loop_bitwise(threads, kw):
    rng = np.random.default_rng(21)
    M, nn, rn = 1500, 3, 2
    labels = rng.integers(0, 5, M)
    nn_idx = synth.random_neighbour_graph(M, nn, rng, labels=labels, hub_alpha=1.2, absent_frac=0.05)
    Y0 = rng.random((M, 2))
    V0 = 0.01 * rng.normal(size=(M, 2))
    args = dict(rn=rn, a=0.9, b=0.004, c=0.1, seed=5, T=23, **({"R": 0} | kw))
    Y1, V1, r1 = oracle.run(Y0, V0, nn_idx, **args)
    Yt, Vt, rt = oracle.run(Y0, V0, nn_idx, threads=threads, **args)
    assert np.array_equal(r1, rt)
    assert np.array_equal(Y1.view(np.int64), Yt.view(np.int64))
    assert np.array_equal(V1.view(np.int64), Vt.view(np.int64))


def test_threaded_loop_on_the_oracle_size_config():
    cfg = synth.CONFIGS["C1"]
    X, labels, Y0 = synth.make_inputs(cfg)
    nn_idx = oracle.knn(X, cfg.nn)
    V0 = np.zeros_like(Y0, dtype=np.float64)
    args = dict(rn=cfg.rn, a=cfg.a, b=cfg.b, c=cfg.c, seed=cfg.seed, R=cfg.R, T=60)
    Y1, V1, _ = oracle.run(Y0, V0, nn_idx, **args)
    Yt, Vt, _ = oracle.run(Y0, V0, nn_idx, threads=4, **args)
    assert np.array_equal(Y1, Yt) and np.array_equal(V1, Vt)
