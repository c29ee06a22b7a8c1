"""Pins of the FP64 oracle's stress, force and step against mathematics the
thesis fixes (Eq. ivhd_cost_function, Eq. eq13 with the sign of -1/2 grad E,
Eq. force_directed_update), not against the oracle itself."""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import laplacian

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _graph(M, nn, rn, seed, absent=0.0):
    rng = np.random.default_rng(seed)
    nn_idx = synth.random_neighbour_graph(M, nn, rng, absent_frac=absent)
    rn_idx = oracle.rn_sample(nn_idx, rn, seed, 0) if rn else np.zeros((M, 0), np.int32)
    Y = rng.normal(0, 1.0, size=(M, 2))
    return nn_idx, rn_idx, Y


def test_splitmix64_published_vectors():
    path = os.path.join(HERE, "golden", "splitmix64_vectors.txt")
    g = 0x9E3779B97F4A7C15
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert rows
    for s, n, want in rows:
        state = (int(s) + (int(n) - 1) * g) & 0xFFFFFFFFFFFFFFFF
        assert oracle.splitmix64(state) == int(want)


@pytest.mark.parametrize("nn,rn,absent", [(2, 1, 0.0), (3, 0, 0.0), (1, 2, 0.0), (5, 1, 0.2)])
def test_gradient_equals_finite_differences(nn, rn, absent):
    c = 0.1
    nn_idx, rn_idx, Y = _graph(40, nn, rn, 7, absent)
    g = oracle.grad(Y, nn_idx, rn_idx, c)
    h = 1e-6
    fd = np.zeros_like(Y)
    for i in range(Y.shape[0]):
        for a in range(2):
            Yp = Y.copy(); Yp[i, a] += h
            Ym = Y.copy(); Ym[i, a] -= h
            fd[i, a] = (oracle.stress(Yp, nn_idx, rn_idx, c) - oracle.stress(Ym, nn_idx, rn_idx, c)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * max(1.0, np.max(np.abs(g)))


def test_duplicate_nn_entry_counts_twice():
    # a directed multiset: listing j twice doubles that edge's term (mutual
    # pairs and repeats are not merged)
    Y = np.array([[0.0, 0.0], [1.0, 2.0], [3.0, -1.0]])
    once = np.array([[1, -1], [2, -1], [0, -1]], np.int32)
    twice = np.array([[1, 1], [2, -1], [0, -1]], np.int32)
    e1 = oracle.stress(Y, once, None, 0.1)
    e2 = oracle.stress(Y, twice, None, 0.1)
    assert e2 - e1 == pytest.approx(5.0)  # |y0 - y1|^2 counted once more


def test_zero_stress_and_force_at_target_distances():
    # two coincident groups at distance 1: nn edges inside groups (d = 0),
    # rn edges across (d = 1) meet every binary target exactly
    M = 8
    Y = np.zeros((M, 2)); Y[4:, 0] = 1.0
    nn_idx = np.array([[1], [2], [3], [0], [5], [6], [7], [4]], np.int32)
    rn_idx = np.array([[4], [5], [6], [7], [0], [1], [2], [3]], np.int32)
    assert oracle.stress(Y, nn_idx, rn_idx, 0.1) == 0.0
    assert np.all(oracle.force(Y, nn_idx, rn_idx, 0.1) == 0.0)
    Y1, V1 = oracle.step(Y, np.zeros_like(Y), oracle.force(Y, nn_idx, rn_idx, 0.1), 0.9, 0.05)
    assert np.array_equal(Y1, Y) and np.all(V1 == 0)


def test_translation_and_rotation_invariance():
    c = 0.1
    nn_idx, rn_idx, Y = _graph(60, 3, 1, 3)
    E = oracle.stress(Y, nn_idx, rn_idx, c)
    g = oracle.grad(Y, nn_idx, rn_idx, c)
    t = np.array([3.7, -12.5])
    assert oracle.stress(Y + t, nn_idx, rn_idx, c) == pytest.approx(E, rel=1e-12)
    np.testing.assert_allclose(oracle.grad(Y + t, nn_idx, rn_idx, c), g, atol=1e-10)
    th = 0.83
    Rm = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    assert oracle.stress(Y @ Rm.T, nn_idx, rn_idx, c) == pytest.approx(E, rel=1e-12)
    np.testing.assert_allclose(oracle.grad(Y @ Rm.T, nn_idx, rn_idx, c), g @ Rm.T, atol=1e-10)


def test_forces_cancel_pairwise_and_carry_no_torque():
    nn_idx, rn_idx, Y = _graph(200, 2, 1, 11)
    f = oracle.force(Y, nn_idx, rn_idx, 0.1)
    scale = np.abs(f).sum()
    assert np.all(np.abs(f.sum(0)) <= 1e-12 * scale)
    torque = np.sum(Y[:, 0] * f[:, 1] - Y[:, 1] * f[:, 0])
    assert abs(torque) <= 1e-12 * scale * np.abs(Y).max()


def test_rn_zero_is_the_graph_laplacian_quadratic_form():
    M = 50
    nn_idx, _, Y = _graph(M, 3, 0, 5, absent=0.1)
    src = np.repeat(np.arange(M), 3)
    dst = nn_idx.ravel()
    keep = dst >= 0
    A = sp.coo_matrix((np.ones(keep.sum()), (src[keep], dst[keep])), shape=(M, M)).toarray()
    L = laplacian(A + A.T)
    E = oracle.stress(Y, nn_idx, None, 0.5)
    assert E == pytest.approx(np.trace(Y.T @ L @ Y), rel=1e-12)
    np.testing.assert_allclose(oracle.grad(Y, nn_idx, None, 0.5), 2 * L @ Y, atol=1e-11)


def test_mutual_nn_pair_follows_its_recurrence():
    a, b = 0.8, 0.05
    Y0 = np.array([[0.0, 0.0], [1.5, 0.0]])
    nn_idx = np.array([[1], [0]], np.int32)
    Y, V, _ = oracle.run(Y0, np.zeros_like(Y0), nn_idx, rn=0, a=a, b=b, c=0.1, T=30)
    s_prev = s = Y0[0, 0] - Y0[1, 0]
    for _ in range(30):
        s, s_prev = (1 + a - 4 * b) * s - a * s_prev, s
    assert Y[0, 0] - Y[1, 0] == pytest.approx(s, rel=1e-12, abs=1e-14)


def test_mutual_rn_pair_follows_its_recurrence():
    # M = 2: the only random neighbour of each vertex is the other one
    a, b, c = 0.7, 0.1, 0.3
    Y0 = np.array([[0.0, 0.0], [0.2, 0.0]])
    nn_idx = np.zeros((2, 0), np.int32)
    Y, V, rn_idx = oracle.run(Y0, np.zeros_like(Y0), nn_idx, rn=1, a=a, b=b, c=c, T=12)
    assert rn_idx.ravel().tolist() == [1, 0]
    u_prev = u = 1.0 - 0.2
    for _ in range(12):
        u, u_prev = (1 + a - 4 * b * c) * u - a * u_prev, u
    assert Y[1, 0] - Y[0, 0] == pytest.approx(1.0 - u, rel=1e-12)
    assert np.all(Y[:, 1] == 0.0)


def test_rn_zero_heavy_ball_matches_eigendecomposition():
    M, a, b, T = 30, 0.9, 0.02, 40
    nn_idx, _, Y0 = _graph(M, 2, 0, 9)
    src = np.repeat(np.arange(M), 2)
    A = sp.coo_matrix((np.ones(2 * M), (src, nn_idx.ravel())), shape=(M, M)).toarray()
    lam, Q = np.linalg.eigh(laplacian(A + A.T))
    Z0 = Q.T @ Y0
    z_prev, z = Z0.copy(), Z0.copy()
    for _ in range(T):
        z, z_prev = (1 + a - b * lam)[:, None] * z - a * z_prev, z
    Y, _, _ = oracle.run(Y0, np.zeros_like(Y0), nn_idx, rn=0, a=a, b=b, c=0.1, T=T)
    np.testing.assert_allclose(Y, Q @ z, atol=1e-10)


def test_centroid_is_conserved_by_the_loop():
    nn_idx, _, Y0 = _graph(300, 2, 0, 13)
    Y, V, _ = oracle.run(Y0, np.zeros_like(Y0), nn_idx, rn=1, a=0.9, b=0.01, c=0.1, R=7, T=50)
    np.testing.assert_allclose(Y.mean(0), Y0.mean(0), atol=1e-12)
    np.testing.assert_allclose(V.sum(0), 0.0, atol=1e-12)


def test_frictionless_small_steps_descend():
    # a = 0 is plain gradient descent: with a small step E never increases
    nn_idx, _, Y0 = _graph(100, 2, 0, 17)
    rn_idx = oracle.rn_sample(nn_idx, 1, 0, 0)
    E_prev = oracle.stress(Y0, nn_idx, rn_idx, 0.1)
    Y, V = Y0.copy(), np.zeros_like(Y0)
    for n in range(40):
        Y, V, _ = oracle.run(Y, V, nn_idx, rn=1, a=0.0, b=0.005, c=0.1, R=0, n0=n, T=1)
        E = oracle.stress(Y, nn_idx, rn_idx, 0.1)
        assert E <= E_prev + 1e-12
        E_prev = E


def test_coincident_random_pair_gives_zero_force():
    # d = 0: the unit vector is undefined; the guard makes the term vanish
    Y = np.array([[0.3, 0.3], [0.3, 0.3]])
    f = oracle.force(Y, np.zeros((2, 0), np.int32), np.array([[1], [0]], np.int32), 0.1)
    assert np.all(f == 0.0)
    assert oracle.stress(Y, np.zeros((2, 0), np.int32), np.array([[1], [0]], np.int32), 0.1) == pytest.approx(0.2)
