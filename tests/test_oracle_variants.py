"""Pins of the oracle's variants of the loop against mathematics, not against
the oracle itself:

* the l1 distance of the late stage (Sec. "L1 norm in late stages of
  embedding"): finite differences of the l1 stress, hand-computed two-point
  values, reduction to the Euclidean case on an axis;
* the Nesterov look-ahead (Sec. "Optimization methods", Nesterov): a = 0
  reduces to the plain loop, the mutual-pair recurrence, and the rn = 0 case
  as a matrix recurrence with the graph Laplacian;
* the reverse-neighbour mask (Sec. "Reverse neighbors mechanism"): checked
  from raw distances of the data, not from the helper list.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import laplacian

import oracle
import synth


def _graph(M, nn, rn, seed, absent=0.0):
    rng = np.random.default_rng(seed)
    nn_idx = synth.random_neighbour_graph(M, nn, rng, absent_frac=absent)
    rn_idx = oracle.rn_sample(nn_idx, rn, seed, 0) if rn else np.zeros((M, 0), np.int32)
    Y = rng.normal(0, 0.4, size=(M, 2))
    return nn_idx, rn_idx, Y


# ---- l1 distance ----------------------------------------------------------

@pytest.mark.parametrize("nn,rn,absent", [(2, 1, 0.0), (3, 2, 0.1), (1, 0, 0.0)])
def test_l1_gradient_equals_finite_differences(nn, rn, absent):
    c = 0.3
    nn_idx, rn_idx, Y = _graph(30, nn, rn, 3, absent)
    g = oracle.grad(Y, nn_idx, rn_idx, c, metric="l1")
    h = 1e-7
    fd = np.empty_like(Y)
    for i in range(Y.shape[0]):
        for a in range(2):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, a] += h
            Ym[i, a] -= h
            fd[i, a] = (oracle.stress(Yp, nn_idx, rn_idx, c, "l1")
                        - oracle.stress(Ym, nn_idx, rn_idx, c, "l1")) / (2 * h)
    # random Gaussian coordinates: no coordinate difference within h of zero
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-6)


def test_l1_two_point_values_by_hand():
    Y = np.array([[0.0, 0.0], [1.0, 2.0]])
    nn_idx = np.array([[1], [-1]], np.int32)
    # d1 = 3: E = 9; d E / d y0 = 2 * 3 * sign(0 - 1, 0 - 2) = (-6, -6); f = -1/2 grad
    assert oracle.stress(Y, nn_idx, None, 0.5, "l1") == 9.0
    np.testing.assert_array_equal(oracle.force(Y, nn_idx, None, 0.5, metric="l1"), [[3, 3], [-3, -3]])
    # rn edge at d1 = 0.5: E = c (1 - 0.5)^2, f0 = c (1 - 0.5) sign(y0 - y1) = c/2 (-1, -1)
    Y = np.array([[0.0, 0.0], [0.25, 0.25]])
    none = np.zeros((2, 0), np.int32)
    rn_idx = np.array([[1], [-1]], np.int32)
    c = 0.2
    assert oracle.stress(Y, none, rn_idx, c, "l1") == pytest.approx(c * 0.25, rel=1e-15)
    np.testing.assert_allclose(oracle.force(Y, none, rn_idx, c, metric="l1"),
                               [[-c / 2, -c / 2], [c / 2, c / 2]], rtol=1e-15)
    # a zero coordinate difference contributes no force along that axis:
    # d1 = 3, f0 = -3 (sign 0, sign -3) = (0, 3)
    Y = np.array([[0.0, 0.0], [0.0, 3.0]])
    f = oracle.force(Y, np.array([[1], [-1]], np.int32), None, 0.5, metric="l1")
    assert f[0, 0] == 0.0 and f[0, 1] == 3.0


def test_l1_on_one_axis_is_the_euclidean_case():
    nn_idx, rn_idx, Y = _graph(40, 2, 1, 8)
    Y[:, 1] = 0.0
    assert oracle.stress(Y, nn_idx, rn_idx, 0.1, "l1") == pytest.approx(
        oracle.stress(Y, nn_idx, rn_idx, 0.1, "l2"), rel=1e-13)
    np.testing.assert_allclose(oracle.force(Y, nn_idx, rn_idx, 0.1, metric="l1"),
                               oracle.force(Y, nn_idx, rn_idx, 0.1, metric="l2"), atol=1e-13)


def test_l1_forces_cancel_in_pairs_and_ignore_translation():
    nn_idx, rn_idx, Y = _graph(60, 3, 1, 11)
    f = oracle.force(Y, nn_idx, rn_idx, 0.1, metric="l1")
    assert np.abs(f.sum(0)).max() <= 1e-12 * np.abs(f).sum()
    t = np.array([3.25, -1.5])
    np.testing.assert_allclose(oracle.force(Y + t, nn_idx, rn_idx, 0.1, metric="l1"), f, atol=1e-12)
    # the l1 distance is invariant under axis swaps and reflections
    E = oracle.stress(Y, nn_idx, rn_idx, 0.1, "l1")
    assert oracle.stress(Y[:, ::-1], nn_idx, rn_idx, 0.1, "l1") == pytest.approx(E, rel=1e-13)
    assert oracle.stress(-Y, nn_idx, rn_idx, 0.1, "l1") == pytest.approx(E, rel=1e-13)


def test_l1_zero_at_targets():
    # nn ends coincide, rn ends at l1 distance exactly 1: E = 0 and f = 0
    M = 20
    Y = np.zeros((M, 2))
    Y[M // 2:, 0] = 1.0
    nn_idx = np.array([[(i + 1) % (M // 2) + (i // (M // 2)) * (M // 2)] for i in range(M)], np.int32)
    rn_idx = np.array([[(i + M // 2) % M] for i in range(M)], np.int32)
    assert oracle.stress(Y, nn_idx, rn_idx, 0.1, "l1") == 0.0
    assert np.all(oracle.force(Y, nn_idx, rn_idx, 0.1, metric="l1") == 0.0)


# ---- Nesterov look-ahead ---------------------------------------------------

def test_nesterov_with_zero_momentum_is_the_plain_loop():
    nn_idx, _, Y0 = _graph(80, 2, 0, 4)
    V0 = np.random.default_rng(1).normal(0, 0.01, Y0.shape)
    for metric in ("l2", "l1"):
        A = oracle.run(Y0, V0, nn_idx, rn=1, a=0.0, b=0.02, c=0.1, T=9, R=4, metric=metric)
        B = oracle.run(Y0, V0, nn_idx, rn=1, a=0.0, b=0.02, c=0.1, T=9, R=4, metric=metric,
                       nesterov=True)
        for x, y in zip(A, B):
            np.testing.assert_array_equal(x, y)


def test_nesterov_mutual_nn_pair_follows_its_recurrence():
    # separation u, velocity w: u_hat = u + a w, w' = a w - 4 b u_hat, u' = u + w'
    # => u_{n+1} = (1 - 4b) ((1 + a) u_n - a u_{n-1})
    a, b = 0.85, 0.04
    Y0 = np.array([[0.0, 0.0], [1.5, 0.0]])
    V0 = np.array([[0.1, 0.0], [-0.05, 0.0]])
    nn_idx = np.array([[1], [0]], np.int32)
    Y, V, _ = oracle.run(Y0, V0, nn_idx, rn=0, a=a, b=b, c=0.1, T=25, nesterov=True)
    u = Y0[0, 0] - Y0[1, 0]
    u_prev = u - (V0[0, 0] - V0[1, 0])
    for _ in range(25):
        u, u_prev = (1 - 4 * b) * ((1 + a) * u - a * u_prev), u
    assert Y[0, 0] - Y[1, 0] == pytest.approx(u, rel=1e-12, abs=1e-14)


def test_nesterov_rn_zero_is_a_laplacian_matrix_recurrence():
    # f = -L Y for rn = 0, so Y_{n+1} = (I - b L) (Y_n + a (Y_n - Y_{n-1}))
    M, a, b, T = 40, 0.9, 0.03, 30
    nn_idx, _, Y0 = _graph(M, 3, 0, 21, absent=0.1)
    src = np.repeat(np.arange(M), 3)
    dst = nn_idx.ravel()
    keep = dst >= 0
    A = sp.coo_matrix((np.ones(keep.sum()), (src[keep], dst[keep])), shape=(M, M)).toarray()
    L = laplacian(A + A.T)
    V0 = np.random.default_rng(2).normal(0, 0.05, Y0.shape)
    Yp, Yc = Y0 - V0, Y0.copy()
    for _ in range(T):
        Yc, Yp = (np.eye(M) - b * L) @ (Yc + a * (Yc - Yp)), Yc
    Y, V, _ = oracle.run(Y0, V0, nn_idx, rn=0, a=a, b=b, c=0.1, T=T, nesterov=True)
    np.testing.assert_allclose(Y, Yc, atol=1e-10)
    np.testing.assert_allclose(V, Yc - Yp, atol=1e-10)


# ---- reverse-neighbour mask ------------------------------------------------

def test_rnn_mask_from_raw_distances():
    rng = np.random.default_rng(6)
    M, N, nn = 120, 6, 3
    X = rng.normal(size=(M, N))
    nn_idx = oracle.knn(X, nn)
    helper = oracle.knn(X, 4 * nn)
    out = oracle.rnn_mask(nn_idx, helper)
    D = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(D, np.inf)
    kth = np.sort(D, axis=1)[:, 4 * nn - 1]        # distance of each point's 4nn-th neighbour
    kept = 0
    for i in range(M):
        for q in range(nn):
            j = nn_idx[i, q]
            want = j if D[j, i] <= kth[j] else -1   # i lies in the 4nn-ball of j
            assert out[i, q] == want
            kept += want >= 0
    assert 0 < kept < M * nn                       # the mask prunes some edges, not all
    # a mutual nn pair is always kept
    for i in range(M):
        for j in nn_idx[i]:
            if i in nn_idx[j]:
                assert j in out[i]


def test_rnn_mask_keeps_absent_slots_absent():
    nn_idx = np.array([[1, -1], [0, 2], [1, 0]], np.int32)
    helper = np.array([[1, 2], [0, 2], [0, 1]], np.int32)
    np.testing.assert_array_equal(oracle.rnn_mask(nn_idx, helper), [[1, -1], [0, 2], [1, 0]])
    helper = np.array([[2, 2], [2, 2], [0, 0]], np.int32)
    np.testing.assert_array_equal(oracle.rnn_mask(nn_idx, helper), [[-1, -1], [-1, -1], [1, 0]])


# ---- self-adaptive b -------------------------------------------------------

def _adaptive_case(seed=5, M=60):
    nn_idx, _, Y0 = _graph(M, 3, 0, seed)
    V0 = np.random.default_rng(seed + 1).normal(0, 0.02, Y0.shape)
    return nn_idx, Y0, V0


def test_adaptive_with_infinite_tau_is_the_plain_loop():
    nn_idx, Y0, V0 = _adaptive_case()
    Y, V, rn_idx, b, tr = oracle.run_adaptive(Y0, V0, nn_idx, rn=1, a=0.9, b=0.02, c=0.1,
                                              tau=np.inf, g1=1.1, g2=0.5, R=5, T=17)
    Yp, Vp, rnp = oracle.run(Y0, V0, nn_idx, rn=1, a=0.9, b=0.02, c=0.1, R=5, T=17)
    np.testing.assert_array_equal(Y, Yp)
    np.testing.assert_array_equal(V, Vp)
    np.testing.assert_array_equal(rn_idx, rnp)
    assert b == 0.02 and tr["kept"].all()


def test_adaptive_steps_are_plain_steps_or_no_move():
    # step by step: a kept step equals one plain step with the b it used, a
    # rejected one leaves (Y, V) as they were; dT is the kinetic energy change
    nn_idx, Y, V = _adaptive_case(seed=9)
    b, tau, n_rej = 0.09, 2e-3, 0
    for n in range(40):
        Y1, V1, _, b1, tr = oracle.run_adaptive(Y, V, nn_idx, rn=1, a=0.9, b=b, c=0.1, tau=tau,
                                                g1=1.25, g2=0.5, R=8, n0=n, T=1)
        Yp, Vp, _ = oracle.run(Y, V, nn_idx, rn=1, a=0.9, b=b, c=0.1, R=8, n0=n, T=1)
        dT = (Vp ** 2).sum() - (V ** 2).sum()
        assert tr["dT"][0] == pytest.approx(dT, rel=1e-9, abs=1e-15)
        if tr["kept"][0]:
            np.testing.assert_array_equal(Y1, Yp)
            assert abs(dT) <= tau and b1 == b
        else:
            np.testing.assert_array_equal(Y1, Y)
            np.testing.assert_array_equal(V1, V)
            assert b1 == pytest.approx(b * (1.25 if dT < -tau else 0.5), rel=1e-15)
            n_rej += 1
        Y, V, b = Y1, V1, b1
    assert 0 < n_rej < 40


def test_adaptive_b_tames_a_step_that_diverges():
    nn_idx, Y0, V0 = _adaptive_case(seed=12, M=100)
    b_bad = 1.5                                  # far beyond 2 (1 + a) / lambda_max
    Yp, _, _ = oracle.run(Y0, V0, nn_idx, rn=1, a=0.9, b=b_bad, c=0.1, T=60)
    assert not np.all(np.abs(Yp) < 1e6)
    Y, V, _, b, tr = oracle.run_adaptive(Y0, V0, nn_idx, rn=1, a=0.9, b=b_bad, c=0.1, tau=1.0,
                                         g1=1.05, g2=0.5, T=60)
    assert np.all(np.isfinite(Y)) and np.abs(Y).max() < 100
    assert b < b_bad and tr["kept"].sum() > 0


# ---- Adam on the stress ----------------------------------------------------

def test_adam_matches_torch_adam_on_the_same_gradients():
    torch = pytest.importorskip("torch")
    nn_idx, rn_idx, Y0 = _graph(50, 3, 1, 17)
    lr, b1, b2, eps_a, c, T = 0.01, 0.9, 0.999, 1e-8, 0.1, 12
    Y, Mo, S, rn_got = oracle.run_adam(Y0, nn_idx, rn=1, lr=lr, c=c, b1=b1, b2=b2, eps_adam=eps_a,
                                       seed=3, T=T)
    rn_idx = oracle.rn_sample(nn_idx, 1, 3, 0)
    assert np.array_equal(rn_got, rn_idx)
    p = torch.tensor(Y0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=(b1, b2), eps=eps_a)
    for _ in range(T):
        opt.zero_grad()
        p.grad = torch.from_numpy(oracle.grad(p.detach().numpy(), nn_idx, rn_idx, c))
        opt.step()
    np.testing.assert_allclose(Y, p.detach().numpy(), rtol=1e-12, atol=1e-12)
    st = opt.state[p]
    np.testing.assert_allclose(Mo, st["exp_avg"].numpy(), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(S, st["exp_avg_sq"].numpy(), rtol=1e-12, atol=1e-18)


def test_adam_split_runs_resume_with_their_moments():
    nn_idx, _, Y0 = _graph(40, 2, 0, 18)
    A = oracle.run_adam(Y0, nn_idx, rn=1, lr=0.02, c=0.1, R=3, T=10)
    Y1, m1, s1, _ = oracle.run_adam(Y0, nn_idx, rn=1, lr=0.02, c=0.1, R=3, T=4)
    B = oracle.run_adam(Y1, nn_idx, rn=1, lr=0.02, c=0.1, R=3, n0=4, T=6, m0=m1, s0=s1, t0=4)
    for x, y in zip(A[:3], B[:3]):
        np.testing.assert_array_equal(x, y)
