"""Pins of the oracle's random-neighbour draw, exact kNN and quality metrics
(chapter "Quality metrics"): library routines on special cases, brute force
on tiny inputs, and the expected values of random layouts."""
import numpy as np
import pytest
from scipy import stats
from scipy.spatial import cKDTree
from sklearn.manifold import trustworthiness as sk_trustworthiness

import oracle
import synth


def test_rn_draw_respects_the_exclusion_rules():
    rng = np.random.default_rng(1)
    M, nn, rn = 500, 3, 4
    nn_idx = synth.random_neighbour_graph(M, nn, rng, absent_frac=0.1)
    for epoch in (0, 1, 17):
        r = oracle.rn_sample(nn_idx, rn, 42, epoch)
        assert r.shape == (M, rn) and r.min() >= 0 and r.max() < M
        assert np.all(r != np.arange(M)[:, None])
        for q in range(nn):
            assert np.all((r != nn_idx[:, q:q + 1]))
        srt = np.sort(r, axis=1)
        assert np.all(srt[:, 1:] != srt[:, :-1])


def test_rn_draw_is_a_pure_function_of_seed_and_epoch():
    rng = np.random.default_rng(2)
    nn_idx = synth.random_neighbour_graph(300, 2, rng)
    a = oracle.rn_sample(nn_idx, 1, 5, 3)
    assert np.array_equal(a, oracle.rn_sample(nn_idx, 1, 5, 3))
    assert not np.array_equal(a, oracle.rn_sample(nn_idx, 1, 5, 4))
    assert not np.array_equal(a, oracle.rn_sample(nn_idx, 1, 6, 3))


def test_rn_draw_is_uniform_over_the_allowed_vertices():
    # vertex 0 has no nn neighbours among 1..M-1 other than {1, 2}; its draws over
    # many epochs must be uniform on the M - 3 remaining vertices
    M = 41
    nn_idx = np.stack([(np.arange(M) + 1) % M, (np.arange(M) + 2) % M], 1).astype(np.int32)
    counts = np.zeros(M, np.int64)
    for e in range(4000):
        counts[oracle.rn_sample(nn_idx, 1, 9, e)[0, 0]] += 1
    assert counts[0] == counts[1] == counts[2] == 0
    obs = counts[3:]
    p = stats.chisquare(obs).pvalue
    assert p > 1e-4


def test_exact_knn_matches_a_kd_tree():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(700, 6))
    k = 5
    got = oracle.knn(X, k)
    d, idx = cKDTree(X).query(X, k=k + 1)
    assert np.array_equal(got, idx[:, 1:])
    q = np.array([5, 77, 699])
    assert np.array_equal(oracle.knn(X, k, queries=q), got[q])


def test_exact_knn_breaks_ties_by_index():
    # points on a line at integer spacing: the neighbours of 5 at distance 1 are 4 and 6
    X = np.arange(10, dtype=np.float64)[:, None]
    got = oracle.knn(X, 4)
    assert got[5].tolist() == [4, 6, 3, 7]
    assert got[0].tolist() == [1, 2, 3, 4]


def test_trustworthiness_matches_scikit_learn():
    rng = np.random.default_rng(4)
    X = rng.normal(size=(120, 8))
    Y = X[:, :2] + 0.3 * rng.normal(size=(120, 2))
    for k in (1, 5, 12):
        assert oracle.trustworthiness(X, Y, k) == pytest.approx(sk_trustworthiness(X, Y, n_neighbors=k), abs=1e-12)


def test_q_nx_brute_force_rank_definition():
    rng = np.random.default_rng(5)
    M, k = 25, 4
    X = rng.normal(size=(M, 5))
    Y = rng.normal(size=(M, 2))

    def sets(Z):
        d = ((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
        out = []
        for i in range(M):
            rho = [sum(1 for l in range(M) if d[i, l] < d[i, j] or (d[i, l] == d[i, j] and l < j))
                   for j in range(M)]
            out.append({j for j in range(M) if 1 <= rho[j] <= k})
        return out
    v, n = sets(X), sets(Y)
    want = sum(len(v[i] & n[i]) for i in range(M)) / (k * M)
    assert oracle.q_nx(X, Y, k) == pytest.approx(want, abs=0)


def test_q_nx_is_one_for_an_isometry_and_k_over_m_minus_1_for_random():
    rng = np.random.default_rng(6)
    X = rng.normal(size=(400, 2))
    assert oracle.q_nx(X, 3.0 * X + 1.0, 10) == 1.0
    assert oracle.r_nx(1.0, 10, 400) == 1.0
    qs = [oracle.q_nx(X, rng.normal(size=(400, 2)), 10) for _ in range(5)]
    assert np.mean(qs) == pytest.approx(10 / 399, abs=0.01)
    assert oracle.r_nx(np.mean(qs), 10, 400) == pytest.approx(0.0, abs=0.01)


def test_q_nx_on_a_sample_of_rows_agrees_with_full():
    rng = np.random.default_rng(7)
    X = rng.normal(size=(300, 4)); Y = X[:, :2] + 0.1 * rng.normal(size=(300, 2))
    full = oracle.q_nx(X, Y, 5)
    rows = np.arange(300)
    assert oracle.q_nx(X, Y, 5, rows=rows) == full


def test_neighbour_hit_of_separated_classes_is_one():
    rng = np.random.default_rng(8)
    lab = np.repeat(np.arange(4), 50)
    Y = np.array([[10.0 * l, 0.0] for l in lab]) + rng.normal(size=(200, 2))
    assert oracle.cf_k(Y, lab, 10) == 1.0
    r = oracle.cf_k(rng.normal(size=(200, 2)), lab, 10)
    assert r == pytest.approx(0.25, abs=0.06)


def test_auc_is_one_for_an_isometry():
    rng = np.random.default_rng(9)
    X = rng.normal(size=(30, 2))
    assert oracle.auc_rnx(X, 2 * X) == pytest.approx(1.0)


def test_knn_gain_is_zero_for_identical_neighbourhoods():
    rng = np.random.default_rng(10)
    X = rng.normal(size=(100, 2)); lab = rng.integers(0, 3, 100)
    assert oracle.g_nn(X, X, lab, 5) == 0.0


def _coranking_q_nx(X, Y):
    """Q_NX(k) for every k from the co-ranking matrix (Lee and Verleysen
    2009): Q[a, b] counts the pairs (i, j) whose rank is a in X and b in Y;
    Q_NX(k) is the sum of its top-left k x k block over kM.  Ranks by pure
    Python loops, ties broken by index as in the rank definition."""
    M = len(X)

    def ranks(Z):
        Z = np.asarray(Z, dtype=np.float64)
        d = [[float(((Z[i] - Z[j]) ** 2).sum()) for j in range(M)] for i in range(M)]
        return [[sum(1 for l in range(M) if d[i][l] < d[i][j] or (d[i][l] == d[i][j] and l < j))
                 for j in range(M)] for i in range(M)]
    rX, rY = ranks(X), ranks(Y)
    Q = np.zeros((M, M), dtype=np.int64)
    for i in range(M):
        for j in range(M):
            if i != j:
                Q[rX[i][j], rY[i][j]] += 1
    return [Q[1:k + 1, 1:k + 1].sum() / (k * M) for k in range(M)]


def test_auc_of_a_hand_computed_four_point_layout():
    # X = 0, 1, 3, 7 on a line; Y swaps the places of points 1 and 2.
    # k = 1: the nearest neighbours are {1}, {0}, {1}, {2} in X and {2}, {2}, {0}, {1}
    #        in Y, no agreement: Q = 0, R = (3 * 0 - 1) / (3 - 1) = -1/2.
    # k = 2: both sides give {1,2}, {0,2}, {0,1}, {1,2}: Q = 1, R = (3 - 2) / (3 - 2) = 1.
    # AUC = (R(1)/1 + R(2)/2) / (1 + 1/2) = 0.  Weights k (0.5), equal weights
    # (0.25), N in place of N - 1 in R (1/3) or a range up to k = N - 1 all differ.
    X = np.array([[0.0], [1.0], [3.0], [7.0]])
    Y = np.array([[0.0], [3.0], [1.0], [7.0]])
    assert oracle.q_nx(X, Y, 1) == 0.0 and oracle.q_nx(X, Y, 2) == 1.0
    assert oracle.auc_rnx(X, Y) == pytest.approx(0.0, abs=1e-15)
    # one more point (x = y = 15) so that the value is not zero.  Orders by hand:
    # k = 1: X {1},{0},{1},{2},{3}, Y {2},{2},{0},{1},{3}: one agreement, Q = 1/5,
    #        R = (4/5 - 1) / 3 = -1/15;
    # k = 2: agreements 2, 2, 2, 2, 1: Q = 9/10, R = (18/5 - 2) / 2 = 4/5;
    # k = 3: every set agrees: Q = 1, R = 1.
    # AUC = (-1/15 + 4/10 + 1/3) / (1 + 1/2 + 1/3) = (2/3) / (11/6) = 4/11.
    X5 = np.array([[0.0], [1.0], [3.0], [7.0], [15.0]])
    Y5 = np.array([[0.0], [3.0], [1.0], [7.0], [15.0]])
    assert [oracle.q_nx(X5, Y5, k) for k in (1, 2, 3)] == pytest.approx([0.2, 0.9, 1.0], abs=1e-15)
    assert oracle.auc_rnx(X5, Y5) == pytest.approx(4 / 11, abs=1e-15)


def test_auc_matches_the_coranking_matrix_on_random_layouts():
    rng = np.random.default_rng(11)
    for M in (9, 14):
        X = rng.normal(size=(M, 4))
        Y = X[:, :2] + 0.7 * rng.normal(size=(M, 2))
        q = _coranking_q_nx(X, Y)
        num = sum(((M - 1) * q[k] - k) / (M - 1 - k) / k for k in range(1, M - 1))
        den = sum(1.0 / k for k in range(1, M - 1))
        assert oracle.auc_rnx(X, Y) == pytest.approx(num / den, abs=1e-13)
        for k in (1, 3, M - 2):
            assert oracle.q_nx(X, Y, k) == pytest.approx(q[k], abs=1e-15)


def test_auc_of_random_layouts_is_near_zero():
    rng = np.random.default_rng(12)
    X = rng.normal(size=(30, 3))
    aucs = [oracle.auc_rnx(X, rng.normal(size=(30, 2))) for _ in range(20)]
    assert abs(np.mean(aucs)) < 0.05
    # a layout that keeps the structure scores well above that
    assert oracle.auc_rnx(X, X[:, :2]) > 0.3


def test_knn_gain_of_a_hand_computed_layout():
    # X = 0, 1, 3, 7 with classes A, B, A, B: the nearest neighbour of every
    # point is of the other class.  Y = 0, 10, 1, 11 pairs each point with its
    # own class.  k = 1: every point gains one same-class neighbour, G = +1.
    # k = 2: same-class counts are 1, 0, 1, 1 in X and 1, 1, 1, 1 in Y, so
    # G = (0 + 1 + 0 + 0) / 4 / 2 = 1/8.  Exchanging X and Y flips the sign.
    X = np.array([[0.0], [1.0], [3.0], [7.0]])
    Y = np.array([[0.0, 0.0], [10.0, 0.0], [1.0, 0.0], [11.0, 0.0]])
    lab = np.array([0, 1, 0, 1])
    assert oracle.g_nn(X, Y, lab, 1) == 1.0
    assert oracle.g_nn(X, Y, lab, 2) == 0.125
    assert oracle.g_nn(Y, X, lab, 1) == -1.0
    assert oracle.g_nn(Y, X, lab, 2) == -0.125


def test_exact_knn_expanded_narrowing_matches_a_kd_tree():
    # the large-input path (candidates narrowed by the expanded form, ranked
    # by the direct distance) on an input small enough for a kd-tree
    rng = np.random.default_rng(8)
    X = np.repeat(rng.normal(size=(1500, 12)), 1, 0) + rng.normal(scale=0.2, size=(1500, 12))
    k = 7
    got = oracle.knn(X, k, expanded_from=0)
    d, idx = cKDTree(X).query(X, k=k + 1)
    assert np.array_equal(got, idx[:, 1:])
    assert np.array_equal(got, oracle.knn(X, k))


def test_exact_knn_expanded_narrowing_keeps_the_tie_order():
    # exact duplicates and integer grids: many equal distances; both paths agree
    rng = np.random.default_rng(9)
    X = rng.integers(0, 4, size=(900, 3)).astype(np.float64)
    got = oracle.knn(X, 30, expanded_from=0)
    assert np.array_equal(got, oracle.knn(X, 30))
    # large offsets make the expanded form lose digits: rows fall back to the direct order
    Xo = X + 1e7
    assert np.array_equal(oracle.knn(Xo, 30, expanded_from=0), got)
