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
