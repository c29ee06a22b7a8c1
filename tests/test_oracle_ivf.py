"""Pins of the FP64 inverted-file reference: probing every list is exact
kNN (the brute-force oracle, itself pinned against a kd-tree), Lloyd
iterations never raise the within-cluster sum of squares, one probe returns
only points of the query's own list, and a well separated mixture is split
along its clusters."""
import numpy as np
import pytest

import oracle
from oracle import ivf
import synth


def _data(M=600, N=6, K=8, seed=0, spread=6.0):
    rng = np.random.default_rng(seed)
    centres = rng.normal(0, spread, (K, N))
    lab = rng.integers(0, K, M)
    return centres[lab] + rng.normal(size=(M, N)), lab


def test_probing_every_list_is_exact_knn():
    X, _ = _data()
    C, a = ivf.ivf_train(X, 16, 3)
    got = ivf.ivf_search(X, C, a, X, 5, nprobe=16, self_idx=np.arange(len(X)))
    assert np.array_equal(got, oracle.knn(X, 5))


def test_lloyd_iterations_do_not_raise_the_inertia():
    X, _ = _data(seed=1)
    prev = np.inf
    for it in range(6):
        C, a = ivf.ivf_train(X, 12, it)
        cur = ivf.inertia(X, C, a)
        assert cur <= prev * (1 + 1e-12)
        prev = cur


def test_centroids_are_the_means_of_their_points():
    X, _ = _data(seed=2)
    C1, a1 = ivf.ivf_train(X, 10, 1)
    # one Lloyd step from the initial centroids, computed with a bincount
    C0 = X[(np.arange(10) * len(X)) // 10]
    a0 = ivf.assign(X, C0)
    cnt = np.bincount(a0, minlength=10)
    for n in range(X.shape[1]):
        means = np.bincount(a0, weights=X[:, n], minlength=10) / np.maximum(cnt, 1)
        np.testing.assert_allclose(C1[cnt > 0, n], means[cnt > 0], rtol=1e-12, atol=1e-12)


def test_one_probe_stays_in_the_query_list():
    X, _ = _data(seed=3)
    C, a = ivf.ivf_train(X, 10, 2)
    got = ivf.ivf_search(X, C, a, X[:50], 4, nprobe=1, self_idx=np.arange(50))
    for r in range(50):
        near = int(np.argmin(((C - X[r]) ** 2).sum(1)))
        valid = got[r][got[r] >= 0]
        assert np.all(a[valid] == near)


def test_separated_clusters_give_high_recall():
    cfg = synth.CONFIGS["C1"]
    X, labels, _ = synth.make_inputs(cfg)
    C, a = ivf.ivf_train(X, 20, 5)
    rows = np.arange(0, cfg.M, 7)
    got = ivf.ivf_search(X, C, a, X[rows], 5, nprobe=3, self_idx=rows)
    want = oracle.knn(X, 5, queries=rows)
    recall = np.mean([len(np.intersect1d(g, w)) / 5 for g, w in zip(got, want)])
    assert recall > 0.9
