"""FP64 reference of the approximate kNN index (an inverted file over a
k-means coarse quantizer), the stand-in for the approximate GPU library the
thesis builds its kNN graphs with (Sec. "IVHD-CUDA": kNN generation
dominates the end-to-end time).

TEST INFRASTRUCTURE ONLY: used by tests/, never by the product package; it
shares no code with the HIP path.

* ``ivf_train``: nlist centroids started at the points with indices
  floor(c M / nlist), then ``n_iter`` Lloyd iterations (assign every point to
  its nearest centroid, squared Euclidean distance, ties to the lower
  centroid index; move each centroid to the mean of its points, an empty one
  stays), then a final assignment.
* ``ivf_search``: per query the ``nprobe`` nearest centroids (ties to the
  lower index); the candidates are the points assigned to them (a query's
  own row excluded when asked); the answer is the k nearest candidates by
  (squared distance, index).  With nprobe = nlist this is the exact kNN.
"""
from __future__ import annotations

import numpy as np


def _sq_dists(A, B):
    """Squared Euclidean distances, FP64, as a plain difference (no expansion)."""
    out = np.empty((A.shape[0], B.shape[0]))
    for s in range(0, A.shape[0], 256):
        d = A[s:s + 256, None, :] - B[None, :, :]
        out[s:s + 256] = np.einsum("qcn,qcn->qc", d, d)
    return out


def assign(X, C):
    """Nearest centroid of every row (np.argmin keeps the lower index on ties)."""
    return np.argmin(_sq_dists(np.asarray(X, np.float64), np.asarray(C, np.float64)), axis=1).astype(np.int32)


def ivf_train(X, nlist: int, n_iter: int):
    """Returns (centroids float64 [nlist, N], assignment int32 [M])."""
    X = np.asarray(X, np.float64)
    M = X.shape[0]
    C = X[(np.arange(nlist) * M) // nlist].copy()
    for _ in range(n_iter):
        a = assign(X, C)
        for c in range(nlist):
            members = np.nonzero(a == c)[0]
            if members.size:
                C[c] = X[members].sum(axis=0) / members.size
    return C, assign(X, C)


def inertia(X, C, a):
    """Within-cluster sum of squared distances."""
    X = np.asarray(X, np.float64)
    d = X - np.asarray(C, np.float64)[a]
    return float(np.einsum("mn,mn->", d, d))


def ivf_search(X, C, a, Q, k: int, nprobe: int, self_idx=None):
    """k approximate nearest neighbours of each query row: int32 [len(Q), k]
    (-1 where fewer than k candidates were probed)."""
    X = np.asarray(X, np.float64)
    Q = np.asarray(Q, np.float64)
    dC = _sq_dists(Q, np.asarray(C, np.float64))
    probes = np.argsort(dC, axis=1, kind="stable")[:, :nprobe]
    lists = [np.nonzero(a == c)[0] for c in range(len(C))]
    out = np.full((Q.shape[0], k), -1, np.int32)
    for r in range(Q.shape[0]):
        cand = np.sort(np.concatenate([lists[c] for c in probes[r]]))
        if self_idx is not None and self_idx[r] >= 0:
            cand = cand[cand != self_idx[r]]
        t = X[cand] - Q[r]
        d = np.einsum("mn,mn->m", t, t)
        order = np.lexsort((cand, d))[:k]
        out[r, :order.size] = cand[order]
    return out
