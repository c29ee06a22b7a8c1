"""FP64 CPU oracle of the IVHD embedding loop and of its evaluation metrics.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product package.  It
shares no code with the HIP path; both read their inputs from ``synth``.

* ``ivhd_oracle.c`` (plain C, FP64): stress, force, the random-neighbour
  draw and the momentum loop, each written as the thesis defines it, with
  the thesis's variants: Nesterov look-ahead, the l1 distance of the late
  stage, and the reverse-neighbour edge mask.
* this module: the ctypes binding of that file, plus numpy FP64 versions of
  the exact kNN graph and of the quality metrics of the thesis's
  "Quality metrics" chapter (trustworthiness / continuity, neighbour hit,
  Q_NX / R_NX / AUC with the rank tie-break by index, kNN gain).
* ``mlp.py``: the FP64 reference of the parametric encoder.

Parity status of each function is stated in its docstring; every function
here is pinned by a test in ``tests/test_oracle_*.py`` against something
other than itself (finite differences, closed forms, invariants, a library
routine on a special case, or brute force on tiny inputs).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ivhd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libivhd_oracle.so")
_lock = threading.Lock()
_lib = None

GCC_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile ivhd_oracle.c with gcc into libivhd_oracle.so (in place)."""
    if not force and os.path.exists(_LIB_PATH) and \
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + f".tmp{os.getpid()}"
    subprocess.run(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        vp = ctypes.c_void_p
        lib.orc_splitmix64.argtypes = [u64]
        lib.orc_splitmix64.restype = u64
        lib.orc_rn_sample.argtypes = [i64, i32, vp, i32, u64, i64, vp]
        lib.orc_rn_sample.restype = None
        lib.orc_force.argtypes = [i64, vp, i32, vp, i32, vp, dbl, dbl, i32, vp]
        lib.orc_force.restype = None
        lib.orc_stress.argtypes = [i64, vp, i32, vp, i32, vp, dbl, i32]
        lib.orc_stress.restype = dbl
        lib.orc_rnn_mask.argtypes = [i64, i32, vp, i32, vp, vp]
        lib.orc_rnn_mask.restype = None
        lib.orc_run.argtypes = [i64, vp, vp, i32, vp, i32, vp, dbl, dbl, dbl, dbl, u64,
                                i64, i64, i64, i32, i32, vp, vp]
        lib.orc_run.restype = None
        lib.orc_run_threads.argtypes = lib.orc_run.argtypes + [i32]
        lib.orc_run_threads.restype = None
        lib.orc_run_adaptive.argtypes = [i64, vp, vp, i32, vp, i32, vp, dbl, vp, dbl, dbl, u64,
                                         i64, i64, i64, dbl, dbl, dbl, i32, vp, vp, vp, vp,
                                         vp, vp]
        lib.orc_run_adaptive.restype = i64
        lib.orc_run_adam.argtypes = [i64, vp, vp, vp, i32, vp, i32, vp, dbl, dbl, dbl, dbl, dbl,
                                     dbl, u64, i64, i64, i64, i64, i32, vp]
        lib.orc_run_adam.restype = None
        _lib = lib
        return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _graph(nn_idx, rn_idx=None):
    nn_idx = np.ascontiguousarray(nn_idx, dtype=np.int32)
    if nn_idx.ndim != 2:
        raise ValueError("nn_idx must be [M, nn]")
    if rn_idx is None:
        rn_idx = np.zeros((nn_idx.shape[0], 0), dtype=np.int32)
    rn_idx = np.ascontiguousarray(rn_idx, dtype=np.int32)
    return nn_idx, rn_idx


# ---------------------------------------------------------------------------
# the loop (C)
# ---------------------------------------------------------------------------

def splitmix64(x: int) -> int:
    """One SplitMix64 output for state ``x`` (gamma added, then mixed)."""
    return int(_load().orc_splitmix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def rn_sample(nn_idx, rn: int, seed: int, epoch: int) -> np.ndarray:
    """Random neighbours of one epoch, int32 [M, rn] (see ivhd_oracle.c)."""
    nn_idx, _ = _graph(nn_idx)
    M, nn = nn_idx.shape
    out = np.zeros((M, rn), dtype=np.int32)
    _load().orc_rn_sample(M, nn, _ptr(nn_idx), rn, seed & 0xFFFFFFFFFFFFFFFF, epoch, _ptr(out))
    return out


METRICS = {"l2": 0, "l1": 1}


def force(Y, nn_idx, rn_idx, c: float, eps: float = 1e-12, metric: str = "l2") -> np.ndarray:
    """f = -1/2 grad E in FP64, float64 [M, 2]; metric "l2" (Euclidean d) or
    "l1" (d = |dx| + |dy|, the late-stage variant)."""
    nn_idx, rn_idx = _graph(nn_idx, rn_idx)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    M = Y.shape[0]
    f = np.empty((M, 2), dtype=np.float64)
    _load().orc_force(M, _ptr(Y), nn_idx.shape[1], _ptr(nn_idx), rn_idx.shape[1], _ptr(rn_idx),
                      c, eps, METRICS[metric], _ptr(f))
    return f


def grad(Y, nn_idx, rn_idx, c: float, eps: float = 1e-12, metric: str = "l2") -> np.ndarray:
    """grad E = -2 f in FP64."""
    return -2.0 * force(Y, nn_idx, rn_idx, c, eps, metric)


def stress(Y, nn_idx, rn_idx, c: float, metric: str = "l2") -> float:
    """E(Y) in FP64 (Eq. ivhd_cost_function, with the Euclidean or the l1 distance)."""
    nn_idx, rn_idx = _graph(nn_idx, rn_idx)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    return float(_load().orc_stress(Y.shape[0], _ptr(Y), nn_idx.shape[1], _ptr(nn_idx),
                                    rn_idx.shape[1], _ptr(rn_idx), c, METRICS[metric]))


def rnn_mask(nn_idx, helper) -> np.ndarray:
    """Reverse-neighbour pruning: nn edge i -> j kept (else -1) when i is
    among the helper neighbours of j.  helper: int32 [M, kh]."""
    nn_idx, _ = _graph(nn_idx)
    helper = np.ascontiguousarray(helper, dtype=np.int32)
    M, nn = nn_idx.shape
    out = np.empty_like(nn_idx)
    _load().orc_rnn_mask(M, nn, _ptr(nn_idx), helper.shape[1], _ptr(helper), _ptr(out))
    return out


def step(Y, V, f, a: float, b: float):
    """One momentum update from a given force: (V', Y')."""
    V1 = a * np.asarray(V, np.float64) + b * np.asarray(f, np.float64)
    return np.asarray(Y, np.float64) + V1, V1


def run(Y0, V0, nn_idx, *, rn: int, a: float, b: float, c: float, eps: float = 1e-12,
        seed: int = 0, R: int = 0, n0: int = 0, T: int = 1, nesterov: bool = False,
        metric: str = "l2", threads: int = 0):
    """T iterations of the loop from (Y0, V0) at iteration n0 (with
    ``nesterov`` the force is taken at Y + a V).

    ``threads`` > 0 runs the same iterations on that many OpenMP threads
    (per-vertex gather in edge order: the same result bit for bit).

    Returns (Y, V, rn_idx) in FP64; rn_idx is the last epoch's draw.
    """
    nn_idx, _ = _graph(nn_idx)
    M, nn = nn_idx.shape
    Y = np.array(Y0, dtype=np.float64, order="C", copy=True)
    V = np.array(V0, dtype=np.float64, order="C", copy=True)
    rn_idx = np.zeros((M, rn), dtype=np.int32)
    f = np.empty((M, 2), dtype=np.float64)
    Yh = np.empty((M, 2), dtype=np.float64)
    args = (M, _ptr(Y), _ptr(V), nn, _ptr(nn_idx), rn, _ptr(rn_idx), a, b, c, eps,
            seed & 0xFFFFFFFFFFFFFFFF, R, n0, T, int(nesterov), METRICS[metric], _ptr(f), _ptr(Yh))
    if threads > 0:
        _load().orc_run_threads(*args, int(threads))
    else:
        _load().orc_run(*args)
    return Y, V, rn_idx


def run_adaptive(Y0, V0, nn_idx, *, rn: int, a: float, b: float, c: float, tau: float,
                 g1: float, g2: float, eps: float = 1e-12, seed: int = 0, R: int = 0,
                 n0: int = 0, T: int = 1, metric: str = "l2"):
    """T iterations with the self-adaptive b (see ivhd_oracle.c).

    Returns (Y, V, rn_idx, b, trace) with trace a dict of per-step arrays
    dT (kinetic energy change of the tentative step), b (the b it used) and
    kept (1 = step taken, 0 = rejected).
    """
    nn_idx, _ = _graph(nn_idx)
    M, nn = nn_idx.shape
    Y = np.array(Y0, dtype=np.float64, order="C", copy=True)
    V = np.array(V0, dtype=np.float64, order="C", copy=True)
    rn_idx = np.zeros((M, rn), dtype=np.int32)
    scratch = [np.empty((M, 2), dtype=np.float64) for _ in range(3)]
    dT = np.empty(T)
    bs = np.empty(T)
    kept = np.empty(T, dtype=np.int32)
    bb = ctypes.c_double(b)
    _load().orc_run_adaptive(M, _ptr(Y), _ptr(V), nn, _ptr(nn_idx), rn, _ptr(rn_idx), a,
                             ctypes.byref(bb), c, eps, seed & 0xFFFFFFFFFFFFFFFF, R, n0, T, tau,
                             g1, g2, METRICS[metric], _ptr(dT), _ptr(bs), _ptr(kept),
                             *[_ptr(x) for x in scratch])
    return Y, V, rn_idx, bb.value, {"dT": dT, "b": bs, "kept": kept}


def run_adam(Y0, nn_idx, *, rn: int, lr: float, c: float, b1: float = 0.9, b2: float = 0.999,
             eps_adam: float = 1e-8, eps: float = 1e-12, seed: int = 0, R: int = 0, n0: int = 0,
             T: int = 1, m0=None, s0=None, t0: int = 0, metric: str = "l2"):
    """T iterations of Adam on the stress (see ivhd_oracle.c).

    Returns (Y, m, s, rn_idx) in FP64; moments start at m0, s0 (zeros).
    """
    nn_idx, _ = _graph(nn_idx)
    M, nn = nn_idx.shape
    Y = np.array(Y0, dtype=np.float64, order="C", copy=True)
    Mo = np.zeros((M, 2)) if m0 is None else np.array(m0, dtype=np.float64, order="C", copy=True)
    S = np.zeros((M, 2)) if s0 is None else np.array(s0, dtype=np.float64, order="C", copy=True)
    rn_idx = np.zeros((M, rn), dtype=np.int32)
    f = np.empty((M, 2), dtype=np.float64)
    _load().orc_run_adam(M, _ptr(Y), _ptr(Mo), _ptr(S), nn, _ptr(nn_idx), rn, _ptr(rn_idx), lr, b1, b2,
                         eps_adam, c, eps, seed & 0xFFFFFFFFFFFFFFFF, R, n0, T, t0, METRICS[metric],
                         _ptr(f))
    return Y, Mo, S, rn_idx


# ---------------------------------------------------------------------------
# exact kNN (numpy, FP64)
# ---------------------------------------------------------------------------

def knn(X, k: int, queries=None, chunk: int = 512, expanded_from: int = 20_000) -> np.ndarray:
    """Exact k nearest neighbours by squared Euclidean distance in FP64.

    Self is excluded (for the rows of ``queries``, the query's own index),
    and ties are broken by the lower index, i.e. the order is (d, j), with
    d the direct sum over dimensions of squared differences.

    From ``expanded_from`` points on, each row's candidates are first
    narrowed with the expanded form |x|^2 + |y|^2 - 2 x.y (one BLAS product
    in FP64) to its k + 24 smallest; those are ranked by the direct d.  The
    narrowing is checked per row with the rounding bound of the expanded
    form, |error| <= 4 g (|x_q|^2 + max_j |x_j|^2), g = (N + 3) u / (1 - (N + 3) u),
    u = 2^-53 (Higham, "Accuracy and Stability of Numerical Algorithms",
    inner products): the k-th direct distance must lie below every
    excluded candidate's expanded value minus that bound, else the row is
    done in full.  So the result is the same as the plain definition.
    Returns int32 [len(queries), k].
    """
    X = np.asarray(X, dtype=np.float64)
    M, N = X.shape
    q_idx = np.arange(M) if queries is None else np.asarray(queries, dtype=np.int64)
    out = np.empty((q_idx.size, k), dtype=np.int32)

    def direct(q, cand=None):
        t = (X if cand is None else X[cand]) - X[q]
        return np.einsum("mn,mn->m", t, t)

    def full_row(q):
        d = direct(q)
        d[q] = np.inf
        return np.argsort(d, kind="stable")[:k]

    m = k + 24
    if M < expanded_from or m + 1 >= M:
        for s in range(0, q_idx.size, chunk):
            qi = q_idx[s:s + chunk]
            diff = X[qi][:, None, :] - X[None, :, :] if M * qi.size * N < 2e7 else None
            if diff is not None:
                d = np.einsum("qmn,qmn->qm", diff, diff)
                d[np.arange(qi.size), qi] = np.inf
                # stable sort on d keeps index order among equal distances
                out[s:s + qi.size] = np.argsort(d, axis=1, kind="stable")[:, :k]
            else:
                for r, q in enumerate(qi):
                    out[s + r] = full_row(q)
        return out
    sq = np.einsum("mn,mn->m", X, X)
    n3 = (N + 3) * 2.0 ** -53
    g = n3 / (1.0 - n3)
    sq_max = float(sq.max())
    for s in range(0, q_idx.size, chunk):
        qi = q_idx[s:s + chunk]
        G = sq[qi][:, None] + sq[None, :] - 2.0 * (X[qi] @ X.T)
        G[np.arange(qi.size), qi] = np.inf
        part = np.argpartition(G, m, axis=1)[:, :m + 1]
        for r, q in enumerate(qi):
            c = part[r]
            gc = G[r, c]
            o = np.lexsort((c, gc))
            c, gc = c[o], gc[o]
            cand, bound_value = c[:m], gc[m]       # every other candidate has G >= bound_value
            d = direct(q, cand)
            o = np.lexsort((cand, d))
            top, dk = cand[o[:k]], d[o[k - 1]]
            err = 4.0 * g * (sq[q] + sq_max)
            out[s + r] = top if bound_value - err > dk else full_row(q)
    return out


# ---------------------------------------------------------------------------
# quality metrics (numpy, FP64), chapter "Quality metrics"
# ---------------------------------------------------------------------------

def _sq_dists_rows(Z, rows):
    Z = np.asarray(Z, dtype=np.float64)
    out = np.empty((len(rows), Z.shape[0]))
    for r, i in enumerate(rows):
        t = Z - Z[i]
        out[r] = np.einsum("mn,mn->m", t, t)
    return out


def rank_neighbours(Z, k: int, rows=None) -> np.ndarray:
    """Sets v_i^k of the rank definition: the j with 1 <= rho_ij <= k.

    rho_ij = |{l : delta_il < delta_ij or (delta_il = delta_ij and l < j)}|,
    so all points (i included) are ordered by (distance, index) and the
    positions 1..k are taken.  Only the points at or below the (k+1)-th
    smallest distance can hold those positions, so just they are sorted
    (stably, which keeps the index order among equal distances).
    Returns int64 [len(rows), k].
    """
    M = np.asarray(Z).shape[0]
    rows = np.arange(M) if rows is None else np.asarray(rows)
    out = np.empty((rows.size, k), dtype=np.int64)
    for s in range(0, rows.size, 256):
        d = _sq_dists_rows(Z, rows[s:s + 256])
        for r in range(d.shape[0]):
            tau = np.partition(d[r], k)[k]
            cand = np.flatnonzero(d[r] <= tau)
            order = cand[np.argsort(d[r, cand], kind="stable")]
            out[s + r] = order[1:k + 1]
    return out


def q_nx(X, Y, k: int, rows=None) -> float:
    """Q_NX(k) = 1/(kM) sum_i |v_i^k & n_i^k| (neighbourhood preservation).

    With ``rows`` the mean runs over that sample of query points instead
    (each still ranked against all M points).
    """
    v = rank_neighbours(X, k, rows)
    n = rank_neighbours(Y, k, rows)
    hits = sum(len(np.intersect1d(v[r], n[r], assume_unique=True)) for r in range(v.shape[0]))
    return hits / (k * v.shape[0])


def r_nx(q: float, k: int, M: int) -> float:
    """R_NX(k) = ((M - 1) Q_NX(k) - k) / (M - 1 - k)."""
    return ((M - 1) * q - k) / (M - 1 - k)


def auc_rnx(X, Y) -> float:
    """AUC of R_NX(k) on a log axis: sum_k R_NX(k)/k / sum_k 1/k, k = 1..M-2."""
    M = np.asarray(X).shape[0]
    full_v = rank_neighbours(X, M - 1)
    full_n = rank_neighbours(Y, M - 1)
    num = den = 0.0
    for k in range(1, M - 1):
        hits = sum(len(np.intersect1d(full_v[i, :k], full_n[i, :k], assume_unique=True))
                   for i in range(M))
        num += r_nx(hits / (k * M), k, M) / k
        den += 1.0 / k
    return num / den


def cf_k(Y, labels, k: int, rows=None) -> float:
    """Neighbour hit cf_nn (Eq. eq12): the share of the k 2-D nearest
    neighbours of each point that carry its class label."""
    labels = np.asarray(labels)
    n = rank_neighbours(Y, k, rows)
    rows = np.arange(labels.size) if rows is None else np.asarray(rows)
    return float((labels[n] == labels[rows][:, None]).sum() / (k * rows.size))


def _ranks_full(Z):
    """r[i, j] = rho_ij (position of j in i's (distance, index) order)."""
    M = np.asarray(Z).shape[0]
    d = _sq_dists_rows(Z, np.arange(M))
    order = np.argsort(d, axis=1, kind="stable")
    r = np.empty_like(order)
    r[np.arange(M)[:, None], order] = np.arange(M)[None, :]
    return r


def trustworthiness(X, Y, k: int) -> float:
    """M1(k) = 1 - 2/(Mk(2M-3k-1)) sum_i sum_{j in U_k(i)} (r(x_i,x_j) - k),
    U_k(i): in the k-neighbourhood of y_i but not of x_i; r: rank in X."""
    M = np.asarray(X).shape[0]
    rX = _ranks_full(X)
    rY = _ranks_full(Y)
    s = 0.0
    for i in range(M):
        U = np.flatnonzero((rY[i] >= 1) & (rY[i] <= k) & ~((rX[i] >= 1) & (rX[i] <= k)))
        s += float((rX[i, U] - k).sum())
    return 1.0 - 2.0 / (M * k * (2 * M - 3 * k - 1)) * s


def continuity(X, Y, k: int) -> float:
    """M2(k): the same with the roles of X and Y exchanged."""
    return trustworthiness(Y, X, k)


def g_nn(X, Y, labels, k: int) -> float:
    """kNN gain G_NN(k): mean over i of (same-class count among the k 2-D
    neighbours - same-class count among the k N-D neighbours) / k."""
    labels = np.asarray(labels)
    v = rank_neighbours(X, k)
    n = rank_neighbours(Y, k)
    own = labels[:, None]
    return float(((labels[n] == own).sum(1) - (labels[v] == own).sum(1)).mean() / k)
