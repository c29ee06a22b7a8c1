"""Python binding of the C ABI in include/ivhd.h.

The functions keep the C names and only marshal arguments: torch tensors
give device pointers and the current HIP stream; every computation runs in
libivhd's kernels.  ``Context`` is a small convenience wrapper that keeps the
tensors a context points at alive.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import IvhdError, check, ivhd_params

MODES = {"det": 0, "atomic": 1}

__all__ = [
    "IvhdError", "Context", "make_params", "ivhd_init", "ivhd_step", "ivhd_stress", "ivhd_grad",
    "ivhd_get_rn", "ivhd_get_in_edges", "ivhd_get_order", "ivhd_set_state", "ivhd_set_iteration",
    "ivhd_get_iteration", "ivhd_set_graphs", "ivhd_destroy", "ivhd_last_error",
    "ivhd_version", "ivhd_knn_build", "ivhd_knn_query", "ivhd_edges_create", "ivhd_edges_stress",
    "ivhd_edges_grad", "ivhd_edges_stress_grad", "ivhd_scale_f32", "ivhd_edges_destroy", "ivhd_grad_edges",
    "ivhd_grad_edges_noalloc", "ivhd_set_adaptive",
    "ivhd_get_adaptive", "ivhd_rnn_mask", "ivhd_set_adam", "ivhd_ivf_train", "ivhd_ivf_search",
    "ivf_knn_graph", "ivhd_eval_neighbours", "ivhd_eval_ranks", "ivhd_eval_scores", "ivhd_probe_gather",
    "ivhd_probe_atomic",
]


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev(t: torch.Tensor, dtype, shape, name: str) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a HIP device, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


FLAG_REORDER, FLAG_NESTEROV, FLAG_L1 = 1, 2, 4
METRICS = {"l2": 0, "l1": FLAG_L1}


def make_params(M: int, nn: int, rn: int, *, a: float, b: float, c: float, eps: float = 1e-12,
                seed: int = 0, rn_resample_every: int = 0, mode: str = "det",
                reorder: bool = True, nesterov: bool = False, metric: str = "l2") -> ivhd_params:
    flags = (FLAG_REORDER if reorder else 0) | (FLAG_NESTEROV if nesterov else 0) | METRICS[metric]
    return ivhd_params(M=M, nn=nn, rn=rn, a=a, b=b, c=c, eps=eps, seed=seed & (2**64 - 1),
                       rn_resample_every=rn_resample_every, mode=MODES[mode], flags=flags,
                       reserved=0)


def ivhd_init(params: ivhd_params, nn_idx: torch.Tensor, y: torch.Tensor, v: torch.Tensor,
              stream: Optional[torch.cuda.Stream] = None) -> ctypes.c_void_p:
    lib = _lib.load()
    M, nn = params.M, params.nn
    p_nn = _dev(nn_idx, torch.int32, (M, nn), "nn_idx")
    p_y = _dev(y, torch.float32, (M, 2), "y")
    p_v = _dev(v, torch.float32, (M, 2), "v")
    h = ctypes.c_void_p()
    check(lib.ivhd_init(ctypes.byref(h), ctypes.byref(params), p_nn, p_y, p_v, _stream_handle(stream)))
    return h


def ivhd_step(ctx, n_iters: int) -> None:
    check(_lib.load().ivhd_step(ctx, int(n_iters)))


def ivhd_stress(ctx, y: Optional[torch.Tensor] = None, M: Optional[int] = None) -> float:
    E = ctypes.c_double()
    p_y = None if y is None else _dev(y, torch.float32, (M if M is not None else y.shape[0], 2), "y")
    check(_lib.load().ivhd_stress(ctx, p_y, ctypes.byref(E)))
    return E.value


def ivhd_grad(ctx, out: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
    M = out.shape[0]
    p_out = _dev(out, torch.float32, (M, 2), "out")
    p_y = None if y is None else _dev(y, torch.float32, (M, 2), "y")
    check(_lib.load().ivhd_grad(ctx, p_y, p_out))
    return out


def ivhd_get_rn(ctx, out: torch.Tensor) -> torch.Tensor:
    p = out.data_ptr() if out.numel() else None
    if out.numel():
        _dev(out, torch.int32, tuple(out.shape), "out")
    check(_lib.load().ivhd_get_rn(ctx, p))
    return out


def ivhd_get_in_edges(ctx, which: int, ptr_out: torch.Tensor, src_out: torch.Tensor):
    _dev(ptr_out, torch.int32, tuple(ptr_out.shape), "ptr_out")
    _dev(src_out, torch.int32, tuple(src_out.shape), "src_out")
    check(_lib.load().ivhd_get_in_edges(ctx, int(which), ptr_out.data_ptr(), src_out.data_ptr()))
    return ptr_out, src_out


def ivhd_get_order(ctx, out: torch.Tensor) -> torch.Tensor:
    _dev(out, torch.int32, tuple(out.shape), "out")
    check(_lib.load().ivhd_get_order(ctx, out.data_ptr()))
    return out


def ivhd_set_state(ctx, y: torch.Tensor, v: torch.Tensor) -> None:
    _dev(y, torch.float32, tuple(y.shape), "y")
    _dev(v, torch.float32, tuple(y.shape), "v")
    check(_lib.load().ivhd_set_state(ctx, y.data_ptr(), v.data_ptr()))


def ivhd_set_iteration(ctx, n: int) -> None:
    check(_lib.load().ivhd_set_iteration(ctx, int(n)))


def ivhd_get_iteration(ctx) -> int:
    n = ctypes.c_int64()
    check(_lib.load().ivhd_get_iteration(ctx, ctypes.byref(n)))
    return n.value


def ivhd_set_graphs(ctx, enable: bool) -> None:
    check(_lib.load().ivhd_set_graphs(ctx, 1 if enable else 0))


def ivhd_destroy(ctx) -> None:
    check(_lib.load().ivhd_destroy(ctx))


def ivhd_set_adaptive(ctx, enable: bool, b: float = 0.0, tau: float = float("inf"), g1: float = 1.05,
                      g2: float = 0.5) -> None:
    check(_lib.load().ivhd_set_adaptive(ctx, 1 if enable else 0, b, tau, g1, g2))


def ivhd_set_adam(ctx, enable: bool, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8) -> None:
    check(_lib.load().ivhd_set_adam(ctx, 1 if enable else 0, lr, beta1, beta2, eps))


def ivhd_get_adaptive(ctx) -> dict:
    b, dT = ctypes.c_float(), ctypes.c_double()
    kept, rej = ctypes.c_int64(), ctypes.c_int64()
    check(_lib.load().ivhd_get_adaptive(ctx, ctypes.byref(b), ctypes.byref(kept), ctypes.byref(rej),
                                        ctypes.byref(dT)))
    return {"b": b.value, "kept": kept.value, "rejected": rej.value, "dT": dT.value}


def ivhd_rnn_mask(nn_idx: torch.Tensor, helper: torch.Tensor, out: Optional[torch.Tensor] = None,
                  stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Reverse-neighbour pruning: int32 [M, nn], edge i -> j kept when i is among helper[j]."""
    M, nn = nn_idx.shape
    kh = helper.shape[1]
    _dev(nn_idx, torch.int32, (M, nn), "nn_idx")
    _dev(helper, torch.int32, (M, kh), "helper")
    if out is None:
        out = torch.empty_like(nn_idx)
    _dev(out, torch.int32, (M, nn), "out")
    check(_lib.load().ivhd_rnn_mask(nn_idx.data_ptr(), M, nn, helper.data_ptr(), kh, out.data_ptr(),
                                    _stream_handle(stream)))
    return out


EDGES_REORDER = 1


def ivhd_edges_create(nn_idx: torch.Tensor, rn_idx: Optional[torch.Tensor] = None,
                      stream: Optional[torch.cuda.Stream] = None, *, reorder: bool = False) -> ctypes.c_void_p:
    M, nn = nn_idx.shape
    p_nn = _dev(nn_idx, torch.int32, (M, nn), "nn_idx")
    rn, p_rn = 0, None
    if rn_idx is not None and rn_idx.numel():
        rn = rn_idx.shape[1]
        p_rn = _dev(rn_idx, torch.int32, (M, rn), "rn_idx")
    h = ctypes.c_void_p()
    check(_lib.load().ivhd_edges_create(ctypes.byref(h), M, p_nn, nn, p_rn, rn,
                                        EDGES_REORDER if reorder else 0, _stream_handle(stream)))
    return h


def ivhd_edges_stress(plan, y: torch.Tensor, c: float, out: torch.Tensor) -> torch.Tensor:
    _dev(out, torch.float64, tuple(out.shape), "out")
    check(_lib.load().ivhd_edges_stress(plan, _dev(y, torch.float32, tuple(y.shape), "y"), float(c),
                                        out.data_ptr()))
    return out


def ivhd_edges_grad(plan, y: torch.Tensor, c: float, eps: float, scale: Optional[torch.Tensor],
                    out: torch.Tensor) -> torch.Tensor:
    p_s = None if scale is None else _dev(scale, torch.float32, tuple(scale.shape), "scale")
    check(_lib.load().ivhd_edges_grad(plan, _dev(y, torch.float32, tuple(y.shape), "y"), float(c),
                                      float(eps), p_s, _dev(out, torch.float32, tuple(y.shape), "out")))
    return out


def ivhd_edges_stress_grad(plan, y: torch.Tensor, c: float, eps: float, scale: Optional[torch.Tensor],
                           E_out: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    p_s = None if scale is None else _dev(scale, torch.float32, tuple(scale.shape), "scale")
    _dev(E_out, torch.float64, tuple(E_out.shape), "E_out")
    check(_lib.load().ivhd_edges_stress_grad(plan, _dev(y, torch.float32, tuple(y.shape), "y"), float(c),
                                             float(eps), p_s, E_out.data_ptr(),
                                             _dev(out, torch.float32, tuple(y.shape), "out")))
    return out


def ivhd_scale_f32(x: torch.Tensor, scale: torch.Tensor, out: torch.Tensor,
                   stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    n = x.numel()
    check(_lib.load().ivhd_scale_f32(_dev(x, torch.float32, tuple(x.shape), "x"), n,
                                     _dev(scale, torch.float32, tuple(scale.shape), "scale"),
                                     _dev(out, torch.float32, tuple(x.shape), "out"), _stream_handle(stream)))
    return out


def ivhd_edges_destroy(plan) -> None:
    check(_lib.load().ivhd_edges_destroy(plan))


def ivhd_grad_edges(y: torch.Tensor, nn_idx: torch.Tensor, rn_idx: Optional[torch.Tensor], c: float,
                    eps: float = 1e-12, out: Optional[torch.Tensor] = None, with_stress: bool = False,
                    stream: Optional[torch.cuda.Stream] = None):
    M, nn = nn_idx.shape
    p_y = _dev(y, torch.float32, (M, 2), "y")
    p_nn = _dev(nn_idx, torch.int32, (M, nn), "nn_idx")
    rn, p_rn = 0, None
    if rn_idx is not None and rn_idx.numel():
        rn = rn_idx.shape[1]
        p_rn = _dev(rn_idx, torch.int32, (M, rn), "rn_idx")
    if out is None:
        out = torch.empty_like(y)
    E = ctypes.c_double()
    check(_lib.load().ivhd_grad_edges(p_y, M, p_nn, nn, p_rn, rn, float(c), float(eps),
                                      _dev(out, torch.float32, (M, 2), "out"),
                                      ctypes.byref(E) if with_stress else None, _stream_handle(stream)))
    return (out, E.value) if with_stress else out


def ivhd_grad_edges_noalloc(y: torch.Tensor, nn_idx: torch.Tensor, rn_idx: Optional[torch.Tensor], c: float,
                            eps: float = 1e-12, out: Optional[torch.Tensor] = None, with_stress: bool = False,
                            stream: Optional[torch.cuda.Stream] = None):
    """ivhd_grad_edges with the library's fixed per-GPU scratch instead of
    temporary allocations (out must be given: this call allocates nothing)."""
    M, nn = nn_idx.shape
    p_y = _dev(y, torch.float32, (M, 2), "y")
    p_nn = _dev(nn_idx, torch.int32, (M, nn), "nn_idx")
    rn, p_rn = 0, None
    if rn_idx is not None and rn_idx.numel():
        rn = rn_idx.shape[1]
        p_rn = _dev(rn_idx, torch.int32, (M, rn), "rn_idx")
    if out is None:
        raise ValueError("out must be given (ivhd_grad_edges_noalloc allocates nothing)")
    E = ctypes.c_double()
    check(_lib.load().ivhd_grad_edges_noalloc(p_y, M, p_nn, nn, p_rn, rn, float(c), float(eps),
                                              _dev(out, torch.float32, (M, 2), "out"),
                                              ctypes.byref(E) if with_stress else None, _stream_handle(stream)))
    return (out, E.value) if with_stress else out


def ivhd_knn_build(x: torch.Tensor, k: int, out: Optional[torch.Tensor] = None,
                   stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Exact kNN graph of the rows of x (float32 [M, N] on the GPU): int32 [M, k]."""
    M, N = x.shape
    _dev(x, torch.float32, (M, N), "x")
    if out is None:
        out = torch.empty((M, k), dtype=torch.int32, device=x.device)
    _dev(out, torch.int32, (M, k), "out")
    check(_lib.load().ivhd_knn_build(x.data_ptr(), M, N, k, out.data_ptr(), _stream_handle(stream)))
    return out


def ivhd_knn_query(x: torch.Tensor, q: torch.Tensor, k: int, self_idx: Optional[torch.Tensor] = None,
                   with_dist: bool = False, stream: Optional[torch.cuda.Stream] = None):
    """k nearest rows of x to each row of q: int32 [Q, k] (and float32 squared distances)."""
    M, N = x.shape
    Q = q.shape[0]
    _dev(x, torch.float32, (M, N), "x")
    _dev(q, torch.float32, (Q, N), "q")
    p_self = None
    if self_idx is not None:
        p_self = _dev(self_idx, torch.int32, (Q,), "self_idx")
    idx = torch.empty((Q, k), dtype=torch.int32, device=x.device)
    dist = torch.empty((Q, k), dtype=torch.float32, device=x.device) if with_dist else None
    check(_lib.load().ivhd_knn_query(x.data_ptr(), M, N, q.data_ptr(), Q, p_self, k, idx.data_ptr(),
                                     dist.data_ptr() if dist is not None else None,
                                     _stream_handle(stream)))
    return (idx, dist) if with_dist else idx


def ivhd_ivf_train(x: torch.Tensor, nlist: int, n_iter: int = 10,
                   stream: Optional[torch.cuda.Stream] = None):
    """k-means coarse quantizer of x (float32 [M, N]): (centroids [nlist, N], assign int32 [M])."""
    M, N = x.shape
    _dev(x, torch.float32, (M, N), "x")
    C = torch.empty((nlist, N), dtype=torch.float32, device=x.device)
    a = torch.empty(M, dtype=torch.int32, device=x.device)
    check(_lib.load().ivhd_ivf_train(x.data_ptr(), M, N, nlist, n_iter, C.data_ptr(), a.data_ptr(),
                                     _stream_handle(stream)))
    return C, a


def ivhd_ivf_search(x: torch.Tensor, centroids: torch.Tensor, assign: torch.Tensor, q: torch.Tensor, k: int,
                    nprobe: int, self_idx: Optional[torch.Tensor] = None, with_dist: bool = False,
                    stream: Optional[torch.cuda.Stream] = None):
    """Approximate k nearest rows of x to each row of q over the nprobe nearest lists."""
    M, N = x.shape
    nlist = centroids.shape[0]
    Q = q.shape[0]
    _dev(x, torch.float32, (M, N), "x")
    _dev(centroids, torch.float32, (nlist, N), "centroids")
    _dev(assign, torch.int32, (M,), "assign")
    _dev(q, torch.float32, (Q, N), "q")
    p_self = _dev(self_idx, torch.int32, (Q,), "self_idx") if self_idx is not None else None
    idx = torch.empty((Q, k), dtype=torch.int32, device=x.device)
    dist = torch.empty((Q, k), dtype=torch.float32, device=x.device) if with_dist else None
    check(_lib.load().ivhd_ivf_search(x.data_ptr(), M, N, centroids.data_ptr(), nlist, assign.data_ptr(),
                                      q.data_ptr(), Q, p_self, k, nprobe, idx.data_ptr(),
                                      dist.data_ptr() if dist is not None else None, _stream_handle(stream)))
    return (idx, dist) if with_dist else idx


def ivf_knn_graph(x: torch.Tensor, k: int, nlist: int, nprobe: int, n_iter: int = 10) -> torch.Tensor:
    """Approximate kNN graph of the rows of x (each row excluded from its own list): int32 [M, k]."""
    C, a = ivhd_ivf_train(x, nlist, n_iter)
    self_idx = torch.arange(x.shape[0], dtype=torch.int32, device=x.device)
    return ivhd_ivf_search(x, C, a, x, k, nprobe, self_idx=self_idx)


def ivhd_last_error() -> str:
    m = _lib.load().ivhd_last_error()
    return m.decode() if m else ""


def ivhd_version() -> int:
    return int(_lib.load().ivhd_version())


class Context:
    """One embedding: a kNN graph, positions and velocities on the GPU.

    ``y`` and ``v`` are advanced in place by ``step``; the context keeps
    references to ``nn_idx``, ``y`` and ``v`` so they outlive it.
    """

    def __init__(self, nn_idx: torch.Tensor, y: torch.Tensor, v: Optional[torch.Tensor] = None, *,
                 rn: int = 1, a: float = 0.9, b: float = 0.01, c: float = 0.1, eps: float = 1e-12,
                 seed: int = 0, rn_resample_every: int = 0, mode: str = "det", reorder: bool = True,
                 nesterov: bool = False, metric: str = "l2",
                 stream: Optional[torch.cuda.Stream] = None):
        M, nn = nn_idx.shape
        if v is None:
            v = torch.zeros_like(y)
        self.params = make_params(M, nn, rn, a=a, b=b, c=c, eps=eps, seed=seed,
                                  rn_resample_every=rn_resample_every, mode=mode, reorder=reorder,
                                  nesterov=nesterov, metric=metric)
        self.nn_idx, self.y, self.v = nn_idx, y, v
        self.M, self.nn, self.rn = M, nn, rn
        self._h = None
        self._h = ivhd_init(self.params, nn_idx, y, v, stream)

    @property
    def handle(self):
        if self._h is None:
            raise IvhdError(-4, "context is closed")
        return self._h

    def step(self, n_iters: int) -> "Context":
        ivhd_step(self.handle, n_iters)
        return self

    def stress(self, y: Optional[torch.Tensor] = None) -> float:
        return ivhd_stress(self.handle, y, self.M)

    def grad(self, y: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.M, 2), dtype=torch.float32, device=self.y.device)
        return ivhd_grad(self.handle, out, y)

    def rn_edges(self) -> torch.Tensor:
        out = torch.empty((self.M, self.rn), dtype=torch.int32, device=self.y.device)
        return ivhd_get_rn(self.handle, out)

    def order(self) -> torch.Tensor:
        """perm [M]: the caller's id of each internal vertex."""
        out = torch.empty(self.M, dtype=torch.int32, device=self.y.device)
        return ivhd_get_order(self.handle, out)

    def set_state(self, y: torch.Tensor, v: torch.Tensor) -> None:
        ivhd_set_state(self.handle, y.contiguous(), v.contiguous())

    def set_iteration(self, n: int) -> None:
        ivhd_set_iteration(self.handle, n)

    def in_edges(self, which: str = "nn"):
        """(ptr [M+1], src) of the transposed nn or rn edge lists (internal order), on the host."""
        k = self.nn if which == "nn" else self.rn
        ptr = torch.empty(self.M + 1, dtype=torch.int32, device=self.y.device)
        src = torch.empty(max(1, self.M * k), dtype=torch.int32, device=self.y.device)
        ivhd_get_in_edges(self.handle, 0 if which == "nn" else 1, ptr, src)
        torch.cuda.synchronize()
        ptr = ptr.cpu().numpy()
        return ptr, src.cpu().numpy()[: ptr[-1]]

    @property
    def iteration(self) -> int:
        return ivhd_get_iteration(self.handle)

    def set_graphs(self, enable: bool) -> None:
        ivhd_set_graphs(self.handle, enable)

    def set_adaptive(self, enable: bool = True, *, b: Optional[float] = None, tau: float = float("inf"),
                     g1: float = 1.05, g2: float = 0.5) -> None:
        """Self-adaptive b (see include/ivhd.h); b defaults to the context's b."""
        ivhd_set_adaptive(self.handle, enable, self.params.b if b is None else b, tau, g1, g2)

    def adaptive(self) -> dict:
        """{"b", "kept", "rejected", "dT"} of the adaptive b."""
        return ivhd_get_adaptive(self.handle)

    def set_adam(self, enable: bool = True, *, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8) -> None:
        """Adam in place of the momentum update (see include/ivhd.h); V holds its first moments."""
        ivhd_set_adam(self.handle, enable, lr, beta1, beta2, eps)

    def close(self) -> None:
        if self._h is not None:
            h, self._h = self._h, None
            ivhd_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- parametric encoder --------------------------------------------------

def ivhd_f32_to_bf16(x: torch.Tensor, out: Optional[torch.Tensor] = None,
                     stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """BF16 (round to nearest even) of an FP32 tensor, as int16 storage of the bits."""
    x = x.contiguous()
    _dev(x, torch.float32, tuple(x.shape), "x")
    if out is None:
        out = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _dev(out, torch.int16, tuple(x.shape), "out")
    check(_lib.load().ivhd_f32_to_bf16(x.data_ptr(), x.numel(), out.data_ptr(), _stream_handle(stream)))
    return out


def ivhd_gemm_bf16(a: torch.Tensor, b: torch.Tensor, M: int, N: int, K: int, *, lda: int, ldb: int,
                   trans_a: bool = False, trans_b: bool = False, epilogue: int = 0,
                   bias: Optional[torch.Tensor] = None, mask: Optional[torch.Tensor] = None,
                   ldm: int = 0, out: Optional[torch.Tensor] = None, ldc: Optional[int] = None,
                   splits: int = 1, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """C = opA @ opB on BF16 bit tensors (int16 storage); see include/ivhd.h."""
    ldc = N if ldc is None else ldc
    if out is None:
        out = torch.empty((M, ldc), dtype=torch.float32 if epilogue == 0 else torch.int16, device=a.device)
    work = None
    if splits > 1:
        work = torch.empty((splits, M, N), dtype=torch.float32, device=a.device)
    check(_lib.load().ivhd_gemm_bf16(a.data_ptr(), b.data_ptr(), M, N, K, lda, ldb, int(trans_a), int(trans_b),
                                     epilogue, None if bias is None else bias.data_ptr(),
                                     None if mask is None else mask.data_ptr(), ldm, out.data_ptr(), ldc,
                                     splits, None if work is None else work.data_ptr(), _stream_handle(stream)))
    return out


def ivhd_enc_create(n_in: int, h1: int, h2: int, seed: int, max_rows: int,
                    stream: Optional[torch.cuda.Stream] = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    check(_lib.load().ivhd_enc_create(ctypes.byref(h), n_in, h1, h2, seed & (2**64 - 1), max_rows,
                                      _stream_handle(stream)))
    return h


def ivhd_enc_num_params(enc) -> int:
    n = ctypes.c_int64()
    check(_lib.load().ivhd_enc_num_params(enc, ctypes.byref(n)))
    return n.value


def ivhd_enc_get_params(enc, params: Optional[torch.Tensor], grads: Optional[torch.Tensor] = None) -> None:
    check(_lib.load().ivhd_enc_get_params(enc, None if params is None else params.data_ptr(),
                                          None if grads is None else grads.data_ptr()))


def ivhd_enc_set_params(enc, params: torch.Tensor) -> None:
    _dev(params, torch.float32, tuple(params.shape), "params")
    check(_lib.load().ivhd_enc_set_params(enc, params.data_ptr()))


def ivhd_enc_embed(enc, x16: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    rows = x16.shape[0]
    _dev(x16, torch.int16, tuple(x16.shape), "x16")
    _dev(out, torch.float32, (rows, 2), "out")
    check(_lib.load().ivhd_enc_embed(enc, x16.data_ptr(), rows, out.data_ptr()))
    return out


def ivhd_enc_train_step(enc, xb16: torch.Tensor, plan, c: float, eps: float, lr: float, loss_scale: float,
                        loss_out: Optional[torch.Tensor] = None) -> None:
    _dev(xb16, torch.int16, tuple(xb16.shape), "xb16")
    check(_lib.load().ivhd_enc_train_step(enc, xb16.data_ptr(), xb16.shape[0], plan, float(c), float(eps),
                                          float(lr), float(loss_scale),
                                          None if loss_out is None else loss_out.data_ptr()))


def ivhd_enc_train_epoch(enc, x16: torch.Tensor, nn_idx: torch.Tensor, rn: int, seed: int, epoch: int,
                         batch: int, c: float, eps: float, lr: float) -> float:
    M, nn = nn_idx.shape
    _dev(x16, torch.int16, tuple(x16.shape), "x16")
    _dev(nn_idx, torch.int32, (M, nn), "nn_idx")
    loss = ctypes.c_double()
    check(_lib.load().ivhd_enc_train_epoch(enc, x16.data_ptr(), M, nn_idx.data_ptr(), nn, rn,
                                           seed & (2**64 - 1), epoch, batch, float(c), float(eps), float(lr),
                                           ctypes.byref(loss)))
    return loss.value


def ivhd_enc_destroy(enc) -> None:
    check(_lib.load().ivhd_enc_destroy(enc))


__all__ += ["ivhd_f32_to_bf16", "ivhd_gemm_bf16", "ivhd_enc_create", "ivhd_enc_num_params",
            "ivhd_enc_get_params", "ivhd_enc_set_params", "ivhd_enc_embed", "ivhd_enc_train_step",
            "ivhd_enc_train_epoch", "ivhd_enc_destroy"]


def ivhd_eval_neighbours(z: torch.Tensor, rows: torch.Tensor, k: int, out: Optional[torch.Tensor] = None,
                         stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Neighbourhoods of size k (positions 1..k of the FP64 (distance, index)
    order) of the sample rows of z (float32 [M, N]): int32 [Q, k]."""
    M, N = z.shape
    _dev(z, torch.float32, (M, N), "z")
    Q = rows.shape[0]
    _dev(rows, torch.int32, (Q,), "rows")
    if out is None:
        out = torch.empty((Q, k), dtype=torch.int32, device=z.device)
    _dev(out, torch.int32, (Q, k), "out")
    check(_lib.load().ivhd_eval_neighbours(z.data_ptr(), M, N, rows.data_ptr(), Q, k, out.data_ptr(),
                                           _stream_handle(stream)))
    return out


def ivhd_eval_ranks(z: torch.Tensor, rows: torch.Tensor, cand: torch.Tensor, out: Optional[torch.Tensor] = None,
                    stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Ranks rho_rj of the given points cand (int32 [Q, kc]) around the
    sample rows of z: int32 [Q, kc]."""
    M, N = z.shape
    _dev(z, torch.float32, (M, N), "z")
    Q, kc = cand.shape
    _dev(rows, torch.int32, (Q,), "rows")
    _dev(cand, torch.int32, (Q, kc), "cand")
    if out is None:
        out = torch.empty((Q, kc), dtype=torch.int32, device=z.device)
    _dev(out, torch.int32, (Q, kc), "out")
    check(_lib.load().ivhd_eval_ranks(z.data_ptr(), M, N, rows.data_ptr(), Q, cand.data_ptr(), kc, out.data_ptr(),
                                      _stream_handle(stream)))
    return out


def ivhd_eval_scores(M: int, rows: torch.Tensor, nx: Optional[torch.Tensor], ny: torch.Tensor, k: int,
                     rank_y: Optional[torch.Tensor] = None, labels: Optional[torch.Tensor] = None,
                     stream: Optional[torch.cuda.Stream] = None):
    """(Q_NX(k), cf_k, T(k)) over the sample; NaN where an input is None."""
    Q, ky = ny.shape
    _dev(rows, torch.int32, (Q,), "rows")
    _dev(ny, torch.int32, (Q, ky), "ny")
    kx, p_nx = 0, None
    if nx is not None:
        kx = nx.shape[1]
        p_nx = _dev(nx, torch.int32, (Q, kx), "nx")
    p_rank = _dev(rank_y, torch.int32, (Q, ky), "rank_y") if rank_y is not None else None
    p_lab = _dev(labels, torch.int32, (M,), "labels") if labels is not None else None
    h = (ctypes.c_double * 3)()
    check(_lib.load().ivhd_eval_scores(M, rows.data_ptr(), Q, p_nx, kx, ny.data_ptr(), ky, p_rank, p_lab, k,
                                       ctypes.cast(h, ctypes.c_void_p), _stream_handle(stream)))
    return h[0], h[1], h[2]


def ivhd_probe_gather(src: torch.Tensor, idx: torch.Tensor, out: Optional[torch.Tensor] = None,
                      stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """out[t] = src[idx[t]] for float32 [n_src, 2] rows (a random-gather rate probe)."""
    n_src = src.shape[0]
    _dev(src, torch.float32, (n_src, 2), "src")
    n = idx.shape[0]
    _dev(idx, torch.int32, (n,), "idx")
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float32, device=src.device)
    _dev(out, torch.float32, (n, 2), "out")
    check(_lib.load().ivhd_probe_gather(src.data_ptr(), n_src, idx.data_ptr(), n, out.data_ptr(),
                                        _stream_handle(stream)))
    return out


def ivhd_probe_atomic(acc: torch.Tensor, idx: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """acc[idx[t]] += 2**32 + 1 with one 64-bit integer atomic per index, on an
    int64 [n_acc] tensor (a random-atomic rate probe)."""
    n_acc = acc.shape[0]
    _dev(acc, torch.int64, (n_acc,), "acc")
    n = idx.shape[0]
    _dev(idx, torch.int32, (n,), "idx")
    check(_lib.load().ivhd_probe_atomic(acc.data_ptr(), n_acc, idx.data_ptr(), n, _stream_handle(stream)))
    return acc
