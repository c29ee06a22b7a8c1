"""The IVHD stress as a differentiable loss.

E(Y) = sum_i [ sum_{j in O_nn(i)} |y_i - y_j|^2 + c sum_{k in O_rn(i)} (1 - |y_i - y_k|)^2 ]
(Eq. ivhd_cost_function).  Forward: FP64 accumulation on the GPU, returned as
an FP32 scalar loss (the FP64 value stays available as ``.last_stress``).
Gradient: the hand-written gather kernel of libivhd, taken together with the
stress in the forward when the layout requires a gradient, and scaled on the
device by the upstream gradient in the backward (no host synchronisation).
"""
from __future__ import annotations

from typing import Optional

import torch

from . import api


class StressEdges:
    """An edge plan: transposed lists of fixed nn / rn edge lists, reused by
    every forward and backward call.  Keeps the index tensors alive.

    The plan's kernels run on the stream that was current when it was made;
    a call from another stream is ordered after that stream's queued work and
    the caller's stream waits for the result, and the tensors it touches are
    marked as used on the plan's stream (so the caching allocator does not
    hand their memory out early).

    reorder=True (the default) lets the plan work in the vertex order of the
    loop's contexts (components, then in-degree): each call gathers Y into
    that order first, and the edge gathers then stay within a component's
    stretch of positions.  Inputs and outputs stay in the caller's order; the
    results equal the unordered plan's up to floating-point summation order."""

    def __init__(self, nn_idx: torch.Tensor, rn_idx: Optional[torch.Tensor] = None, *,
                 c: float = 0.1, eps: float = 1e-12, reorder: bool = True):
        self.nn_idx = nn_idx.contiguous()
        self.rn_idx = None if rn_idx is None else rn_idx.contiguous()
        self.M = nn_idx.shape[0]
        self.c, self.eps = float(c), float(eps)
        self._h = None
        self.stream = torch.cuda.current_stream(nn_idx.device)
        self._h = api.ivhd_edges_create(self.nn_idx, self.rn_idx, stream=self.stream, reorder=reorder)
        self._E = torch.zeros((), dtype=torch.float64, device=nn_idx.device)

    def _run(self, fn, *tensors):
        cur = torch.cuda.current_stream(self.nn_idx.device)
        if cur == self.stream:
            return fn()
        self.stream.wait_stream(cur)
        r = fn()
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)
        cur.wait_stream(self.stream)
        return r

    @property
    def handle(self):
        if self._h is None:
            raise api.IvhdError(-4, "edge plan is closed")
        return self._h

    def stress64(self, y: torch.Tensor) -> torch.Tensor:
        """E(y) as a float64 device scalar (asynchronous)."""
        out = torch.empty((), dtype=torch.float64, device=y.device)
        y = y.contiguous()
        return self._run(lambda: api.ivhd_edges_stress(self.handle, y, self.c, out), y, out)

    def grad(self, y: torch.Tensor, scale: Optional[torch.Tensor] = None,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
        y = y.contiguous()
        if out is None:
            out = torch.empty_like(y)
        return self._run(lambda: api.ivhd_edges_grad(self.handle, y, self.c, self.eps, scale, out), y, scale, out)

    def stress_grad(self, y: torch.Tensor, scale: Optional[torch.Tensor] = None,
                    out: Optional[torch.Tensor] = None):
        """(E(y) as a float64 device scalar, scale * grad E(y)) from one pass
        over the edges (asynchronous)."""
        y = y.contiguous()
        E = torch.empty((), dtype=torch.float64, device=y.device)
        if out is None:
            out = torch.empty_like(y)
        self._run(lambda: api.ivhd_edges_stress_grad(self.handle, y, self.c, self.eps, scale, E, out),
                  y, scale, E, out)
        return E, out

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            api.ivhd_edges_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IVHDStress(torch.autograd.Function):
    """loss = IVHDStress.apply(y, edges): y float32 [M, 2] on the GPU.

    When y requires a gradient, the forward takes the stress and its
    gradient in one pass over the edges (``StressEdges.stress_grad``) and
    keeps the gradient; the backward only scales it by the upstream
    gradient.  Otherwise the forward takes the stress alone."""

    @staticmethod
    def forward(ctx, y: torch.Tensor, edges: StressEdges):
        if y.dtype != torch.float32 or y.dim() != 2 or y.shape[1] != 2:
            raise TypeError("y must be float32 [M, 2]")
        y = y.contiguous()
        if ctx.needs_input_grad[0]:
            E64, g = edges.stress_grad(y)
            ctx.save_for_backward(g)
        else:
            E64 = edges.stress64(y)
        edges.last_stress = E64
        ctx.edges = edges
        return E64.to(torch.float32)

    @staticmethod
    def backward(ctx, g_out: torch.Tensor):
        (g,) = ctx.saved_tensors
        edges = ctx.edges
        scale = g_out.detach().to(torch.float32).reshape(1).contiguous()
        out = torch.empty_like(g)
        edges._run(lambda: api.ivhd_scale_f32(g, scale, out, stream=edges.stream), g, scale, out)
        return out, None


def ivhd_stress_loss(y: torch.Tensor, edges: StressEdges) -> torch.Tensor:
    return IVHDStress.apply(y, edges)
