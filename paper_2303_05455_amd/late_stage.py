"""The late stages of the thesis's improvements chapter as one call.

    from paper_2303_05455_amd.late_stage import staged_run
    info = staged_run(nn_idx, y, v, T=2000, x=x, a=0.9, b=0.002, c=0.01, rn_resample_every=100)

T iterations of the loop in three stages (Sec. "Reverse neighbors
mechanism", Sec. "L1 norm in late stages of embedding"; when they start is
the reading the figure captions give):
  1. plain IVHD for the first T - mask_iters iterations;
  2. the nn edges pruned by the reverse-neighbour mask (an edge i -> j is
     kept when i is among the kh = 4 nn nearest neighbours of j) for the next
     mask_iters - l1_iters iterations;
  3. the same pruned edges with the l1 distance for the last l1_iters, at
     half the step factor b (the l1 iteration is up to twice as stiff).
Each stage is a Context started where the previous one stopped (positions,
velocities and the iteration counter, so the random-neighbour schedule runs
on unbroken).  The helper graph comes from the exact kNN builder unless one
is given.  Every step runs in libivhd's kernels; this module only sequences
the calls.
"""
from __future__ import annotations

from typing import Optional

import torch

from .api import Context, ivhd_knn_build, ivhd_rnn_mask


def staged_run(nn_idx: torch.Tensor, y: torch.Tensor, v: torch.Tensor, *, T: int, x: Optional[torch.Tensor] = None,
               helper: Optional[torch.Tensor] = None, mask_iters: int = 200, l1_iters: int = 50,
               kh_factor: int = 4, rn: int = 1, a: float = 0.9, b: float = 0.01, c: float = 0.1,
               eps: float = 1e-12, seed: int = 0, rn_resample_every: int = 0, mode: str = "det") -> dict:
    """Advance y, v (float32 [M, 2], in place) by T iterations; returns the
    share of nn edges the mask kept and the pruned lists."""
    if not (0 <= l1_iters <= mask_iters <= T):
        raise ValueError("need 0 <= l1_iters <= mask_iters <= T")
    kw = dict(rn=rn, a=a, c=c, eps=eps, seed=seed, rn_resample_every=rn_resample_every, mode=mode)
    n1 = T - mask_iters
    ctx = Context(nn_idx, y, v, b=b, **kw)
    ctx.step(n1)
    ctx.close()
    if mask_iters == 0:
        return {"kept": 1.0, "nn_masked": nn_idx}
    if helper is None:
        if x is None:
            raise ValueError("the mask needs the helper graph or the data x")
        helper = ivhd_knn_build(x.contiguous(), kh_factor * nn_idx.shape[1])
    masked = ivhd_rnn_mask(nn_idx, helper)
    kept = float((masked >= 0).float().mean())
    n2 = mask_iters - l1_iters
    if n2 > 0:
        ctx = Context(masked, y, v, b=b, **kw)
        ctx.set_iteration(n1)
        ctx.step(n2)
        ctx.close()
    if l1_iters > 0:
        ctx = Context(masked, y, v, b=b / 2, metric="l1", **kw)
        ctx.set_iteration(T - l1_iters)
        ctx.step(l1_iters)
        ctx.close()
    return {"kept": kept, "nn_masked": masked}
