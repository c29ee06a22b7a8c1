"""Quality of a layout on a sample of points, on the GPU (the criteria of the
thesis's chapter "Quality metrics").

    from paper_2303_05455_amd.evaluate import quality
    q = quality(x, y, rows, labels=labels)   # x [M, N], y [M, 2] float32 on the GPU
    q["q_nx"][10], q["cf"][100], q["trust"][10]

Every number comes from the library's evaluation kernels (ivhd_eval_*): the
neighbourhoods and ranks around each sample row are taken in the FP64
(distance, index) order of Sec. "Rank-based criteria"; this module only
chains the calls.  Off the timed path of the loop.
"""
from __future__ import annotations

from typing import Iterable, Optional

import numpy as np
import torch

from .api import ivhd_eval_neighbours, ivhd_eval_ranks, ivhd_eval_scores


def sample_rows(M: int, n: int, seed: int = 0) -> np.ndarray:
    """n distinct rows of range(M) (all of them when n >= M), sorted."""
    if n >= M:
        return np.arange(M, dtype=np.int32)
    return np.sort(np.random.default_rng(seed).choice(M, n, replace=False)).astype(np.int32)


def data_neighbours(x: torch.Tensor, rows, k: int) -> torch.Tensor:
    """The data-space neighbourhoods of size k of the sample rows (int32
    [Q, k] on the GPU), to be shared by the evaluations of several layouts."""
    rows_t = torch.as_tensor(np.asarray(rows, dtype=np.int32), device=x.device)
    return ivhd_eval_neighbours(x.contiguous(), rows_t, k)


def quality(x: torch.Tensor, y: torch.Tensor, rows, labels=None, ks: Iterable[int] = (2, 10, 100),
            k_qnx: Iterable[int] = (10,), k_trust: Iterable[int] = (10,),
            nx: Optional[torch.Tensor] = None) -> dict:
    """Q_NX(k) for k in k_qnx, cf_k for k in ks (with labels), T(k) for k in
    k_trust, over the sample ``rows`` (every row: the whole layout).

    x: float32 [M, N] data, y: float32 [M, 2] layout, both on the GPU;
    rows: int array of sample rows; labels: int array [M] or None; nx: the
    data neighbourhoods of the rows from ``data_neighbours`` (at least as
    many columns as the largest k of k_qnx and k_trust), when already known.
    """
    M = x.shape[0]
    dev = x.device
    rows_t = torch.as_tensor(np.asarray(rows, dtype=np.int32), device=dev)
    ks, k_qnx, k_trust = tuple(ks), tuple(k_qnx), tuple(k_trust)
    lab_t = None if labels is None else torch.as_tensor(np.asarray(labels, dtype=np.int32), device=dev)
    kx = max(k_qnx + k_trust)
    ky = max(ks + k_qnx + k_trust) if lab_t is not None else max(k_qnx + k_trust)
    if nx is None or nx.shape[1] < kx:
        nx = ivhd_eval_neighbours(x.contiguous(), rows_t, kx)
    ny = ivhd_eval_neighbours(y.contiguous(), rows_t, ky)
    out = {"rows": int(rows_t.numel()), "M": M, "q_nx": {}, "cf": {}, "trust": {}}
    for k in k_qnx:
        out["q_nx"][k] = ivhd_eval_scores(M, rows_t, nx.contiguous(), ny, k)[0]
    if lab_t is not None:
        for k in ks:
            out["cf"][k] = ivhd_eval_scores(M, rows_t, None, ny, k, labels=lab_t)[1]
    for k in k_trust:
        cand = ny[:, :k].contiguous()
        rank = ivhd_eval_ranks(x.contiguous(), rows_t, cand)
        out["trust"][k] = ivhd_eval_scores(M, rows_t, nx[:, :k].contiguous(), cand, k, rank_y=rank)[2]
    out["nx"] = nx
    out["q_nx_random"] = {k: k / (M - 1) for k in k_qnx}
    return out
