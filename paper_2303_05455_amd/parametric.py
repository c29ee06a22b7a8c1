"""Parametric IVHD: a learned N-D -> 2-D map trained on the IVHD stress.

The network (MLP n_in -> 512 -> 512 -> 2, ReLU, BF16 on the matrix cores)
is trained by libivhd's own forward, backward and Adam kernels on batches of
IVHD edges: each batch holds `batch` source vertices, their nn neighbours
from the kNN graph and their random neighbours of the epoch, and the loss is
the binary-distance stress of those edges.  New points are then placed by
one forward pass (``embed``); plain IVHD (``Context``) serves as fallback and
as the reference layout its kNN preservation is compared with.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import api


class ParametricIVHD:
    def __init__(self, n_in: int, hidden=(512, 512), *, seed: int = 0, batch: int = 8192, nn: int = 5,
                 rn: int = 1, c: float = 0.1, eps: float = 1e-12, lr: float = 1e-3,
                 max_rows: Optional[int] = None):
        self.n_in, self.h1, self.h2 = n_in, hidden[0], hidden[1]
        self.batch, self.nn, self.rn = batch, nn, rn
        self.c, self.eps, self.lr, self.seed = c, eps, lr, seed
        self.max_rows = max_rows or batch * (1 + nn + rn)
        self._h = None
        self._h = api.ivhd_enc_create(n_in, self.h1, self.h2, seed, self.max_rows)
        self.epochs_done = 0
        self.losses = []

    @property
    def handle(self):
        if self._h is None:
            raise api.IvhdError(-4, "encoder is closed")
        return self._h

    @staticmethod
    def to_bf16(x: torch.Tensor) -> torch.Tensor:
        return api.ivhd_f32_to_bf16(x.contiguous())

    def fit(self, x16: torch.Tensor, nn_idx: torch.Tensor, epochs: int) -> "ParametricIVHD":
        """x16: BF16 bits (int16) [M, n_in] on the GPU; nn_idx int32 [M, nn]."""
        for _ in range(epochs):
            loss = api.ivhd_enc_train_epoch(self.handle, x16, nn_idx, self.rn, self.seed, self.epochs_done,
                                            self.batch, self.c, self.eps, self.lr)
            self.losses.append(loss)
            self.epochs_done += 1
        return self

    def embed(self, x16: torch.Tensor, out: Optional[torch.Tensor] = None, *, refine_iters: int = 0,
              x: Optional[torch.Tensor] = None, nn_idx: Optional[torch.Tensor] = None, a: float = 0.9,
              b: Optional[float] = None, rn_resample_every: int = 100, seed: int = 0,
              mode: str = "det") -> torch.Tensor:
        """Place the rows of x16 (BF16 bits [rows, n_in]) with one forward
        pass; with ``refine_iters`` > 0 the placement then starts plain IVHD
        (the fallback: the loop of ``Context`` initialised from the network's
        layout, as the thesis starts IVHD from another method's layout) on the
        kNN graph of these rows -- ``nn_idx`` (int32 [rows, nn]) or, when it
        is None, the exact graph of ``x`` (float32 [rows, n_in]) -- with this
        encoder's nn, rn and c.  b defaults to a quarter of the heavy-ball
        stability bound 2 (1 + a) / (max in-degree + nn + 2 rn + 2)."""
        if out is None:
            out = torch.empty((x16.shape[0], 2), dtype=torch.float32, device=x16.device)
        api.ivhd_enc_embed(self.handle, x16, out)
        if refine_iters > 0:
            if nn_idx is None:
                if x is None:
                    raise ValueError("refine_iters needs nn_idx or the float32 rows x")
                nn_idx = api.ivhd_knn_build(x.contiguous(), self.nn)
            if b is None:
                indeg = torch.bincount(nn_idx.reshape(-1).long().clamp(min=0), minlength=nn_idx.shape[0])
                b = 0.25 * 2 * (1 + a) / (int(indeg.max()) + nn_idx.shape[1] + 2 * self.rn + 2)
            ctx = api.Context(nn_idx, out, rn=self.rn, a=a, b=b, c=self.c, eps=self.eps, seed=seed,
                              rn_resample_every=rn_resample_every, mode=mode)
            ctx.step(refine_iters)
            ctx.close()
        return out

    def params(self) -> torch.Tensor:
        n = api.ivhd_enc_num_params(self.handle)
        p = torch.empty(n, dtype=torch.float32, device="cuda")
        api.ivhd_enc_get_params(self.handle, p)
        return p

    def grads(self) -> torch.Tensor:
        n = api.ivhd_enc_num_params(self.handle)
        g = torch.empty(n, dtype=torch.float32, device="cuda")
        api.ivhd_enc_get_params(self.handle, None, g)
        return g

    def set_params(self, p: torch.Tensor) -> None:
        api.ivhd_enc_set_params(self.handle, p.contiguous())

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            api.ivhd_enc_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
