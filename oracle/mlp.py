"""FP64 reference of the parametric encoder (MLP n_in -> h1 -> h2 -> 2, ReLU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy in FP64.
With ``bf16=True`` the values the GPU stores in BF16 are rounded to BF16
(round to nearest even) at the same points: the weights W1, W2, W3 used in
the products, the input rows, the hidden activations after ReLU, and the
back-propagated hidden gradients after the ReLU mask.  Z and every
accumulation stay wide.

The training loss is the IVHD stress of the batch's local edge lists (the
oracle's own ``stress``/``grad``), optimised by Adam with the textbook bias
correction 1/(1 - beta^t).

Pins (tests/test_oracle_mlp.py): the gradient equals torch.autograd's and
central finite differences (bf16=False), the rounding equals torch's
float32 -> bfloat16 conversion, and one Adam step equals torch.optim.Adam.
"""
from __future__ import annotations

import numpy as np

from . import grad as stress_grad
from . import stress as stress_value


def bf16_round(x) -> np.ndarray:
    """Round to BF16 (nearest even) through FP32; returns float64 values."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    out = (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def bf16_bits(x) -> np.ndarray:
    """The BF16 bit patterns (int16 storage) of bf16_round(x)."""
    f = bf16_round(x).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def layout(n_in: int, h1: int, h2: int):
    """Offsets of W1 [h1][n_in], b1, W2 [h2][h1], b2, W3 [2][h2], b3 in the flat vector."""
    o = {}
    k = 0
    for name, size in (("W1", h1 * n_in), ("b1", h1), ("W2", h2 * h1), ("b2", h2), ("W3", 2 * h2), ("b3", 2)):
        o[name] = (k, size)
        k += size
    o["n"] = k
    return o


def unpack(p, n_in, h1, h2):
    L = layout(n_in, h1, h2)
    g = lambda k: np.asarray(p[L[k][0]:L[k][0] + L[k][1]], dtype=np.float64)
    return (g("W1").reshape(h1, n_in), g("b1"), g("W2").reshape(h2, h1), g("b2"),
            g("W3").reshape(2, h2), g("b3"))


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def forward(p, X, n_in, h1, h2, bf16: bool = True):
    """Returns (Z, cache) with Z = W3 relu(W2 relu(W1 x + b1) + b2) + b3 per row."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, h1, h2)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    X = r(X)
    W1r, W2r, W3r = r(W1), r(W2), r(W3)
    A1 = r(np.maximum(X @ W1r.T + b1, 0.0))
    A2 = r(np.maximum(A1 @ W2r.T + b2, 0.0))
    Z = A2 @ W3r.T + b3
    return Z, (X, A1, A2, W2r, W3r)


def backward(cache, dZ, bf16: bool = True):
    """Gradient of sum(dZ * Z) with respect to the flat parameters."""
    X, A1, A2, W2r, W3r = cache
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    dZ = np.asarray(dZ, dtype=np.float64)
    dA2 = r((dZ @ W3r) * (A2 > 0))
    dW3 = dZ.T @ A2
    db3 = dZ.sum(0)
    dA1 = r((dA2 @ W2r) * (A1 > 0))
    dW2 = dA2.T @ A1
    db2 = dA2.sum(0)
    dW1 = dA1.T @ X
    db1 = dA1.sum(0)
    return pack(dW1, db1, dW2, db2, dW3, db3)


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def batch_edges(B: int, nn: int, rn: int):
    """Local edge lists of a batch of B sources followed by their nn and rn
    targets: source b's nn edges point at rows B + b*nn + q, its rn edges at
    rows B + B*nn + b*rn + q; the other rows have none (-1)."""
    R = B * (1 + nn + rn)
    lnn = -np.ones((R, nn), np.int32)
    lrn = -np.ones((R, rn), np.int32)
    b = np.arange(B)
    for q in range(nn):
        lnn[:B, q] = B + b * nn + q
    for q in range(rn):
        lrn[:B, q] = B + B * nn + b * rn + q
    return lnn, lrn


def train_step(p, m, v, t, X, lnn, lrn, n_in, h1, h2, *, c, eps, lr, scale, bf16=True):
    """One Adam step on the batch stress.  Returns (p, m, v, grad, E)."""
    Z, cache = forward(p, X, n_in, h1, h2, bf16)
    E = stress_value(Z, lnn, lrn, c)
    dZ = stress_grad(Z, lnn, lrn, c, eps)
    g = backward(cache, dZ, bf16)
    p2, m2, v2 = adam(np.asarray(p, np.float64), g * scale, m, v, t, lr)
    return p2, m2, v2, g, E
