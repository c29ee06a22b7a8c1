"""Pins of the FP64 encoder reference: torch autograd (FP64, CPU), central
finite differences, torch's BF16 conversion and torch.optim.Adam."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp


def _params(n_in, h1, h2, seed):
    rng = np.random.default_rng(seed)
    L = mlp.layout(n_in, h1, h2)
    return rng.normal(0, 0.3, L["n"])


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.normal(0, 1e-3, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -2.5, 1e-40]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)
    np.testing.assert_array_equal(mlp.from_bf16_bits(mlp.bf16_bits(x)), ref)


def _torch_net(p, X, n_in, h1, h2):
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a, dtype=torch.float64, requires_grad=True)
                              for a in mlp.unpack(p, n_in, h1, h2)]
    Xt = torch.tensor(X, dtype=torch.float64)
    Z = torch.relu(torch.relu(Xt @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    return Z, [W1, b1, W2, b2, W3, b3]


def test_backward_matches_torch_autograd_without_rounding():
    n_in, h1, h2 = 9, 8, 16
    p = _params(n_in, h1, h2, 1)
    X = np.random.default_rng(2).normal(size=(30, n_in))
    dZ = np.random.default_rng(3).normal(size=(30, 2))
    Z, cache = mlp.forward(p, X, n_in, h1, h2, bf16=False)
    g = mlp.backward(cache, dZ, bf16=False)
    Zt, ws = _torch_net(p, X, n_in, h1, h2)
    np.testing.assert_allclose(Z, Zt.detach().numpy(), rtol=1e-12, atol=1e-12)
    (Zt * torch.tensor(dZ)).sum().backward()
    np.testing.assert_allclose(g, mlp.pack(*[w.grad.numpy() for w in ws]), rtol=1e-10, atol=1e-12)


def test_stress_gradient_of_the_network_matches_finite_differences():
    n_in, h1, h2, B, nn, rn = 6, 8, 8, 5, 2, 1
    p = _params(n_in, h1, h2, 4)
    R = B * (1 + nn + rn)
    X = np.random.default_rng(5).normal(size=(R, n_in))
    lnn, lrn = mlp.batch_edges(B, nn, rn)

    def loss(q):
        Z, _ = mlp.forward(q, X, n_in, h1, h2, bf16=False)
        return oracle.stress(Z, lnn, lrn, 0.1)
    Z, cache = mlp.forward(p, X, n_in, h1, h2, bf16=False)
    g = mlp.backward(cache, oracle.grad(Z, lnn, lrn, 0.1), bf16=False)
    h = 1e-6
    for i in np.random.default_rng(6).choice(p.size, 40, replace=False):
        e = np.zeros_like(p); e[i] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-7)


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    w0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(3)]
    wt = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        wt.grad = torch.tensor(g)
        opt.step()
        w, m, v = mlp.adam(w, g, m, v, t, 1e-2)
    np.testing.assert_allclose(w, wt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_batch_edges_layout():
    lnn, lrn = mlp.batch_edges(3, 2, 1)
    assert lnn.shape == (12, 2) and lrn.shape == (12, 1)
    assert lnn[1].tolist() == [5, 6] and lrn[2].tolist() == [11]
    assert np.all(lnn[3:] == -1) and np.all(lrn[3:] == -1)
