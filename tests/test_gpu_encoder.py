"""The BF16 MFMA encoder kernels against the FP64 reference.

GEMMs: on identical BF16 operands, |gpu - ref| <= 1e-5 * sum_k |a_k b_k| per
element (FP32 accumulation) for FP32 outputs, plus one BF16 rounding step
(2^-8 relative) for BF16 outputs.  A training step: gradients and updated
parameters against oracle/mlp.py with BF16 rounding emulated at the same
points, norm-wise within 1e-3.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05455_amd as m
    from paper_2303_05455_amd import api, autograd, parametric
    return m, api, autograd, parametric


def _bits(x):
    return torch.from_numpy(mlp.bf16_bits(x).copy()).cuda()


def _norm_rel(x, ref):
    return float(np.linalg.norm(np.asarray(x, np.float64) - ref) / max(np.linalg.norm(ref), 1e-300))


@pytest.mark.parametrize("M,N,K,ta,tb,epi,splits", [
    (257, 130, 100, 0, 1, 0, 1), (128, 128, 32, 0, 0, 0, 1), (300, 77, 513, 1, 0, 0, 4),
    (64, 200, 1000, 1, 1, 0, 3), (1000, 512, 784, 0, 1, 1, 1), (999, 512, 512, 0, 0, 2, 1),
    (512, 784, 4096, 1, 0, 0, 16), (5, 3, 7, 0, 1, 0, 1),
    # K-contiguous operands with K % 8 == 0 (the double-buffered path): ragged
    # M and N, a K tail inside the last step, split-K, every epilogue, K = 8,
    # more column tiles than row tiles
    (300, 200, 840, 0, 1, 0, 5), (999, 136, 512, 0, 1, 2, 1), (64, 8, 8, 0, 1, 0, 1),
    (130, 640, 4160, 0, 1, 0, 16), (200, 1000, 72, 0, 1, 1, 1), (136, 4104, 512, 0, 1, 2, 1),
    # tall products like the training step's: ragged rows and columns, a K
    # tail inside the last step, every epilogue, split-K
    (33001, 520, 792, 0, 1, 0, 1), (33001, 520, 792, 0, 1, 1, 1), (33001, 520, 792, 0, 1, 2, 1),
    (4096, 512, 4096, 0, 1, 0, 8), (65536, 512, 784, 0, 1, 1, 1),
    # K-contiguous operands with an output width that is not a multiple of 8
    # (element-wise output and mask chunks), every epilogue, split-K
    (300, 77, 512, 0, 1, 1, 1), (300, 77, 512, 0, 1, 2, 1), (300, 77, 520, 0, 1, 0, 3),
    # both operands K-major with widths that are multiples of 8 (the K-major
    # kernel the weight gradients use): ragged M and N tiles, K tails inside
    # a step and inside a split, split-K like the training step's, a tiny case
    (256, 136, 1000, 1, 0, 0, 3), (264, 512, 33001, 1, 0, 0, 32), (520, 784, 20000, 1, 0, 0, 32),
    (8, 16, 40, 1, 0, 0, 1), (512, 512, 4104, 1, 0, 0, 1),
])
def test_gemm_matches_fp64_on_identical_bf16_operands(pkg, M, N, K, ta, tb, epi, splits):
    m, api, _, _ = pkg
    rng = np.random.default_rng(M * 7 + N + K)
    A = mlp.bf16_round(rng.normal(size=(K, M) if ta else (M, K)))
    B = mlp.bf16_round(rng.normal(size=(N, K) if tb else (K, N)))
    opA = A.T if ta else A
    opB = B.T if tb else B
    ref = opA @ opB
    bound = np.abs(opA) @ np.abs(opB)
    bias = rng.normal(size=N).astype(np.float32)
    mask = mlp.bf16_round(rng.normal(size=(M, N)))
    out = api.ivhd_gemm_bf16(_bits(A), _bits(B), M, N, K, lda=A.shape[1], ldb=B.shape[1], trans_a=bool(ta),
                             trans_b=bool(tb), epilogue=epi,
                             bias=torch.from_numpy(bias).cuda() if epi == 1 else None,
                             mask=_bits(mask) if epi == 2 else None, ldm=N, splits=splits)
    torch.cuda.synchronize()
    if epi == 0:
        got = out.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - ref) <= 1e-5 * bound + 1e-30)
    else:
        got = mlp.from_bf16_bits(out.cpu().numpy())
        want = np.maximum(ref + bias, 0) if epi == 1 else np.where(mask > 0, ref, 0.0)
        tol = 1e-5 * (bound + np.abs(bias) if epi == 1 else bound) + 2.0 ** -8 * np.abs(want) + 1e-30
        assert np.all(np.abs(got - want) <= tol)


@pytest.mark.parametrize("epi", [0, 1, 2])
def test_gemm_on_operands_not_16_byte_aligned(pkg, epi):
    # K-contiguous operands whose base sits 2 bytes past a 16-byte boundary:
    # the element-wise staging must give the same bound as the vector path
    m, api, _, _ = pkg
    M, N, K = 200, 72, 96
    rng = np.random.default_rng(epi + 40)
    A = mlp.bf16_round(rng.normal(size=(M, K)))
    B = mlp.bf16_round(rng.normal(size=(N, K)))
    ref = A @ B.T
    bound = np.abs(A) @ np.abs(B.T)
    bias = rng.normal(size=N).astype(np.float32)
    mask = mlp.bf16_round(rng.normal(size=(M, N)))
    a_buf = _bits(np.concatenate([[0.0], A.ravel()]))   # element 1 onwards: 2 bytes past the base
    b_buf = _bits(np.concatenate([[0.0], B.ravel()]))
    out = api.ivhd_gemm_bf16(a_buf[1:], b_buf[1:], M, N, K, lda=K, ldb=K, trans_a=False, trans_b=True,
                             epilogue=epi, bias=torch.from_numpy(bias).cuda() if epi == 1 else None,
                             mask=_bits(mask) if epi == 2 else None, ldm=N)
    torch.cuda.synchronize()
    if epi == 0:
        assert np.all(np.abs(out.cpu().numpy().astype(np.float64) - ref) <= 1e-5 * bound + 1e-30)
    else:
        got = mlp.from_bf16_bits(out.cpu().numpy())
        want = np.maximum(ref + bias, 0) if epi == 1 else np.where(mask > 0, ref, 0.0)
        tol = 1e-5 * (bound + np.abs(bias) if epi == 1 else bound) + 2.0 ** -8 * np.abs(want) + 1e-30
        assert np.all(np.abs(got - want) <= tol)


def _setup(pkg, n_in, h1, h2, B, nn, rn, seed):
    m, api, ag, par = pkg
    rng = np.random.default_rng(seed)
    R = B * (1 + nn + rn)
    X = mlp.bf16_round(np.maximum(rng.normal(1.0, 1.0, size=(R, n_in)), 0))
    L = mlp.layout(n_in, h1, h2)
    p = np.zeros(L["n"])
    for name, (o, n), fan in (("W1", L["W1"], (n_in, h1)), ("W2", L["W2"], (h1, h2)), ("W3", L["W3"], (h2, 2))):
        s = np.sqrt(6.0 / sum(fan))
        p[o:o + n] = rng.uniform(-s, s, n)
    p = p.astype(np.float32).astype(np.float64)
    lnn, lrn = mlp.batch_edges(B, nn, rn)
    return X, p, lnn, lrn, R


# (45, .., 51, 2, 1): 204 batch rows, not a multiple of 8 (the feature-major
# copies are padded with zeros to 208), and an input width that is not a
# multiple of 8 (element-wise staging of the batch input)
@pytest.mark.parametrize("n_in,h1,h2,B,nn,rn", [(40, 32, 24, 50, 2, 1), (784, 512, 512, 256, 5, 1),
                                               (45, 40, 16, 51, 2, 1)])
def test_training_step_matches_the_reference(pkg, n_in, h1, h2, B, nn, rn):
    m, api, ag, par = pkg
    X, p, lnn, lrn, R = _setup(pkg, n_in, h1, h2, B, nn, rn, 11)
    c, eps, lr, scale = 0.1, 1e-12, 1e-3, 1.0 / B
    enc = par.ParametricIVHD(n_in, (h1, h2), batch=B, nn=nn, rn=rn, max_rows=R)
    enc.set_params(torch.from_numpy(p.astype(np.float32)).cuda())
    plan = ag.StressEdges(torch.from_numpy(lnn).cuda(), torch.from_numpy(lrn).cuda(), c=c)
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    api.ivhd_enc_train_step(enc.handle, _bits(X), plan.handle, c, eps, lr, scale, loss)
    torch.cuda.synchronize()
    _, _, _, g_ref, E_ref = mlp.train_step(p, np.zeros_like(p), np.zeros_like(p), 1, X, lnn, lrn, n_in, h1, h2,
                                            c=np.float32(c), eps=np.float32(eps), lr=lr, scale=scale)
    assert loss.item() == pytest.approx(E_ref, rel=1e-4)
    g_gpu = enc.grads().cpu().numpy().astype(np.float64)
    assert _norm_rel(g_gpu, g_ref) <= 1e-3
    L = mlp.layout(n_in, h1, h2)
    blk = lambda g, name: g[L[name][0]:L[name][0] + L[name][1]]
    for name in ("W1", "b1", "W2", "b2", "W3"):   # each block on its own, biases included
        assert _norm_rel(blk(g_gpu, name), blk(g_ref, name)) <= 2e-3, name
    # the output bias receives the sum of all forces, zero because every
    # pair pushes its two ends equally and oppositely: only rounding is left
    assert np.linalg.norm(blk(g_gpu, "b3")) <= 1e-3 * np.linalg.norm(blk(g_ref, "W3"))
    # the Adam step itself, on the GPU's own gradients (a sign flip of a
    # near-zero gradient moves a weight by 2 lr, so it is checked apart)
    p1_from_gpu_grads, _, _ = mlp.adam(p, g_gpu * scale, np.zeros_like(p), np.zeros_like(p), 1, lr)
    np.testing.assert_allclose(enc.params().cpu().numpy(), p1_from_gpu_grads, rtol=1e-5, atol=1e-7)
    # forward alone
    Z = enc.embed(_bits(X[:B]))
    Z_ref, _ = mlp.forward(enc.params().cpu().numpy().astype(np.float64), X[:B], n_in, h1, h2)
    assert _norm_rel(Z.cpu().numpy(), Z_ref) <= 1e-3
    enc.close()
    plan.close()


def test_training_lowers_the_batch_stress_and_separates_clusters(pkg):
    # small mixture: 6,000 points in 64-D, 6 clusters; a few epochs of training
    m, api, ag, par = pkg
    import synth
    rng = synth.rng_for(77)
    X, labels = synth.gaussian_mixture(6000, 64, 6, centre_var=16.0, sigma=1.0, rng=rng)
    dX = torch.from_numpy(X).cuda()
    nn_idx = m.ivhd_knn_build(dX, 5)
    enc = par.ParametricIVHD(64, (64, 64), batch=256, nn=5, rn=1, lr=3e-3, seed=1)
    x16 = par.ParametricIVHD.to_bf16(dX)
    enc.fit(x16, nn_idx, epochs=8)
    assert enc.losses[-1] < 0.7 * enc.losses[0]
    Z = enc.embed(x16).cpu().numpy()
    assert np.all(np.isfinite(Z))
    assert oracle.cf_k(Z, labels, 10) > 0.9
    enc.close()


def _epoch_order(M, batch, seed, epoch):
    """Sources of each step of a training epoch: s = (a t + c0) mod M over the
    epoch's step slots t, a coprime to M, a and c0 from SplitMix64 of seed and
    epoch (the definition the encoder documents)."""
    from math import gcd
    mask = (1 << 64) - 1
    a = oracle.splitmix64((seed ^ oracle.splitmix64((0x5EED + epoch) & mask)) & mask) % M
    if a == 0:
        a = 1
    while gcd(a, M) != 1:
        a = 1 if a + 1 == M else a + 1
    c0 = oracle.splitmix64((seed + 7919 * epoch) & mask) % M
    steps = (M + batch - 1) // batch
    t = np.arange(steps * batch, dtype=np.int64)
    return ((a * t + c0) % M).reshape(steps, batch)


@pytest.mark.parametrize("M,n_in,h1,h2,batch,nn,rn,absent", [(1000, 40, 32, 24, 128, 3, 1, 0.0),
                                                            (777, 45, 40, 16, 100, 2, 2, 0.1)])
def test_training_epochs_match_the_reference_composition(pkg, M, n_in, h1, h2, batch, nn, rn, absent):
    # two whole epochs of ivhd_enc_train_epoch against the oracle composed step
    # by step: the epoch's visiting order, each batch's rows (sources, their nn
    # targets with an absent slot repeating the source, their rn targets of the
    # epoch's draw), the batch edge lists, the reference training step
    m, api, ag, par = pkg
    import synth
    rng = np.random.default_rng(M)
    X32 = np.maximum(rng.normal(1.0, 1.0, size=(M, n_in)), 0).astype(np.float32)
    Xb = mlp.bf16_round(X32)
    nn_idx = synth.random_neighbour_graph(M, nn, rng, hub_alpha=1.0, absent_frac=absent)
    seed, c, eps, lr = 5, 0.1, 1e-12, 3e-4
    enc = par.ParametricIVHD(n_in, (h1, h2), batch=batch, nn=nn, rn=rn, c=c, lr=lr, seed=seed)
    p = enc.params().cpu().numpy().astype(np.float64)
    p0 = p.copy()
    mo, vo = np.zeros_like(p), np.zeros_like(p)
    t = 0
    lnn, lrn = mlp.batch_edges(batch, nn, rn)
    x16 = par.ParametricIVHD.to_bf16(torch.from_numpy(X32).cuda())
    d_nn = torch.from_numpy(nn_idx).cuda()
    for epoch in range(2):
        loss_gpu = api.ivhd_enc_train_epoch(enc.handle, x16, d_nn, rn, seed, epoch, batch, c, eps, lr)
        rn_e = oracle.rn_sample(nn_idx, rn, seed, epoch)
        losses = []
        for src in _epoch_order(M, batch, seed, epoch):
            nbr = nn_idx[src]
            nbr = np.where(nbr >= 0, nbr, src[:, None])
            rows = np.concatenate([src, nbr.ravel(), rn_e[src].ravel()])
            t += 1
            p, mo, vo, _, E = mlp.train_step(p, mo, vo, t, Xb[rows], lnn, lrn, n_in, h1, h2, c=np.float32(c),
                                             eps=np.float32(eps), lr=lr, scale=1.0 / batch)
            losses.append(E / batch)
        loss_ref = float(np.mean(losses))
        print(f"epoch {epoch}: loss gpu {loss_gpu:.6f} reference {loss_ref:.6f}")
        assert loss_gpu == pytest.approx(loss_ref, rel=2e-3)
    pg = enc.params().cpu().numpy().astype(np.float64)
    # the parameters moved the same way (Adam steps of size about lr per weight)
    assert _norm_rel(pg - p0, p - p0) <= 0.05
    enc.close()
