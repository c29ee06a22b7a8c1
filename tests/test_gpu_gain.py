"""What the trained encoder gains over plain IVHD on points it has not seen.

Input with local structure: a 2-D sheet curled into 64 dimensions
(synth.lifted_sheet), where a good layout keeps most 10-NN (Q_NX(10) of the
sheet's own coordinates is about 0.9, of a random layout 0.003).  The
encoder is trained on 20,000 points and places 5,000 held-out points; plain
IVHD embeds the same held-out points from a random start on their own
exact kNN graph.  Measured on the GPU:
* quality per time: the encoder's one forward pass against the time plain
  IVHD (graph build included) needs to reach the same Q_NX(10);
* quality per iteration: plain IVHD started from the encoder's layout (the
  fallback, ParametricIVHD.embed(refine_iters=...)) against plain IVHD from
  a random start after the same number of iterations.
Q_NX(10) is the oracle's, on every held-out point."""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05455_amd as m
    from paper_2303_05455_amd.parametric import ParametricIVHD
    return m, ParametricIVHD


def _plain(m, nn_idx, y0, iters, b):
    y = y0.clone()
    ctx = m.Context(nn_idx, y, rn=1, a=0.9, b=b, c=0.1, seed=3, rn_resample_every=100)
    ctx.step(iters)
    torch.cuda.synchronize()
    ctx.close()
    return y


@pytest.mark.timeout(900)
def test_encoder_gains_over_plain_ivhd_on_held_out_points(pkg):
    m, Enc = pkg
    N, nn = 64, 5
    Xt, lt, _ = synth.lifted_sheet(20_000, N, np.random.default_rng(1))
    Xh, lh, uh = synth.lifted_sheet(5_000, N, np.random.default_rng(2))
    dXt, dXh = torch.from_numpy(Xt).cuda(), torch.from_numpy(Xh).cuda()
    enc = Enc(N, (128, 128), batch=512, nn=nn, rn=1, c=0.1, lr=1e-3, seed=4)
    enc.fit(Enc.to_bf16(dXt), m.ivhd_knn_build(dXt, nn), epochs=40)
    xh16 = Enc.to_bf16(dXh)
    z = enc.embed(xh16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z = enc.embed(xh16, z)
    torch.cuda.synchronize()
    t_enc = time.perf_counter() - t0
    q = lambda y: oracle.q_nx(Xh, y.cpu().numpy(), 10)
    q_enc = q(z)
    q_rand = 10 / (Xh.shape[0] - 1)
    # plain IVHD on the held-out points: its own graph, random start
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nn_h = m.ivhd_knn_build(dXh, nn)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    indeg = int(torch.bincount(nn_h.reshape(-1).long(), minlength=Xh.shape[0]).max())
    b = 0.25 * 2 * 1.9 / (indeg + nn + 4)
    y0 = torch.from_numpy(synth.init_positions(Xh.shape[0], np.random.default_rng(5))).cuda()
    curve = []
    for iters in (25, 50, 100, 200, 400, 800, 1600, 3200):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = _plain(m, nn_h, y0, iters, b)
        curve.append((iters, time.perf_counter() - t0 + t_graph, q(y)))
    # the fallback: plain IVHD from the encoder's layout
    warm = [(it, q(enc.embed(xh16, refine_iters=it, nn_idx=nn_h, b=b, seed=3))) for it in (25, 50, 100)]
    print(f"encoder: Q_NX(10) = {q_enc:.3f} in {t_enc * 1e3:.2f} ms (random layout {q_rand:.4f})")
    for it, t, qq in curve:
        print(f"plain IVHD {it:5d} it: Q_NX(10) = {qq:.3f} in {t * 1e3:.1f} ms (graph included)")
    for it, qq in warm:
        print(f"plain IVHD from the encoder's layout, {it} it: Q_NX(10) = {qq:.3f}")
    assert q_enc > 30 * q_rand
    # quality per time: plain IVHD needs longer than one forward pass to match it
    reach = [t for it, t, qq in curve if qq >= q_enc]
    assert not reach or min(reach) > 5 * t_enc
    # quality per iteration: the warm start is ahead of the random start
    cold = dict((it, qq) for it, _, qq in curve)
    for it, qq in warm:
        assert qq >= cold[it] + 0.05, (it, qq, cold[it])
    enc.close()
