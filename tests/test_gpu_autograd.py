"""The stress as a differentiable loss (edge plans + torch.autograd.Function)
against the FP64 oracle and against finite differences of the GPU's own
FP64 stress."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def m():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05455_amd as pkg
    from paper_2303_05455_amd import autograd
    return pkg, autograd


def f32(x):
    return float(np.float32(x))


def _rel(x, ref):
    return float(np.max(np.abs(np.asarray(x, np.float64) - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _case(M, nn, rn, seed, hub=0.0, absent=0.0):
    rng = np.random.default_rng(seed)
    nn_idx = synth.random_neighbour_graph(M, nn, rng, hub_alpha=hub, absent_frac=absent)
    rn_idx = oracle.rn_sample(nn_idx, rn, seed, 0)
    Y = rng.normal(0, 1.5, size=(M, 2)).astype(np.float32)
    return nn_idx, rn_idx, Y


@pytest.mark.parametrize("M,nn,rn,seed,hub,absent", [
    (1000, 3, 1, 0, 0.0, 0.0), (4001, 5, 1, 1, 0.8, 0.1), (777, 2, 0, 2, 0.0, 0.0),
    (2500, 1, 3, 3, 1.0, 0.0),
])
@pytest.mark.parametrize("reorder", [True, False])
def test_plan_stress_and_gradient_match_oracle(m, M, nn, rn, seed, hub, absent, reorder):
    pkg, ag = m
    nn_idx, rn_idx, Y = _case(M, nn, rn, seed, hub, absent)
    c = f32(0.1)
    edges = ag.StressEdges(torch.from_numpy(nn_idx).cuda(),
                           torch.from_numpy(rn_idx).cuda() if rn else None, c=c, reorder=reorder)
    y = torch.from_numpy(Y).cuda()
    E = edges.stress64(y).item()
    assert E == pytest.approx(oracle.stress(Y, nn_idx, rn_idx, c), rel=1e-10)
    g = edges.grad(y).cpu().numpy()
    assert _rel(g, oracle.grad(Y, nn_idx, rn_idx, c, f32(1e-12))) <= 1e-5
    edges.close()


def test_autograd_backward_scales_by_the_upstream_gradient(m):
    pkg, ag = m
    nn_idx, rn_idx, Y = _case(1000, 3, 1, 4)
    edges = ag.StressEdges(torch.from_numpy(nn_idx).cuda(), torch.from_numpy(rn_idx).cuda(), c=0.1)
    y = torch.from_numpy(Y).cuda().requires_grad_(True)
    loss = 3.0 * ag.IVHDStress.apply(y, edges)
    loss.backward()
    ref = 3.0 * oracle.grad(Y, nn_idx, rn_idx, f32(0.1), f32(1e-12))
    assert _rel(y.grad.cpu().numpy(), ref) <= 1e-5
    assert loss.item() == pytest.approx(3.0 * oracle.stress(Y, nn_idx, rn_idx, f32(0.1)), rel=1e-6)


def test_backward_matches_finite_differences_of_the_fp64_stress(m):
    # M = 1000, nn = 3, rn = 1; central differences with the perturbation the
    # FP32 layout actually receives, on 40 sampled coordinates
    pkg, ag = m
    nn_idx, rn_idx, Y = _case(1000, 3, 1, 5)
    edges = ag.StressEdges(torch.from_numpy(nn_idx).cuda(), torch.from_numpy(rn_idx).cuda(), c=0.1)
    y = torch.from_numpy(Y).cuda()
    g = edges.grad(y).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    errs = []
    for _ in range(40):
        i, a = int(rng.integers(1000)), int(rng.integers(2))
        h = 1e-3
        yp, ym = Y.copy(), Y.copy()
        yp[i, a] = np.float32(Y[i, a] + h)
        ym[i, a] = np.float32(Y[i, a] - h)
        Ep = edges.stress64(torch.from_numpy(yp).cuda()).item()
        Em = edges.stress64(torch.from_numpy(ym).cuda()).item()
        fd = (Ep - Em) / (float(yp[i, a]) - float(ym[i, a]))
        errs.append(abs(fd - g[i, a]) / max(1.0, abs(g[i, a])))
    assert max(errs) <= 1e-3


@pytest.mark.parametrize("reorder", [True, False])
def test_gradient_at_the_differentiable_stress_workload_size(m, reorder):
    # 1M vertices, nn = 5, rn = 1 (edge lists drawn without a neighbour search,
    # inside 8 labels: 8 components, as the clusters give)
    pkg, ag = m
    cfg = synth.CONFIGS["C4"]
    rng = np.random.default_rng(40)
    labels = rng.integers(0, cfg.K, cfg.M).astype(np.int32)
    nn_idx = synth.random_neighbour_graph(cfg.M, cfg.nn, rng, labels=labels, hub_alpha=1.5)
    rn_idx = oracle.rn_sample(nn_idx, cfg.rn, 1, 0)
    Y = rng.random((cfg.M, 2)).astype(np.float32)
    edges = ag.StressEdges(torch.from_numpy(nn_idx).cuda(), torch.from_numpy(rn_idx).cuda(), c=cfg.c,
                           reorder=reorder)
    y = torch.from_numpy(Y).cuda()
    E_ref = oracle.stress(Y, nn_idx, rn_idx, f32(cfg.c))
    assert edges.stress64(y).item() == pytest.approx(E_ref, rel=1e-10)
    g = edges.grad(y)
    assert _rel(g.cpu().numpy(), oracle.grad(Y, nn_idx, rn_idx, f32(cfg.c), f32(1e-12))) <= 1e-5
    E_f, g_f = edges.stress_grad(y)
    assert E_f.item() == pytest.approx(E_ref, rel=1e-10)
    assert torch.equal(g_f, g)


def test_one_shot_gradient_and_stress(m):
    pkg, ag = m
    nn_idx, rn_idx, Y = _case(3000, 2, 1, 6, hub=0.9)
    g, E = pkg.ivhd_grad_edges(torch.from_numpy(Y).cuda(), torch.from_numpy(nn_idx).cuda(),
                               torch.from_numpy(rn_idx).cuda(), 0.1, with_stress=True)
    assert E == pytest.approx(oracle.stress(Y, nn_idx, rn_idx, f32(0.1)), rel=1e-10)
    assert _rel(g.cpu().numpy(), oracle.grad(Y, nn_idx, rn_idx, f32(0.1), f32(1e-12))) <= 1e-5


def test_bad_random_neighbour_index_is_rejected(m):
    pkg, ag = m
    nn_idx, rn_idx, Y = _case(500, 2, 1, 7)
    bad = rn_idx.copy()
    bad[10, 0] = 500
    with pytest.raises(pkg.IvhdError):
        ag.StressEdges(torch.from_numpy(nn_idx).cuda(), torch.from_numpy(bad).cuda())


def test_gradient_descent_on_the_loss_lowers_the_stress(m):
    pkg, ag = m
    nn_idx, rn_idx, Y = _case(2000, 3, 1, 8)
    edges = ag.StressEdges(torch.from_numpy(nn_idx).cuda(), torch.from_numpy(rn_idx).cuda(), c=0.1)
    y = torch.from_numpy(Y).cuda().requires_grad_(True)
    opt = torch.optim.SGD([y], lr=0.002)
    losses = []
    for _ in range(30):
        opt.zero_grad()
        loss = ag.IVHDStress.apply(y, edges)
        loss.backward()
        opt.step()
        losses.append(loss.item())
    assert losses[-1] < 0.5 * losses[0]
    assert all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:]))


def test_forward_and_backward_on_another_torch_stream(m):
    # the plan is made on the default stream; the loss and its gradient are
    # then taken under a side stream, with no explicit synchronisation, and
    # must equal the same computation on the plan's own stream
    pkg, ag = m
    nn_idx, rn_idx, Y = _case(20000, 5, 1, 21, hub=0.8)
    edges = ag.StressEdges(torch.from_numpy(nn_idx).cuda(), torch.from_numpy(rn_idx).cuda(), c=0.1)
    y_ref = torch.from_numpy(Y).cuda().requires_grad_(True)
    loss_ref = ag.IVHDStress.apply(y_ref, edges)
    loss_ref.backward()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        y = torch.from_numpy(Y).to("cuda", non_blocking=False).mul_(1.0).requires_grad_(True)
        loss = ag.IVHDStress.apply(y, edges) * 3.0
        loss.backward()
        got_loss = loss.clone()
        got_grad = y.grad.clone()
    torch.cuda.synchronize()
    assert got_loss.item() == pytest.approx(3.0 * loss_ref.item(), rel=1e-6)
    assert torch.equal(got_grad, 3.0 * y_ref.grad)
    edges.close()


def test_reordered_plan_keeps_its_own_lists_and_agrees_with_the_plain_plan(m):
    # three label groups (so three or more components) with hubs and absent
    # slots; after creation the reordered plan no longer reads the caller's
    # lists, and both plans give the same stress and gradient up to summation
    # order, in the caller's order, on two different layouts
    pkg, ag = m
    rng = np.random.default_rng(31)
    M = 30011
    labels = rng.integers(0, 3, M).astype(np.int32)
    nn_idx = synth.random_neighbour_graph(M, 4, rng, labels=labels, hub_alpha=1.2, absent_frac=0.05)
    rn_idx = oracle.rn_sample(nn_idx, 2, 9, 0)
    c = f32(0.1)
    nn_t, rn_t = torch.from_numpy(nn_idx).cuda(), torch.from_numpy(rn_idx).cuda()
    plain = ag.StressEdges(nn_t.clone(), rn_t.clone(), c=c, reorder=False)
    ordered = ag.StressEdges(nn_t, rn_t, c=c, reorder=True)
    nn_t.fill_(-1)
    rn_t.fill_(-1)
    for s in (1.0, 3.0):
        Y = (rng.normal(0, s, size=(M, 2))).astype(np.float32)
        y = torch.from_numpy(Y).cuda()
        E_ref = oracle.stress(Y, nn_idx, rn_idx, c)
        assert ordered.stress64(y).item() == pytest.approx(E_ref, rel=1e-10)
        assert ordered.stress64(y).item() == pytest.approx(plain.stress64(y).item(), rel=1e-12)
        g_ref = oracle.grad(Y, nn_idx, rn_idx, c, f32(1e-12))
        g_o, g_p = ordered.grad(y).cpu().numpy(), plain.grad(y).cpu().numpy()
        assert _rel(g_o, g_ref) <= 1e-5
        assert _rel(g_o, g_p.astype(np.float64)) <= 1e-6
    ordered.close()
    plain.close()


@pytest.mark.parametrize("reorder", [True, False])
@pytest.mark.parametrize("M,nn,rn,seed,hub,absent", [
    (1000, 3, 1, 0, 0.0, 0.0), (4001, 5, 2, 1, 0.8, 0.1), (777, 2, 0, 2, 0.0, 0.0), (2500, 1, 3, 3, 1.0, 0.0),
    # tiny and ragged graphs: two vertices, three, half the nn slots absent,
    # and no nn edge at all (every vertex its own component)
    (2, 1, 0, 4, 0.0, 0.0), (3, 1, 1, 5, 0.0, 0.0), (65, 2, 1, 6, 0.0, 0.5), (500, 2, 1, 7, 0.0, 1.0),
])
def test_stress_and_gradient_from_one_pass(m, M, nn, rn, seed, hub, absent, reorder):
    # the fused call's stress is the oracle's (the per-edge terms of the
    # stress kernel, summed per block of the gradient kernel), its gradient
    # the gradient call's bit for bit, scaled or not; hubs (in-degree above
    # the threshold) exercise the wavefront-per-vertex path
    pkg, ag = m
    nn_idx, rn_idx, Y = _case(M, nn, rn, seed, hub, absent)
    c = f32(0.1)
    edges = ag.StressEdges(torch.from_numpy(nn_idx).cuda(),
                           torch.from_numpy(rn_idx).cuda() if rn else None, c=c, reorder=reorder)
    y = torch.from_numpy(Y).cuda()
    E_ref = oracle.stress(Y, nn_idx, rn_idx, c)
    E, g = edges.stress_grad(y)
    assert E.item() == pytest.approx(E_ref, rel=1e-10)
    assert E.item() == pytest.approx(edges.stress64(y).item(), rel=1e-12)
    assert torch.equal(g, edges.grad(y))
    s = torch.tensor([0.375], dtype=torch.float32, device="cuda")
    E2, g2 = edges.stress_grad(y, scale=s)
    assert E2.item() == E.item()
    assert torch.equal(g2, edges.grad(y, s))
    # the chain-rule scale, in place and out of place
    out = torch.empty_like(g)
    pkg.ivhd_scale_f32(g, s, out)
    assert torch.equal(out, g2)
    pkg.ivhd_scale_f32(g, s, g)
    assert torch.equal(g, g2)
    edges.close()


def test_autograd_takes_one_pass_when_the_layout_requires_a_gradient(m):
    # with a gradient the forward runs the fused call and the backward only
    # scales; without one the forward takes the stress alone; both losses
    # equal, and the gradient equals the gradient call's
    pkg, ag = m
    nn_idx, rn_idx, Y = _case(3001, 4, 1, 12, hub=0.9)
    edges = ag.StressEdges(torch.from_numpy(nn_idx).cuda(), torch.from_numpy(rn_idx).cuda(), c=0.1)
    y = torch.from_numpy(Y).cuda().requires_grad_(True)
    loss = ag.IVHDStress.apply(y, edges)
    (0.5 * loss).backward()
    with torch.no_grad():
        loss_ng = ag.IVHDStress.apply(y, edges)
    assert loss.item() == pytest.approx(loss_ng.item(), rel=1e-6)
    half = torch.tensor([0.5], dtype=torch.float32, device="cuda")
    assert torch.equal(y.grad, edges.grad(y.detach(), half))
    assert _rel(y.grad.cpu().numpy(), 0.5 * oracle.grad(Y, nn_idx, rn_idx, f32(0.1), f32(1e-12))) <= 1e-5
    edges.close()
