"""Parity of the HIP loop (through the C ABI) with the FP64 oracle.

Single steps from the same FP32 state must agree to 1e-5, norm-wise over
the whole array (the infinity norm of the oracle's array is the scale, so
near-zero entries do not dominate); the random neighbours must agree bit
for bit; the FP64 stress to 1e-10 relative; whole runs, whose trajectories
diverge, by their kNN-preservation score Q_NX(10) within 0.01.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ivhd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05455_amd as m
    return m


def _case(M, nn, rn, seed, *, hub=0.0, absent=0.0, clusters=1, star=0):
    rng = np.random.default_rng(seed)
    labels = rng.integers(0, clusters, M).astype(np.int32) if clusters > 1 else None
    nn_idx = synth.random_neighbour_graph(M, nn, rng, labels=labels, hub_alpha=hub, absent_frac=absent)
    if star:
        # the first `star` vertices all point at vertex 0: one very long in-edge list
        nn_idx[1:star + 1, 0] = 0
    Y = rng.normal(0, 2.0, size=(M, 2)).astype(np.float32)
    V = (0.01 * rng.normal(size=(M, 2))).astype(np.float32)
    return nn_idx, Y, V


def f32(x):
    """The value a float parameter takes once it crosses the ABI (float32)."""
    return float(np.float32(x))


def _transpose(idx, M):
    """Plain transpose of an [M][k] edge list: per target, the sources ascending."""
    k = idx.shape[1]
    src = np.repeat(np.arange(M, dtype=np.int64), k)
    dst = idx.ravel().astype(np.int64)
    keep = dst >= 0
    src, dst = src[keep], dst[keep]
    order = np.lexsort((src, dst))
    ptr = np.concatenate([[0], np.cumsum(np.bincount(dst, minlength=M))]).astype(np.int32)
    return ptr, src[order].astype(np.int32)


def _rel(x, ref):
    return float(np.max(np.abs(np.asarray(x, np.float64) - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _ctx(ivhd, nn_idx, Y, V, **kw):
    d_nn = torch.from_numpy(nn_idx).cuda()
    d_y = torch.from_numpy(Y).cuda()
    d_v = torch.from_numpy(V).cuda()
    return ivhd.Context(d_nn, d_y, d_v, **kw)


CASES = [
    # M, nn, rn, seed, extra
    (2000, 2, 1, 0, {}),
    (5003, 5, 1, 1, dict(absent=0.1)),
    (4099, 3, 2, 2, dict(hub=0.7)),
    (3001, 2, 1, 3, dict(star=2500)),
    (777, 1, 0, 4, {}),
    (3, 1, 1, 5, {}),
    (2, 1, 0, 6, {}),
]


@pytest.mark.parametrize("mode,reorder", [("det", True), ("det", False), ("atomic", True)])
@pytest.mark.parametrize("M,nn,rn,seed,extra", CASES)
def test_single_step_matches_oracle(ivhd, mode, reorder, M, nn, rn, seed, extra):
    a, b, c, eps = f32(0.9), f32(0.01), f32(0.1), f32(1e-12)
    nn_idx, Y, V = _case(M, nn, rn, seed, **extra)
    ctx = _ctx(ivhd, nn_idx, Y, V, rn=rn, a=a, b=b, c=c, eps=eps, seed=seed, mode=mode, reorder=reorder)
    rn_idx = ctx.rn_edges().cpu().numpy()
    assert np.array_equal(rn_idx, oracle.rn_sample(nn_idx, rn, seed, 0))
    f_ref = oracle.force(Y, nn_idx, rn_idx, c, eps)
    g = ctx.grad().cpu().numpy()
    assert _rel(-0.5 * g, f_ref) <= 1e-5
    Y1_ref, V1_ref = oracle.step(Y, V, f_ref, a, b)
    ctx.step(1)
    torch.cuda.synchronize()
    assert _rel(ctx.y.cpu().numpy(), Y1_ref) <= 1e-5
    assert _rel(ctx.v.cpu().numpy(), V1_ref) <= 1e-5
    assert ctx.iteration == 1
    ctx.close()


@pytest.mark.parametrize("mode", ["det", "atomic"])
def test_single_step_at_full_size(ivhd, mode):
    # 1.4M vertices, Zipf-sized clusters, heavy-tailed in-degree: the C3 shape
    cfg = synth.CONFIGS["C3"]
    rng = np.random.default_rng(30)
    sizes = synth.cluster_sizes(cfg.M, cfg.K, "zipf", cfg.zipf_s)
    labels = np.repeat(np.arange(cfg.K, dtype=np.int32), sizes)[rng.permutation(cfg.M)]
    nn_idx = synth.random_neighbour_graph(cfg.M, cfg.nn, rng, labels=labels, hub_alpha=1.2)
    Y = rng.random((cfg.M, 2)).astype(np.float32)
    V = (0.01 * rng.normal(size=(cfg.M, 2))).astype(np.float32)
    ctx = _ctx(ivhd, nn_idx, Y, V, rn=cfg.rn, a=cfg.a, b=cfg.b, c=cfg.c, seed=0,
               rn_resample_every=cfg.R, mode=mode)
    rn_idx = ctx.rn_edges().cpu().numpy()
    assert np.array_equal(rn_idx, oracle.rn_sample(nn_idx, cfg.rn, 0, 0))
    f_ref = oracle.force(Y, nn_idx, rn_idx, f32(cfg.c), f32(1e-12))
    assert _rel(-0.5 * ctx.grad().cpu().numpy(), f_ref) <= 1e-5
    Y1_ref, V1_ref = oracle.step(Y, V, f_ref, f32(cfg.a), f32(cfg.b))
    ctx.step(1)
    torch.cuda.synchronize()
    assert _rel(ctx.y.cpu().numpy(), Y1_ref) <= 1e-5
    assert _rel(ctx.v.cpu().numpy(), V1_ref) <= 1e-5
    E_ref = oracle.stress(ctx.y.cpu().numpy(), nn_idx, rn_idx, f32(cfg.c))
    assert ctx.stress() == pytest.approx(E_ref, rel=1e-10)
    ctx.close()


def _atomic_step_check(ivhd, nn_idx, Y, V, rn, seed, mask=None):
    a, b, c, eps = f32(0.9), f32(0.01), f32(0.1), f32(1e-12)
    ctx = _ctx(ivhd, nn_idx, Y, V, rn=rn, a=a, b=b, c=c, eps=eps, seed=seed, mode="atomic")
    rn_idx = ctx.rn_edges().cpu().numpy()
    f_ref = oracle.force(Y, nn_idx, rn_idx, c, eps)
    g = ctx.grad().cpu().numpy()
    assert _rel(-0.5 * g, f_ref) <= 1e-5
    if mask is not None:
        # vertices whose edges all stay inside the fixed-point range, on their own scale
        keep = mask(rn_idx)
        assert keep.sum() > 0
        assert _rel(-0.5 * g[keep], f_ref[keep]) <= 1e-5
    Y1_ref, V1_ref = oracle.step(Y, V, f_ref, a, b)
    ctx.step(1)
    torch.cuda.synchronize()
    assert _rel(ctx.y.cpu().numpy(), Y1_ref) <= 1e-5
    assert _rel(ctx.v.cpu().numpy(), V1_ref) <= 1e-5
    # three more steps, each from the GPU's own state, one of them without a
    # gradient call between (the float accumulator's flag slots alternate)
    for k in range(3):
        Yk, Vk = ctx.y.cpu().numpy(), ctx.v.cpu().numpy()
        fk = oracle.force(Yk, nn_idx, rn_idx, c, eps)
        if k != 1:
            assert _rel(-0.5 * ctx.grad().cpu().numpy(), fk) <= 1e-5
        Yn, Vn = oracle.step(Yk, Vk, fk, a, b)
        ctx.step(1)
        torch.cuda.synchronize()
        assert _rel(ctx.y.cpu().numpy(), Yn) <= 1e-5, k
        assert _rel(ctx.v.cpu().numpy(), Vn) <= 1e-5, k
    ctx.close()


def test_atomic_mode_reactions_beyond_the_fixed_range(ivhd):
    # a far cluster: its rn reactions (about c * 1000) exceed the fixed-point
    # range and take the float path, the rest stay in fixed point
    M, far = 3000, 40
    rng = np.random.default_rng(41)
    labels = np.zeros(M, np.int32); labels[:far] = 1
    nn_idx = synth.random_neighbour_graph(M, 2, rng, labels=labels)
    Y = rng.normal(0, 2.0, size=(M, 2)).astype(np.float32)
    Y[:far] += np.float32(1000.0)
    V = (0.01 * rng.normal(size=(M, 2))).astype(np.float32)

    def clear_of_the_far_cluster(rn_idx):
        touched = np.zeros(M, bool)
        touched[:far] = True
        hit = (rn_idx < far) & (rn_idx >= 0)
        touched[np.nonzero(hit.any(1))[0]] = True
        touched[rn_idx[:far].ravel()] = True
        return ~touched

    _atomic_step_check(ivhd, nn_idx, Y, V, 2, 5, mask=clear_of_the_far_cluster)


def test_atomic_mode_with_a_large_rn_in_degree(ivhd):
    # rn = 40 of 80 vertices: in-degrees near 60 narrow the fixed-point range
    # to a few c, so many reactions take the float path
    nn_idx, Y, V = _case(80, 2, 40, 42)
    _atomic_step_check(ivhd, nn_idx, Y, V, 40, 6)


def test_atomic_mode_is_bitwise_reproducible(ivhd):
    # the rn reactions are integer sums: the order of the atomics does not
    # change a bit, with or without graph replay, over redraws
    nn_idx, Y, V = _case(20000, 3, 2, 43)
    runs = []
    for graphs in (True, True, False):
        ctx = _ctx(ivhd, nn_idx, Y, V, rn=2, b=0.002, seed=7, rn_resample_every=7, mode="atomic")
        ctx.set_graphs(graphs)
        ctx.step(40)
        torch.cuda.synchronize()
        runs.append((ctx.y.cpu().numpy(), ctx.v.cpu().numpy(), ctx.grad().cpu().numpy()))
        ctx.close()
    assert np.all(np.isfinite(runs[0][0])) and not np.array_equal(runs[0][0], Y)
    for y, v, g in runs[1:]:
        assert np.array_equal(y, runs[0][0])
        assert np.array_equal(v, runs[0][1])
        assert np.array_equal(g, runs[0][2])


@pytest.mark.parametrize("M,nn,rn,seed,extra", CASES[:4])
def test_fp64_stress_matches_oracle(ivhd, M, nn, rn, seed, extra):
    nn_idx, Y, V = _case(M, nn, rn, seed, **extra)
    ctx = _ctx(ivhd, nn_idx, Y, V, rn=rn, c=0.1, seed=seed)
    rn_idx = ctx.rn_edges().cpu().numpy()
    c = f32(0.1)
    assert ctx.stress() == pytest.approx(oracle.stress(Y, nn_idx, rn_idx, c), rel=1e-10)
    Y2 = (Y * 1.5 + 0.25).astype(np.float32)
    E2 = ctx.stress(torch.from_numpy(Y2).cuda())
    assert E2 == pytest.approx(oracle.stress(Y2, nn_idx, rn_idx, c), rel=1e-10)
    ctx.close()


@pytest.mark.parametrize("mode", ["det", "atomic"])
def test_resample_schedule_matches_oracle_draws(ivhd, mode):
    nn_idx, Y, V = _case(3000, 2, 2, 7)
    R = 5
    ctx = _ctx(ivhd, nn_idx, Y, V, rn=2, b=0.005, seed=99, rn_resample_every=R, mode=mode)
    assert np.array_equal(ctx.rn_edges().cpu().numpy(), oracle.rn_sample(nn_idx, 2, 99, 0))
    ctx.step(1)
    # epoch e is drawn at the start of iteration e*R, so after e*R + 1 iterations
    for epoch in range(4):
        got = ctx.rn_edges().cpu().numpy()
        assert np.array_equal(got, oracle.rn_sample(nn_idx, 2, 99, epoch)), epoch
        ctx.step(R)
    ctx.close()


@pytest.mark.parametrize("mode", ["det", "atomic"])
def test_steps_across_redraws_match_the_oracle(ivhd, mode):
    # every step from the GPU's own state against the oracle's step with the
    # draw of that iteration's epoch: the transposed rn lists (det) and the
    # fixed-point range of the reactions (atomic) are rebuilt at each redraw
    M, nn, rn, R, seed = 3000, 2, 2, 3, 17
    a, b, c, eps = f32(0.9), f32(0.005), f32(0.1), f32(1e-12)
    nn_idx, Y, V = _case(M, nn, rn, seed)
    ctx = _ctx(ivhd, nn_idx, Y, V, rn=rn, a=a, b=b, c=c, eps=eps, seed=seed, rn_resample_every=R, mode=mode)
    for n in range(8):
        Yn, Vn = ctx.y.cpu().numpy(), ctx.v.cpu().numpy()
        rn_e = oracle.rn_sample(nn_idx, rn, seed, n // R)
        f_ref = oracle.force(Yn, nn_idx, rn_e, c, eps)
        Y1, V1 = oracle.step(Yn, Vn, f_ref, a, b)
        ctx.step(1)
        torch.cuda.synchronize()
        assert np.array_equal(ctx.rn_edges().cpu().numpy(), rn_e), n
        assert _rel(ctx.y.cpu().numpy(), Y1) <= 1e-5, n
        assert _rel(ctx.v.cpu().numpy(), V1) <= 1e-5, n
    ctx.close()


def _components(nn_idx, M):
    """Component label (smallest id) of each vertex of the undirected nn graph."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    src = np.repeat(np.arange(M), nn_idx.shape[1])
    dst = nn_idx.ravel()
    keep = dst >= 0
    A = sp.coo_matrix((np.ones(keep.sum()), (src[keep], dst[keep])), shape=(M, M))
    _, lab = connected_components(A, directed=False)
    first = np.full(lab.max() + 1, M)
    np.minimum.at(first, lab, np.arange(M))
    return first[lab]


def _internal(lists, perm, inv):
    out = lists[perm]
    return np.where(out >= 0, inv[np.maximum(out, 0)], -1).astype(np.int32)


@pytest.mark.parametrize("reorder", [True, False])
@pytest.mark.parametrize("M,nn,rn,seed,extra", CASES)
def test_in_edge_lists_are_the_exact_transpose(ivhd, M, nn, rn, seed, extra, reorder):
    nn_idx, Y, V = _case(M, nn, rn, seed, **extra)
    ctx = _ctx(ivhd, nn_idx, Y, V, rn=rn, seed=seed, rn_resample_every=3, reorder=reorder)
    perm = ctx.order().cpu().numpy()
    if reorder:
        # vertices grouped by connected component (smallest id first), then by
        # nn in-degree capped one above the hub threshold (80 from 500,000
        # vertices on, 16 below), then by first nn neighbour (absent last),
        # then by id
        comp = _components(nn_idx, M)
        indeg = np.bincount(nn_idx[nn_idx >= 0].ravel(), minlength=M)
        cap = 81 if M >= 500_000 else 17
        first = np.where(nn_idx[:, 0] >= 0, nn_idx[:, 0].astype(np.int64), 2**32 - 1)
        want = np.lexsort((np.arange(M), first, np.minimum(indeg, cap), comp))
        assert np.array_equal(perm, want)
    else:
        assert np.array_equal(perm, np.arange(M))
    inv = np.empty(M, np.int64)
    inv[perm] = np.arange(M)
    for step in range(3):
        ptr, src = ctx.in_edges("nn")
        want_ptr, want_src = _transpose(_internal(nn_idx, perm, inv), M)
        assert np.array_equal(ptr, want_ptr) and np.array_equal(src, want_src)
        if rn:
            ptr, src = ctx.in_edges("rn")
            want_ptr, want_src = _transpose(_internal(ctx.rn_edges().cpu().numpy(), perm, inv), M)
            assert np.array_equal(ptr, want_ptr) and np.array_equal(src, want_src)
        ctx.step(3)
    ctx.close()


def test_checkpoint_and_resume_is_bitwise(ivhd):
    nn_idx, Y, V = _case(5000, 3, 1, 14, hub=0.6)
    kw = dict(rn=1, b=5e-4, seed=21, rn_resample_every=6)
    ref = _ctx(ivhd, nn_idx, Y.copy(), V.copy(), **kw)
    ref.step(30)
    torch.cuda.synchronize()
    want_y, want_v = ref.y.cpu().numpy().copy(), ref.v.cpu().numpy().copy()
    ref.close()
    first = _ctx(ivhd, nn_idx, Y.copy(), V.copy(), **kw)
    first.step(17)
    torch.cuda.synchronize()
    ck_y, ck_v, ck_n = first.y.cpu().numpy().copy(), first.v.cpu().numpy().copy(), first.iteration
    first.close()
    resumed = _ctx(ivhd, nn_idx, ck_y, ck_v, **kw)
    resumed.set_iteration(ck_n)
    resumed.step(13)
    torch.cuda.synchronize()
    assert np.array_equal(resumed.y.cpu().numpy(), want_y)
    assert np.array_equal(resumed.v.cpu().numpy(), want_v)
    # set_state loads a layout into a running context
    resumed.set_state(torch.from_numpy(ck_y).cuda(), torch.from_numpy(ck_v).cuda())
    resumed.set_iteration(ck_n)
    resumed.step(13)
    torch.cuda.synchronize()
    assert np.array_equal(resumed.y.cpu().numpy(), want_y)
    resumed.close()


def test_two_contexts_give_bitwise_equal_gradients_and_steps(ivhd):
    nn_idx, Y, V = _case(6007, 3, 1, 8, hub=0.8)
    res = []
    for _ in range(2):
        ctx = _ctx(ivhd, nn_idx, Y.copy(), V.copy(), rn=1, seed=3)
        g = ctx.grad().cpu().numpy().copy()
        ctx.step(1)
        torch.cuda.synchronize()
        res.append((g, ctx.y.cpu().numpy().copy()))
        ctx.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


def test_det_mode_is_bitwise_reproducible_with_and_without_graphs(ivhd):
    # hubs of in-degree ~1e3 bound the stable step: b * lambda_max < 2 (1 + a)
    nn_idx, Y, V = _case(6007, 3, 1, 8, hub=0.8)
    outs = []
    for graphs, split in ((True, (23,)), (True, (5, 18)), (False, (23,)), (True, (1, 1, 21)),
                          (True, (7, 7, 7, 2)), (True, (14, 9))):
        ctx = _ctx(ivhd, nn_idx, Y.copy(), V.copy(), rn=1, b=1e-4, seed=3, rn_resample_every=7)
        ctx.set_graphs(graphs)
        for t in split:
            ctx.step(t)
        torch.cuda.synchronize()
        assert ctx.iteration == 23
        outs.append((ctx.y.cpu().numpy().copy(), ctx.v.cpu().numpy().copy()))
        assert np.all(np.isfinite(outs[-1][0]))
        ctx.close()
    for n, (y, v) in enumerate(outs[1:]):
        assert np.array_equal(y, outs[0][0]) and np.array_equal(v, outs[0][1]), f"variant {n + 1}"


def test_long_chunks_without_resampling_use_graphs_and_match_direct(ivhd):
    nn_idx, Y, V = _case(2000, 2, 1, 9)
    res = []
    for graphs in (True, False):
        ctx = _ctx(ivhd, nn_idx, Y.copy(), V.copy(), rn=1, seed=1)
        ctx.set_graphs(graphs)
        ctx.step(131)
        torch.cuda.synchronize()
        res.append(ctx.y.cpu().numpy().copy())
        ctx.close()
    assert np.array_equal(res[0], res[1])


@pytest.mark.parametrize("mode", ["det", "atomic"])
def test_centroid_stays_put(ivhd, mode):
    nn_idx, Y, V0 = _case(4000, 2, 1, 10)
    V = np.zeros_like(V0)
    ctx = _ctx(ivhd, nn_idx, Y, V, rn=1, seed=2, rn_resample_every=50, mode=mode)
    ctx.step(300)
    torch.cuda.synchronize()
    y = ctx.y.cpu().numpy().astype(np.float64)
    scale = np.abs(y).max()
    assert np.all(np.abs(y.mean(0) - Y.astype(np.float64).mean(0)) <= 1e-5 * scale)
    ctx.close()


@pytest.mark.parametrize("mode", ["det", "atomic"])
def test_c1_run_matches_oracle_kNN_preservation(ivhd, mode):
    cfg = synth.CONFIGS["C1"]
    X, labels, Y0 = synth.make_inputs(cfg)
    nn_idx = oracle.knn(X, cfg.nn)
    V0 = np.zeros_like(Y0)
    Yo, _, _ = oracle.run(Y0, V0, nn_idx, rn=cfg.rn, a=cfg.a, b=cfg.b, c=cfg.c, seed=cfg.seed,
                          R=cfg.R, T=cfg.T)
    ctx = _ctx(ivhd, nn_idx, Y0.copy(), V0.copy(), rn=cfg.rn, a=cfg.a, b=cfg.b, c=cfg.c,
               seed=cfg.seed, rn_resample_every=cfg.R, mode=mode)
    ctx.step(cfg.T)
    torch.cuda.synchronize()
    Yg = ctx.y.cpu().numpy()
    q_gpu, q_ref = oracle.q_nx(X, Yg, 10), oracle.q_nx(X, Yo, 10)
    print(f"Q_NX(10) gpu={q_gpu:.4f} oracle={q_ref:.4f}")
    assert abs(q_gpu - q_ref) <= 0.01
    assert oracle.cf_k(Yg, labels, 10) >= 0.9
    ctx.close()


def test_invalid_neighbour_index_is_rejected_on_the_device(ivhd):
    nn_idx, Y, V = _case(500, 2, 1, 11)
    for bad in (500, -2, 10**6):
        g = nn_idx.copy(); g[17, 1] = bad
        with pytest.raises(ivhd.IvhdError) as e:
            _ctx(ivhd, g, Y, V)
        assert e.value.status == "IVHD_EINVAL"
    g = nn_idx.copy(); g[17, 0] = 17
    with pytest.raises(ivhd.IvhdError):
        _ctx(ivhd, g, Y, V)


def test_non_finite_positions_are_reported(ivhd):
    nn_idx, Y, V = _case(500, 2, 1, 12)
    Y[3] = np.nan
    ctx = _ctx(ivhd, nn_idx, Y, V)
    ctx.step(2)
    with pytest.raises(ivhd.IvhdError) as e:
        ctx.stress()
    assert e.value.status == "IVHD_ENUMERIC"
    ctx.close()


def test_zero_iterations_and_closed_context(ivhd):
    nn_idx, Y, V = _case(100, 2, 1, 13)
    ctx = _ctx(ivhd, nn_idx, Y, V)
    ctx.step(0)
    torch.cuda.synchronize()
    assert np.array_equal(ctx.y.cpu().numpy(), Y) and ctx.iteration == 0
    ctx.close()
    with pytest.raises(ivhd.IvhdError):
        ctx.step(1)
