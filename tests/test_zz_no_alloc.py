"""ivhd_grad_edges_noalloc (the entry point for callers that cannot allocate)
against ivhd_grad_edges on the same inputs, through the C ABI: several calls
in a row share the library's per-GPU scratch array, each later one on a
smaller input than the one before, so anything a call leaves behind that the
next one failed to clear would show."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05455_amd as p
    return p


def _case(M, nn, rn, seed, hub, absent):
    rng = np.random.default_rng(seed)
    nn_idx = synth.random_neighbour_graph(M, nn, rng, hub_alpha=hub, absent_frac=absent)
    rn_idx = oracle.rn_sample(nn_idx, rn, seed, 0) if rn else None
    Y = rng.normal(0, 1.5, size=(M, 2)).astype(np.float32)
    return nn_idx, rn_idx, Y


def test_noalloc_gradient_equals_the_allocating_entry_point_on_shrinking_inputs(pkg):
    c = float(np.float32(0.1))
    # the largest case is about the biggest the 64 MiB scratch holds at nn = 5, rn = 1
    for M, nn, rn, seed, hub, absent in [(1_000_000, 5, 1, 0, 1.0, 0.0), (60_001, 3, 2, 1, 0.8, 0.1),
                                         (4_097, 2, 1, 2, 1.2, 0.0), (777, 2, 0, 3, 0.0, 0.05)]:
        print(f"[case] M={M} nn={nn} rn={rn} seed={seed}", flush=True)
        nn_idx, rn_idx, Y = _case(M, nn, rn, seed, hub, absent)
        d_nn = torch.from_numpy(nn_idx).cuda()
        d_rn = torch.from_numpy(rn_idx).cuda() if rn else None
        y = torch.from_numpy(Y).cuda()
        ref, E_ref = pkg.ivhd_grad_edges(y, d_nn, d_rn, c, with_stress=True)
        out = torch.full_like(y, float("nan"))
        got, E = pkg.ivhd_grad_edges_noalloc(y, d_nn, d_rn, c, out=out, with_stress=True)
        torch.cuda.synchronize()
        # same kernels on the same lists: equal bit for bit (the floating-point
        # bar of the gradient, 1e-5 of its largest entry, is implied)
        assert torch.equal(got, ref), float((got - ref).abs().max())
        assert E == E_ref
        # and without the stress
        out2 = torch.full_like(y, float("nan"))
        pkg.ivhd_grad_edges_noalloc(y, d_nn, d_rn, c, out=out2)
        torch.cuda.synchronize()
        assert torch.equal(out2, ref)


def test_noalloc_rejects_a_bad_index_and_recovers(pkg):
    nn_idx, rn_idx, Y = _case(5000, 3, 1, 7, 0.5, 0.0)
    bad = nn_idx.copy()
    bad[123, 1] = 123   # a self edge
    y = torch.from_numpy(Y).cuda()
    out = torch.empty_like(y)
    with pytest.raises(pkg.IvhdError, match="equals its row"):
        pkg.ivhd_grad_edges_noalloc(y, torch.from_numpy(bad).cuda(), torch.from_numpy(rn_idx).cuda(), 0.1, out=out)
    d_nn, d_rn = torch.from_numpy(nn_idx).cuda(), torch.from_numpy(rn_idx).cuda()
    ref = pkg.ivhd_grad_edges(y, d_nn, d_rn, 0.1)
    pkg.ivhd_grad_edges_noalloc(y, d_nn, d_rn, 0.1, out=out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
