"""The measurement probes against their plain definitions: the gather probe
returns the indexed rows, the atomic probe counts each index's hits in both
32-bit halves of its word (exact integers)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ivhd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05455_amd as m
    return m


@pytest.mark.parametrize("n_src,n,seed", [(1, 5, 0), (1000, 70000, 1), (1400000, 1400000, 2)])
def test_gather_probe_returns_the_indexed_rows(ivhd, n_src, n, seed):
    rng = np.random.default_rng(seed)
    src = rng.random((n_src, 2)).astype(np.float32)
    idx = rng.integers(0, n_src, n).astype(np.int32)
    out = ivhd.ivhd_probe_gather(torch.from_numpy(src).cuda(), torch.from_numpy(idx).cuda())
    assert np.array_equal(out.cpu().numpy(), src[idx])


@pytest.mark.parametrize("n_acc,n,seed", [(1, 1000, 0), (77, 100000, 1), (1400000, 1400000, 2)])
def test_atomic_probe_counts_every_hit(ivhd, n_acc, n, seed):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, n_acc, n).astype(np.int32)
    acc = torch.zeros(n_acc, dtype=torch.int64, device="cuda")
    ivhd.ivhd_probe_atomic(acc, torch.from_numpy(idx).cuda())
    ivhd.ivhd_probe_atomic(acc, torch.from_numpy(idx).cuda())
    w = acc.cpu().numpy().view(np.uint64)
    want = 2 * np.bincount(idx, minlength=n_acc).astype(np.uint64)
    assert np.array_equal(w >> np.uint64(32), want)
    assert np.array_equal(w & np.uint64(0xFFFFFFFF), want)
