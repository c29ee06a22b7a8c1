"""The C ABI on the CPU: the library loads, exports every entry point that
include/ivhd.h declares, and rejects bad arguments on the host before any
device work (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2303_05455_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2303_05455_amd import build
        build.build()
    return _lib.load()


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ivhd_\w+)\s*\(", text)))


HEADERS = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))


def test_every_declared_symbol_is_exported(lib):
    names = _declared("ivhd.h")
    assert "ivhd_init" in names and "ivhd_step" in names
    for h in HEADERS:
        for n in _declared(h):
            assert hasattr(lib, n), (h, n)


def test_binding_covers_every_declared_symbol():
    from paper_2303_05455_amd import _lib, api
    for h in HEADERS:
        for n in _declared(h):
            assert n in _lib.SIGNATURES, n
            assert hasattr(api, n), n


def test_struct_layout_matches_header():
    from paper_2303_05455_amd._lib import ivhd_params
    assert ctypes.sizeof(ivhd_params) == 56
    assert ivhd_params.seed.offset == 32 and ivhd_params.mode.offset == 44
    assert ivhd_params.flags.offset == 48


def _params(**kw):
    from paper_2303_05455_amd._lib import ivhd_params
    base = dict(M=100, nn=2, rn=1, a=0.9, b=0.01, c=0.1, eps=1e-12, seed=0,
                rn_resample_every=0, mode=0, flags=1, reserved=0)
    base.update(kw)
    return ivhd_params(**base)


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


@pytest.mark.parametrize("kw,frag", [
    (dict(M=1), "M ="), (dict(M=2**31), "M ="), (dict(nn=0), "nn ="), (dict(nn=65), "nn ="),
    (dict(rn=-1), "rn ="), (dict(M=3, nn=2, rn=1), "exceeds M - 1"),
    (dict(a=1.5), "a ="), (dict(a=float("nan")), "a ="), (dict(b=0.0), "b ="),
    (dict(b=float("inf")), "b ="), (dict(c=0.0), "c ="), (dict(c=1.0), "c ="),
    (dict(eps=-1.0), "eps ="), (dict(rn_resample_every=-3), "rn_resample_every"),
    (dict(mode=7), "mode ="), (dict(M=2**30, nn=4), "2^31-1 edges"), (dict(flags=8), "flags ="),
    (dict(reserved=3), "reserved ="),
])
def test_init_rejects_bad_parameters(lib, kw, frag):
    h = ctypes.c_void_p(123)
    p = _params(**kw)
    rc = lib.ivhd_init(ctypes.byref(h), ctypes.byref(p), FAKE, FAKE, ctypes.c_void_p(0x2000), None)
    assert rc == -1
    assert frag in lib.ivhd_last_error().decode()
    assert h.value is None


def test_init_rejects_null_pointers(lib):
    p = _params()
    h = ctypes.c_void_p()
    assert lib.ivhd_init(None, ctypes.byref(p), FAKE, FAKE, FAKE, None) == -1
    assert lib.ivhd_init(ctypes.byref(h), None, FAKE, FAKE, FAKE, None) == -1
    assert lib.ivhd_init(ctypes.byref(h), ctypes.byref(p), None, FAKE, FAKE, None) == -1
    assert "d_nn_idx" in lib.ivhd_last_error().decode()
    assert lib.ivhd_init(ctypes.byref(h), ctypes.byref(p), FAKE, None, FAKE, None) == -1
    assert lib.ivhd_init(ctypes.byref(h), ctypes.byref(p), FAKE, FAKE, None, None) == -1
    assert lib.ivhd_init(ctypes.byref(h), ctypes.byref(p), FAKE, FAKE, FAKE, None) == -1
    assert "alias" in lib.ivhd_last_error().decode()


def test_calls_on_a_missing_or_foreign_context_report_state(lib):
    bogus = ctypes.c_void_p(0xDEAD0)
    n = ctypes.c_int64()
    E = ctypes.c_double()
    for ctx in (None, bogus):
        assert lib.ivhd_step(ctx, 1) == -4
        assert lib.ivhd_stress(ctx, None, ctypes.byref(E)) == -4
        assert lib.ivhd_grad(ctx, None, FAKE) == -4
        assert lib.ivhd_get_rn(ctx, FAKE) == -4
        assert lib.ivhd_get_iteration(ctx, ctypes.byref(n)) == -4
        assert lib.ivhd_set_graphs(ctx, 1) == -4
        assert lib.ivhd_set_iteration(ctx, 0) == -4
        assert lib.ivhd_set_state(ctx, FAKE, FAKE) == -4
        assert lib.ivhd_get_order(ctx, FAKE) == -4
        assert lib.ivhd_set_adaptive(ctx, 1, 0.01, 1.0, 1.1, 0.5) == -4
        assert lib.ivhd_get_adaptive(ctx, None, None, None, None) == -4
        assert lib.ivhd_set_adam(ctx, 1, 1e-3, 0.9, 0.999, 1e-8) == -4
    assert lib.ivhd_destroy(None) == 0
    assert lib.ivhd_destroy(bogus) == -4
    assert "invalid context" in lib.ivhd_last_error().decode()


def test_version(lib):
    assert lib.ivhd_version() >= 100


@pytest.mark.parametrize("M,nn,kh,frag", [
    (1, 2, 8, "M ="), (100, 0, 8, "nn ="), (100, 65, 8, "nn ="), (100, 2, 0, "kh ="),
    (100, 2, 257, "kh ="), (2**30, 4, 8, "max(nn, kh)"),
])
def test_rnn_mask_rejects_bad_sizes(lib, M, nn, kh, frag):
    assert lib.ivhd_rnn_mask(FAKE, M, nn, FAKE, kh, ctypes.c_void_p(0x2000), None) == -1
    assert frag in lib.ivhd_last_error().decode()


def test_rnn_mask_rejects_null_and_aliased_buffers(lib):
    assert lib.ivhd_rnn_mask(None, 100, 2, FAKE, 8, FAKE, None) == -1
    assert lib.ivhd_rnn_mask(FAKE, 100, 2, FAKE, 8, FAKE, None) == -1
    assert "alias" in lib.ivhd_last_error().decode()


@pytest.mark.parametrize("M,nn,rn,frag", [
    (1, 2, 1, "M ="), (100, 0, 1, "nn ="), (100, 2, 65, "rn ="),
    (2_000_000, 2, 1, "above the 67108864-byte limit"), (1_100_000, 5, 1, "above the 67108864-byte limit"),
])
def test_grad_edges_noalloc_rejects_bad_sizes_before_device_work(lib, M, nn, rn, frag):
    E = ctypes.c_double()
    rc = lib.ivhd_grad_edges_noalloc(FAKE, M, FAKE, nn, FAKE, rn, 0.1, 1e-12, ctypes.c_void_p(0x2000),
                                     ctypes.byref(E), None)
    assert rc == -1
    assert frag in lib.ivhd_last_error().decode()


def test_grad_edges_noalloc_rejects_null_and_aliased_buffers(lib):
    assert lib.ivhd_grad_edges_noalloc(FAKE, 100, None, 2, FAKE, 1, 0.1, 1e-12, FAKE, None, None) == -1
    assert lib.ivhd_grad_edges_noalloc(FAKE, 100, FAKE, 2, FAKE, 1, 0.1, 1e-12, FAKE, None, None) == -1
    assert "alias" in lib.ivhd_last_error().decode()


def test_eval_calls_reject_bad_sizes_before_device_work(lib):
    out = (ctypes.c_double * 3)()
    assert lib.ivhd_eval_neighbours(FAKE, 1, 2, FAKE, 10, 1, FAKE, None) == -1
    assert "M =" in lib.ivhd_last_error().decode()
    assert lib.ivhd_eval_neighbours(FAKE, 100, 1025, FAKE, 10, 1, FAKE, None) == -1
    assert "N =" in lib.ivhd_last_error().decode()
    assert lib.ivhd_eval_neighbours(FAKE, 100, 2, FAKE, 10, 129, FAKE, None) == -1
    assert "k =" in lib.ivhd_last_error().decode()
    assert lib.ivhd_eval_neighbours(FAKE, 10, 2, FAKE, 10, 10, FAKE, None) == -1
    assert lib.ivhd_eval_neighbours(FAKE, 100, 2, FAKE, 10, 5, None, None) == -1
    assert lib.ivhd_eval_ranks(FAKE, 100, 2, FAKE, 10, FAKE, 65, FAKE, None) == -1
    assert "kc =" in lib.ivhd_last_error().decode()
    assert lib.ivhd_eval_ranks(FAKE, 100, 2, FAKE, 10, None, 5, FAKE, None) == -1
    assert lib.ivhd_eval_scores(100, FAKE, 10, FAKE, 5, FAKE, 10, None, None, 11, ctypes.cast(out, ctypes.c_void_p),
                                None) == -1
    assert "k =" in lib.ivhd_last_error().decode()
    assert lib.ivhd_eval_scores(100, FAKE, 10, FAKE, 5, FAKE, 10, None, None, 6, ctypes.cast(out, ctypes.c_void_p),
                                None) == -1
    assert "kx" in lib.ivhd_last_error().decode()
    assert lib.ivhd_eval_scores(100, FAKE, 10, None, 0, FAKE, 10, FAKE, None, 6, ctypes.cast(out, ctypes.c_void_p),
                                None) == -1
    assert "d_rank_y needs d_nx" in lib.ivhd_last_error().decode()
    assert lib.ivhd_eval_scores(100, FAKE, 0, None, 0, FAKE, 10, None, None, 6, ctypes.cast(out, ctypes.c_void_p),
                                None) == -1


def test_probe_atomic_rejects_bad_sizes(lib):
    assert lib.ivhd_probe_atomic(FAKE, 0, FAKE, 10, None) == -1
    assert lib.ivhd_probe_atomic(FAKE, 10, FAKE, -1, None) == -1
    assert lib.ivhd_probe_atomic(None, 10, FAKE, 5, None) == -1
    assert lib.ivhd_probe_atomic(None, 10, None, 0, None) == 0


def test_probe_gather_rejects_bad_sizes(lib):
    assert lib.ivhd_probe_gather(FAKE, 0, FAKE, 10, FAKE, None) == -1
    assert lib.ivhd_probe_gather(FAKE, 10, FAKE, -1, FAKE, None) == -1
    assert lib.ivhd_probe_gather(None, 10, FAKE, 5, FAKE, None) == -1
    assert lib.ivhd_probe_gather(None, 10, None, 0, None, None) == 0


def test_edges_create_rejects_unknown_flags_and_bad_sizes(lib):
    h = ctypes.c_void_p()
    assert lib.ivhd_edges_create(ctypes.byref(h), 100, FAKE, 2, FAKE, 1, 2, None) == -1
    assert "unknown flags" in lib.ivhd_last_error().decode()
    assert not h.value
    assert lib.ivhd_edges_create(ctypes.byref(h), 1, FAKE, 2, FAKE, 1, 1, None) == -1
    assert lib.ivhd_edges_create(ctypes.byref(h), 100, FAKE, 0, FAKE, 1, 1, None) == -1
    assert lib.ivhd_edges_create(ctypes.byref(h), 100, None, 2, FAKE, 1, 1, None) == -1
    assert lib.ivhd_edges_create(None, 100, FAKE, 2, FAKE, 1, 0, None) == -1


def test_fused_stress_gradient_and_scale_reject_bad_arguments(lib):
    assert lib.ivhd_edges_stress_grad(None, FAKE, 0.1, 1e-12, None, FAKE, FAKE) != 0
    assert "invalid edge plan" in lib.ivhd_last_error().decode()
    assert lib.ivhd_scale_f32(FAKE, -1, FAKE, FAKE, None) == -1
    assert lib.ivhd_scale_f32(None, 0, None, None, None) == 0
    assert lib.ivhd_scale_f32(FAKE, 10, None, FAKE, None) == -1
    assert lib.ivhd_scale_f32(None, 10, FAKE, FAKE, None) == -1
