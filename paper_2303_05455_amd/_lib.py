"""ctypes loader of libivhd.so (the HIP library built from csrc/).

There is no fallback: if the library is missing or does not load, every
entry point raises, naming the build command.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libivhd.so")

_lock = threading.Lock()
_lib = None

i32, i64, u64, f32, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float, ctypes.c_double
vp = ctypes.c_void_p


class ivhd_params(ctypes.Structure):
    """Mirror of ``ivhd_params`` in include/ivhd.h."""
    _fields_ = [
        ("M", i64), ("nn", i32), ("rn", i32),
        ("a", f32), ("b", f32), ("c", f32), ("eps", f32),
        ("seed", u64), ("rn_resample_every", i32), ("mode", i32),
        ("flags", i32), ("reserved", i32),
    ]


# name -> (restype, argtypes); every symbol declared in include/ivhd.h
SIGNATURES = {
    "ivhd_init": (i32, [ctypes.POINTER(vp), ctypes.POINTER(ivhd_params), vp, vp, vp, vp]),
    "ivhd_step": (i32, [vp, i64]),
    "ivhd_stress": (i32, [vp, vp, ctypes.POINTER(f64)]),
    "ivhd_grad": (i32, [vp, vp, vp]),
    "ivhd_get_rn": (i32, [vp, vp]),
    "ivhd_get_in_edges": (i32, [vp, i32, vp, vp]),
    "ivhd_get_order": (i32, [vp, vp]),
    "ivhd_set_state": (i32, [vp, vp, vp]),
    "ivhd_set_iteration": (i32, [vp, i64]),
    "ivhd_get_iteration": (i32, [vp, ctypes.POINTER(i64)]),
    "ivhd_set_graphs": (i32, [vp, i32]),
    "ivhd_set_adaptive": (i32, [vp, i32, f32, f64, f32, f32]),
    "ivhd_get_adaptive": (i32, [vp, vp, vp, vp, vp]),
    "ivhd_set_adam": (i32, [vp, i32, f32, f32, f32, f32]),
    "ivhd_rnn_mask": (i32, [vp, i64, i32, vp, i32, vp, vp]),
    "ivhd_ivf_train": (i32, [vp, i64, i32, i32, i32, vp, vp, vp]),
    "ivhd_ivf_search": (i32, [vp, i64, i32, vp, i32, vp, vp, i64, vp, i32, i32, vp, vp, vp]),
    "ivhd_destroy": (i32, [vp]),
    "ivhd_edges_create": (i32, [ctypes.POINTER(vp), i64, vp, i32, vp, i32, i32, vp]),
    "ivhd_edges_stress": (i32, [vp, vp, f32, vp]),
    "ivhd_edges_grad": (i32, [vp, vp, f32, f32, vp, vp]),
    "ivhd_edges_stress_grad": (i32, [vp, vp, f32, f32, vp, vp, vp]),
    "ivhd_scale_f32": (i32, [vp, i64, vp, vp, vp]),
    "ivhd_edges_destroy": (i32, [vp]),
    "ivhd_grad_edges": (i32, [vp, i64, vp, i32, vp, i32, f32, f32, vp, ctypes.POINTER(f64), vp]),
    "ivhd_grad_edges_noalloc": (i32, [vp, i64, vp, i32, vp, i32, f32, f32, vp, ctypes.POINTER(f64), vp]),
    "ivhd_enc_create": (i32, [ctypes.POINTER(vp), i32, i32, i32, u64, i64, vp]),
    "ivhd_enc_num_params": (i32, [vp, ctypes.POINTER(i64)]),
    "ivhd_enc_get_params": (i32, [vp, vp, vp]),
    "ivhd_enc_set_params": (i32, [vp, vp]),
    "ivhd_enc_embed": (i32, [vp, vp, i64, vp]),
    "ivhd_enc_train_step": (i32, [vp, vp, i64, vp, f32, f32, f32, f32, vp]),
    "ivhd_enc_train_epoch": (i32, [vp, vp, i64, vp, i32, i32, u64, i64, i64, f32, f32, f32,
                                   ctypes.POINTER(f64)]),
    "ivhd_enc_destroy": (i32, [vp]),
    "ivhd_f32_to_bf16": (i32, [vp, i64, vp, vp]),
    "ivhd_gemm_bf16": (i32, [vp, vp, i64, i64, i64, i64, i64, i32, i32, i32, vp, vp, i64, vp, i64, i32,
                             vp, vp]),
    "ivhd_knn_build": (i32, [vp, i64, i32, i32, vp, vp]),
    "ivhd_knn_query": (i32, [vp, i64, i32, vp, i64, vp, i32, vp, vp, vp]),
    "ivhd_eval_neighbours": (i32, [vp, i64, i32, vp, i64, i32, vp, vp]),
    "ivhd_eval_ranks": (i32, [vp, i64, i32, vp, i64, vp, i32, vp, vp]),
    "ivhd_eval_scores": (i32, [i64, vp, i64, vp, i32, vp, i32, vp, vp, i32, vp, vp]),
    "ivhd_probe_gather": (i32, [vp, i64, vp, i64, vp, vp]),
    "ivhd_probe_atomic": (i32, [vp, i64, vp, i64, vp]),
    "ivhd_last_error": (ctypes.c_char_p, []),
    "ivhd_version": (i32, []),
}

STATUS = {0: "IVHD_OK", -1: "IVHD_EINVAL", -2: "IVHD_ENOMEM", -3: "IVHD_EDEVICE",
          -4: "IVHD_ESTATE", -5: "IVHD_ENUMERIC"}


class IvhdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


def load():
    """Load libivhd.so once; raise if it is not built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_2303_05455_amd.build` "
                "(hipcc --offload-arch=gfx950). There is no CPU fallback.")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def check(code: int) -> int:
    if code != 0:
        msg = load().ivhd_last_error()
        raise IvhdError(code, msg.decode() if msg else "")
    return code
