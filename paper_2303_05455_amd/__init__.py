"""IVHD on MI355X: the binary-distance stress embedding loop as HIP kernels
for gfx950 behind a C ABI (include/ivhd.h).

    from paper_2303_05455_amd import Context
    ctx = Context(nn_idx, y, rn=1, a=0.9, b=0.01, c=0.1, rn_resample_every=100)
    ctx.step(2000); E = ctx.stress()

The HIP library (``libivhd.so``) is built in place by
``python -m paper_2303_05455_amd.build``; nothing here falls back to the CPU.
"""
from .api import (Context, IvhdError, ivhd_destroy, ivhd_get_in_edges, ivhd_get_iteration,
                  ivhd_get_rn, ivhd_grad, ivhd_init, ivhd_knn_build, ivhd_knn_query,
                  ivhd_last_error, ivhd_set_graphs, ivhd_step, ivhd_stress, ivhd_version,
                  make_params)

__all__ = [
    "Context", "IvhdError", "ivhd_destroy", "ivhd_get_in_edges", "ivhd_get_iteration",
    "ivhd_knn_build", "ivhd_knn_query", "ivhd_get_rn", "ivhd_grad",
    "ivhd_init", "ivhd_last_error", "ivhd_set_graphs", "ivhd_step", "ivhd_stress", "ivhd_version",
    "make_params",
]
