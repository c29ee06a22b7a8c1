"""IVHD on MI355X: the binary-distance stress embedding loop as HIP kernels
for gfx950 behind a C ABI (include/ivhd.h).

    from paper_2303_05455_amd import Context
    ctx = Context(nn_idx, y, rn=1, a=0.9, b=0.01, c=0.1, rn_resample_every=100)
    ctx.step(2000); E = ctx.stress()

The HIP library (``libivhd.so``) is built in place by
``python -m paper_2303_05455_amd.build``; nothing here falls back to the CPU.
"""
from .api import *  # noqa: F401,F403  (the C ABI under its own names, plus Context)
from .api import __all__  # noqa: F401
