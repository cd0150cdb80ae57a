"""MI355X (gfx950) library for the hot path of real-space deep variational QMC.

The compute path is libqmc.so (hand-written HIP kernels behind the C ABI in
include/qmc.h); qmc.py is its ctypes binding.
"""
from . import qmc  # noqa: F401
