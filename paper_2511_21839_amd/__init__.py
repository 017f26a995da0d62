"""Forward-mode differentiable 3D PIC space-charge step on AMD MI355X (gfx950).

The compute path is libdpic.so (HIP kernels behind the C ABI of
include/dpic.h); this package only loads it (`dpic.lib()`) and marshals
arguments (`dpic.Simulation` and the dpic_* wrappers).
"""
from . import dpic  # noqa: F401
from .dpic import DpicError, Simulation  # noqa: F401

__all__ = ["dpic", "DpicError", "Simulation"]
