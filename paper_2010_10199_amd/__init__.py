"""Grouped Fourier transform (ANOVA-structured NFFT) with LSQR and FISTA solvers on
MI355X (gfx950).

The compute path is the HIP library ``libgrouped.so`` (C ABI in ``include/grouped.h``),
reached through the ctypes binding in ``lib``; ``autograd`` wraps the forward transform
as a differentiable torch function.  PyTorch supplies device memory and streams only.
"""
from . import lib  # noqa: F401

__all__ = ["lib"]
