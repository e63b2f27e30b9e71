"""MI355X (gfx950) implementation of the MultiPhaseshift sparse Fourier method.

The compute path lives in libsfft.so (HIP kernels behind the C ABI of
include/sfft.h); `sfft` is its Python binding.
"""
from . import sfft  # noqa: F401

__all__ = ["sfft"]
