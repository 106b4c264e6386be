"""MI355X multiple rank-1 lattice FFT and dimension-incremental sparse FFT (arXiv 1711.05152).

The compute lives in ``libmr1l.so`` (hand-written HIP for gfx950, C ABI in ``include/mr1l.h``);
this package is its thin Python binding.
"""
from ._lib import Mr1lError, LIB_PATH  # noqa: F401

__all__ = ["Mr1lError", "LIB_PATH"]
