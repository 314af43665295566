"""MI355X (gfx950) implementation of the per-time-step particle update of the hybrid
stochastic-particle-Shakhov / DSMC method (arXiv 2506.23917).

The library is libhs.so (HIP kernels + C ABI, include/hs.h); `hs` is its Python binding.
"""
from . import hs  # noqa: F401
from .hs import Sim, HsError, FP64, FP32_MIXED  # noqa: F401
