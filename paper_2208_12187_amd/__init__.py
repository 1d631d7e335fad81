"""MI355X-native GRAPE (piecewise-constant quantum optimal control).

libqoc.so holds the HIP kernels and the C ABI (include/qoc.h); ``qoc`` is its
ctypes binding.
"""
from . import qoc

__all__ = ["qoc"]
