"""Exact and colour-sampled k-clique counting on AMD Instinct MI355X (gfx950).

The counting path lives in the HIP library libkc.so (sources in csrc/, C ABI in
include/kc.h); ``kc`` is its ctypes binding.
"""
from . import kc  # noqa: F401
