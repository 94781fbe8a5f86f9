"""ctypes binding of libkc_peaks.so (include/kc_peaks.h): on-device peak
microbenchmarks used as roofline denominators.  Marshalling only."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkc_peaks.so")
EXPORTS = ["kcp_hbm_copy", "kcp_lds_read", "kcp_valu_int32", "kcp_and_popcount"]
_lib = None


def load(path: str = LIB_PATH):
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"libkc_peaks.so not found at {path}: build it with `python -m paper_1403_0734_amd.build`")
        lib = ctypes.CDLL(path)
        P, i32, f32p, f64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
        lib.kcp_hbm_copy.restype = ctypes.c_int
        lib.kcp_hbm_copy.argtypes = [P, P, ctypes.c_size_t, i32, P, f32p, f64p]
        for name in EXPORTS[1:]:
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [i32, i32, i32, P, f32p, f64p]
        _lib = lib
    return _lib


def _call(name, *args):
    ms, work = ctypes.c_float(), ctypes.c_double()
    st = getattr(load(), name)(*args, ctypes.byref(ms), ctypes.byref(work))
    if st != 0:
        raise RuntimeError(f"{name} failed with status {st}")
    return ms.value, work.value


def hbm_copy(src_ptr: int, dst_ptr: int, nbytes: int, iters: int = 10, stream=None):
    """(ms per copy, bytes moved per copy)"""
    return _call("kcp_hbm_copy", src_ptr, dst_ptr, nbytes, iters, stream)


def lds_read(blocks: int, reps: int, iters: int = 10, stream=None):
    return _call("kcp_lds_read", blocks, reps, iters, stream)


def valu_int32(blocks: int, reps: int, iters: int = 10, stream=None):
    return _call("kcp_valu_int32", blocks, reps, iters, stream)


def and_popcount(blocks: int, reps: int, iters: int = 10, stream=None):
    return _call("kcp_and_popcount", blocks, reps, iters, stream)
