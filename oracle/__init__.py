"""CPU oracle (test infrastructure only).

A plain, slow, obviously correct k-clique counter in C (``oracle.c``) behind
ctypes.  Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may use it; the GPU library never imports it.

Definitions follow the paper (Finocchi, Finocchi & Fusco, arXiv 1403.0734):
the total order and high-neighbourhoods of Section 2, exact counting of
Section 3 (Algorithm 1, Theorem 1), colour sampling of Section 6.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, EOVERFLOW = 0, -1, -3, -4
COLOR_PER_ROOT, COLOR_GLOBAL = 0, 1


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        sig = {
            "kco_create": (i32, [P, P, u64, u32, ctypes.POINTER(P)]),
            "kco_destroy": (None, [P]),
            "kco_n": (u32, [P]),
            "kco_m": (u64, [P]),
            "kco_canon_edges": (None, [P, P, P]),
            "kco_degrees": (None, [P, P]),
            "kco_rank2id": (None, [P, P]),
            "kco_high_csr": (None, [P, P, P]),
            "kco_rank_csr": (None, [P, P, P]),
            "kco_max_outdeg": (u32, [P]),
            "kco_count_root": (i32, [P, u32, i32, P]),
            "kco_count_roots": (i32, [P, i32, P, u64, i32, P]),
            "kco_count_per_root": (i32, [P, i32, i32, P]),
            "kco_count": (i32, [P, i32, i32, P]),
            "kco_mix64": (u64, [u64]),
            "kco_hash_root": (u64, [u64, u32, u32]),
            "kco_hash_node": (u64, [u64, u32]),
            "kco_color": (u32, [u64, u32]),
            "kco_count_colored_root": (i32, [P, u32, i32, u32, u64, i32, P]),
            "kco_count_colored_per_root": (i32, [P, i32, u32, u64, i32, i32, P]),
            "kco_count_colored": (i32, [P, i32, u32, u64, i32, i32, P]),
            "kco_hash_pair": (u64, [u64, u32, u32, u32]),
            "kco_count_pair_sampled_root": (i32, [P, u32, i32, u64, u64, P]),
            "kco_count_pair_sampled": (i32, [P, i32, u64, u64, i32, P]),
            "kco_work_root": (i32, [P, u32, i32, P, P]),
            "kco_work_per_root": (i32, [P, i32, i32, P, P]),
            "kco_count_per_node": (i32, [P, i32, i32, P]),
            "kco_count_node": (i32, [P, u32, i32, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _check(st: int, what: str):
    if st != OK:
        raise OracleError(st, what)


def mix64(z: int) -> int:
    return int(_load().kco_mix64(z & (2**64 - 1)))


def hash_root(seed: int, u: int, x: int) -> int:
    return int(_load().kco_hash_root(seed, u, x))


def hash_node(seed: int, x: int) -> int:
    return int(_load().kco_hash_node(seed, x))


def color(h: int, c: int) -> int:
    return int(_load().kco_color(h, c))


def hash_pair(seed: int, u: int, x: int, y: int) -> int:
    """Pair-sampling hash of the pair (x, y) of Gamma+(u), x before y in the order."""
    return int(_load().kco_hash_pair(seed, u, x, y))


def pair_threshold(p: float) -> int:
    """t = floor(p * 2^32): a pair is kept iff (hash >> 32) < t (Section 6, plain pair
    sampling; t = 2^32 keeps every pair)."""
    if not (0.0 < p <= 1.0):
        raise ValueError("p must be in (0, 1]")
    return min(int(p * 2**32), 2**32)


class OracleGraph:
    """The simple graph, the paper's total order and the Gamma+ lists, on the CPU."""

    def __init__(self, n: int, src, dst):
        lib = _load()
        src = np.ascontiguousarray(src, dtype=np.uint32)
        dst = np.ascontiguousarray(dst, dtype=np.uint32)
        if src.shape != dst.shape:
            raise ValueError("src and dst differ in length")
        h = ctypes.c_void_p()
        _check(lib.kco_create(_p(src), _p(dst), src.shape[0], n, ctypes.byref(h)), "kco_create")
        self._h = h
        self.n = int(lib.kco_n(h))
        self.m = int(lib.kco_m(h))

    @classmethod
    def from_edgelist(cls, el):
        return cls(el.n, el.src, el.dst)

    def close(self):
        if getattr(self, "_h", None):
            _load().kco_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- structure --------------------------------------------------------
    def canon_edges(self):
        eu = np.empty(self.m, np.uint32)
        ev = np.empty(self.m, np.uint32)
        _load().kco_canon_edges(self._h, _p(eu), _p(ev))
        return eu, ev

    def degrees(self):
        d = np.empty(self.n, np.uint32)
        _load().kco_degrees(self._h, _p(d))
        return d

    def rank2id(self):
        r = np.empty(self.n, np.uint32)
        _load().kco_rank2id(self._h, _p(r))
        return r

    def high_csr(self):
        hp = np.empty(self.n + 1, np.uint64)
        hn = np.empty(self.m, np.uint32)
        _load().kco_high_csr(self._h, _p(hp), _p(hn))
        return hp, hn

    def rank_csr(self):
        optr = np.empty(self.n + 1, np.uint64)
        ocol = np.empty(self.m, np.uint32)
        _load().kco_rank_csr(self._h, _p(optr), _p(ocol))
        return optr, ocol

    def max_outdeg(self) -> int:
        return int(_load().kco_max_outdeg(self._h))

    # -- counts -------------------------------------------------------------
    def count(self, k: int, threads: int = 0) -> int:
        q = np.zeros(1, np.uint64)
        _check(_load().kco_count(self._h, k, threads, _p(q)), f"count(k={k})")
        return int(q[0])

    def count_per_root(self, k: int, threads: int = 0) -> np.ndarray:
        c = np.empty(self.n, np.uint64)
        _check(_load().kco_count_per_root(self._h, k, threads, _p(c)), f"count_per_root(k={k})")
        return c

    def count_root(self, u: int, k: int) -> int:
        q = np.zeros(1, np.uint64)
        _check(_load().kco_count_root(self._h, u, k, _p(q)), f"count_root(u={u},k={k})")
        return int(q[0])

    def count_roots(self, roots, k: int, threads: int = 0) -> np.ndarray:
        r = np.ascontiguousarray(roots, dtype=np.uint32)
        out = np.empty(r.shape[0], np.uint64)
        _check(_load().kco_count_roots(self._h, k, _p(r), r.shape[0], threads, _p(out)), "count_roots")
        return out

    def count_colored(self, k: int, c: int, seed: int, scheme: int = COLOR_PER_ROOT, threads: int = 0) -> int:
        q = np.zeros(1, np.uint64)
        _check(_load().kco_count_colored(self._h, k, c, seed, scheme, threads, _p(q)), "count_colored")
        return int(q[0])

    def count_colored_per_root(self, k: int, c: int, seed: int, scheme: int = COLOR_PER_ROOT,
                               threads: int = 0) -> np.ndarray:
        out = np.empty(self.n, np.uint64)
        _check(_load().kco_count_colored_per_root(self._h, k, c, seed, scheme, threads, _p(out)),
               "count_colored_per_root")
        return out

    def count_colored_root(self, u: int, k: int, c: int, seed: int, scheme: int = COLOR_PER_ROOT) -> int:
        q = np.zeros(1, np.uint64)
        _check(_load().kco_count_colored_root(self._h, u, k, c, seed, scheme, _p(q)), "count_colored_root")
        return int(q[0])

    def count_pair_sampled(self, k: int, p: float, seed: int, threads: int = 0) -> int:
        """Raw plain-pair-sampled count: the (k-1)-cliques of every sampled G+(u)."""
        q = np.zeros(1, np.uint64)
        _check(_load().kco_count_pair_sampled(self._h, k, pair_threshold(p), seed, threads, _p(q)),
               "count_pair_sampled")
        return int(q[0])

    def count_pair_sampled_root(self, u: int, k: int, p: float, seed: int) -> int:
        q = np.zeros(1, np.uint64)
        _check(_load().kco_count_pair_sampled_root(self._h, u, k, pair_threshold(p), seed, _p(q)),
               "count_pair_sampled_root")
        return int(q[0])

    def work_root(self, u: int, k: int):
        a = np.zeros(1, np.uint64)
        b = np.zeros(1, np.uint64)
        _check(_load().kco_work_root(self._h, u, k, _p(a), _p(b)), "work_root")
        return int(a[0]), int(b[0])

    def work_per_root(self, k: int, threads: int = 0):
        a = np.empty(self.n, np.uint64)
        b = np.empty(self.n, np.uint64)
        _check(_load().kco_work_per_root(self._h, k, threads, _p(a), _p(b)), "work_per_root")
        return a, b


    def count_per_node(self, k: int, threads: int = 0) -> np.ndarray:
        """k-cliques containing each node (by original id), summed over the roots'
        sub-problems (Section 3, remark after the round-3 reducers)."""
        out = np.empty(self.n, np.uint64)
        _check(_load().kco_count_per_node(self._h, k, threads, _p(out)), f"count_per_node(k={k})")
        return out

    def count_node(self, v: int, k: int) -> int:
        """k-cliques containing v, as the (k-1)-cliques inside its neighbourhood."""
        q = np.zeros(1, np.uint64)
        _check(_load().kco_count_node(self._h, v, k, _p(q)), f"count_node(v={v},k={k})")
        return int(q[0])


def scale_exponent(k: int, scheme: int) -> int:
    """Colour sampling keeps a k-clique with probability c^-(k-2) when each
    root colours its own high-neighbourhood (Section 6), and c^-(k-1) when all
    nodes share one colouring."""
    return k - 2 if scheme == COLOR_PER_ROOT else k - 1
