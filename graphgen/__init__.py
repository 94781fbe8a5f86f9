"""Seeded synthetic graph generators (raw edge lists, numpy uint32).

The C source (``graphgen.c``) holds only random draws; it knows nothing about
degrees, orientation or cliques, so both the CPU oracle and the GPU library can
consume its output without sharing any of the method's arithmetic.

The five workloads below stand in for the paper's SNAP social and web graphs
(Section 4, Table 1), which are not available: heavy-tailed degrees, skewed
high-neighbourhood sizes and, for the planted workload, dense local structure.
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u32, u64, i64, dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
        P = ctypes.c_void_p
        lib.gg_mix64_export.restype = u64
        lib.gg_mix64_export.argtypes = [u64]
        lib.gg_rand_export.restype = u64
        lib.gg_rand_export.argtypes = [u64, u64, u64]
        lib.gg_er.restype = u64
        lib.gg_er.argtypes = [u32, dbl, u64, P, P]
        lib.gg_solve_wmin.restype = dbl
        lib.gg_solve_wmin.argtypes = [dbl, dbl, dbl]
        lib.gg_chung_lu_edges.restype = i64
        lib.gg_chung_lu_edges.argtypes = [u32, dbl, dbl, dbl, u64]
        lib.gg_chung_lu.restype = i64
        lib.gg_chung_lu.argtypes = [u32, dbl, dbl, dbl, u64, P, P]
        lib.gg_planted.restype = i64
        lib.gg_planted.argtypes = [u32, u32, u32, u64, P, P]
        lib.gg_rmat.restype = i64
        lib.gg_rmat.argtypes = [u32, u32, dbl, dbl, dbl, u64, ctypes.c_int, P, P]
        lib.gg_batch_n.restype = u32
        lib.gg_batch_n.argtypes = [u64, u32, dbl, dbl]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class EdgeList:
    """Raw undirected edge list on ids [0, n); may hold self-loops and repeats."""

    def __init__(self, n: int, src: np.ndarray, dst: np.ndarray, name: str = ""):
        self.n = int(n)
        self.src = np.ascontiguousarray(src, dtype=np.uint32)
        self.dst = np.ascontiguousarray(dst, dtype=np.uint32)
        self.name = name

    @property
    def m_in(self) -> int:
        return int(self.src.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.uint64(self.n).tobytes())
        h.update(self.src.tobytes())
        h.update(self.dst.tobytes())
        return h.hexdigest()[:16]

    def __repr__(self):
        return f"EdgeList({self.name!r}, n={self.n}, m_in={self.m_in})"


def mix64(z: int) -> int:
    return int(_load().gg_mix64_export(z & (2**64 - 1)))


def rand(seed: int, stream: int, i: int) -> int:
    return int(_load().gg_rand_export(seed, stream, i))


def erdos_renyi(n: int, p: float, seed: int) -> EdgeList:
    lib = _load()
    m = int(lib.gg_er(n, p, seed, None, None))
    src = np.empty(m, np.uint32)
    dst = np.empty(m, np.uint32)
    lib.gg_er(n, p, seed, _ptr(src), _ptr(dst))
    return EdgeList(n, src, dst, f"er(n={n},p={p},seed={seed})")


def solve_wmin(mean: float, wmax: float, gamma: float) -> float:
    return float(_load().gg_solve_wmin(mean, wmax, gamma))


def chung_lu(n: int, gamma: float, mean: float, wmax: float, seed: int) -> EdgeList:
    lib = _load()
    M = int(lib.gg_chung_lu_edges(n, gamma, mean, wmax, seed))
    if M < 0:
        raise ValueError("no truncated power law with these parameters")
    src = np.empty(M, np.uint32)
    dst = np.empty(M, np.uint32)
    got = int(lib.gg_chung_lu(n, gamma, mean, wmax, seed, _ptr(src), _ptr(dst)))
    assert got == M
    return EdgeList(n, src, dst, f"chung_lu(n={n},g={gamma},mean={mean},wmax={wmax:.0f},seed={seed})")


def planted_cliques(n: int, count: int, size: int, seed: int):
    lib = _load()
    e = count * size * (size - 1) // 2
    src = np.empty(e, np.uint32)
    dst = np.empty(e, np.uint32)
    got = int(lib.gg_planted(n, count, size, seed, _ptr(src), _ptr(dst)))
    if got != e:
        raise ValueError("bad planted-clique parameters")
    return src, dst


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         permute: bool = True) -> EdgeList:
    lib = _load()
    M = edge_factor << scale
    src = np.empty(M, np.uint32)
    dst = np.empty(M, np.uint32)
    got = int(lib.gg_rmat(scale, edge_factor, a, b, c, seed, int(permute), _ptr(src), _ptr(dst)))
    if got != M:
        raise ValueError("bad R-MAT parameters")
    return EdgeList(1 << scale, src, dst, f"rmat(scale={scale},ef={edge_factor},seed={seed})")


def batch_sizes(count: int, seed: int, nlo: float = 1000.0, nhi: float = 200000.0):
    lib = _load()
    return [int(lib.gg_batch_n(seed, i, nlo, nhi)) for i in range(count)]


# --------------------------------------------------------------------------
# The benchmark workloads.  Seeds and parameters are fixed here so that every
# consumer reads byte-identical edge lists.

def workload_er2000() -> EdgeList:
    """G(2000, 0.01), seed 1."""
    g = erdos_renyi(2000, 0.01, 1)
    g.name = "er_n2000_p0.01"
    return g


def workload_chung_lu_1m(n: int = 1_000_000) -> EdgeList:
    """Chung-Lu, exponent 2.1, mean weight 20, max weight 5000, seed 2."""
    g = chung_lu(n, 2.1, 20.0, 5000.0, 2)
    g.name = f"chung_lu_n{n}_g2.1_mean20_wmax5000"
    return g


def workload_rmat22(scale: int = 22) -> EdgeList:
    """R-MAT scale 22, edge factor 16, (0.57, 0.19, 0.19, 0.05), permuted labels, seed 3."""
    g = rmat(scale, 16, 0.57, 0.19, 0.19, 3, permute=True)
    g.name = f"rmat{scale}_ef16"
    return g


def workload_batch(count: int = 512, seed: int = 4):
    """512 Chung-Lu graphs, exponent 2.3, mean 20, n_i log-uniform in [1000, 200000],
    max weight sqrt(20 n_i), graph i seeded with mix64(4 ^ i)."""
    out = []
    for i, n in enumerate(batch_sizes(count, seed)):
        gs = mix64(seed ^ i)
        g = chung_lu(n, 2.3, 20.0, math.sqrt(20.0 * n), gs)
        g.name = f"batch{i}_n{n}"
        out.append(g)
    return out


def workload_planted(n: int = 4_000_000, cliques: int = 200, size: int = 30) -> EdgeList:
    """Chung-Lu, exponent 2.0, mean 30, max weight sqrt(30 n), seed 5, plus
    `cliques` planted cliques of `size` uniform distinct nodes (seed 5)."""
    g = chung_lu(n, 2.0, 30.0, math.sqrt(30.0 * n), 5)
    ps, pd = planted_cliques(n, cliques, size, 5)
    out = EdgeList(n, np.concatenate([g.src, ps]), np.concatenate([g.dst, pd]),
                   f"chung_lu_n{n}_g2.0_mean30_planted{cliques}x{size}")
    return out
