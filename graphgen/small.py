"""Small structured and random test graphs (raw edge lists as numpy uint32).

Pure input construction: no degrees, orders or counts are computed here.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import EdgeList


def _el(n, pairs, name):
    if pairs:
        a = np.array(pairs, dtype=np.uint32)
        return EdgeList(n, a[:, 0], a[:, 1], name)
    return EdgeList(n, np.zeros(0, np.uint32), np.zeros(0, np.uint32), name)


def complete(n: int, offset: int = 0, total_n: int | None = None) -> EdgeList:
    pairs = [(offset + i, offset + j) for i in range(n) for j in range(i + 1, n)]
    return _el(total_n if total_n is not None else offset + n, pairs, f"K{n}")


def complete_multipartite(parts) -> EdgeList:
    """Nodes split into consecutive blocks of the given sizes; every pair of nodes
    in different blocks is an edge."""
    block = []
    for b, s in enumerate(parts):
        block += [b] * s
    n = len(block)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if block[i] != block[j]]
    return _el(n, pairs, "K" + "_".join(map(str, parts)))


def turan(n: int, r: int) -> EdgeList:
    parts = [n // r + (1 if i < n % r else 0) for i in range(r)]
    g = complete_multipartite(parts)
    g.name = f"T({n},{r})"
    return g


def cycle(n: int) -> EdgeList:
    return _el(n, [(i, (i + 1) % n) for i in range(n)], f"C{n}")


def star(n: int) -> EdgeList:
    return _el(n, [(0, i) for i in range(1, n)], f"S{n}")


def path(n: int) -> EdgeList:
    return _el(n, [(i, i + 1) for i in range(n - 1)], f"P{n}")


def empty(n: int) -> EdgeList:
    return _el(n, [], f"E{n}")


def disjoint_union(*graphs: EdgeList) -> EdgeList:
    src, dst, off = [], [], 0
    for g in graphs:
        src.append(g.src.astype(np.uint64) + off)
        dst.append(g.dst.astype(np.uint64) + off)
        off += g.n
    s = np.concatenate(src) if src else np.zeros(0)
    d = np.concatenate(dst) if dst else np.zeros(0)
    return EdgeList(off, s.astype(np.uint32), d.astype(np.uint32),
                    "+".join(g.name for g in graphs))


def relabel(g: EdgeList, perm: np.ndarray) -> EdgeList:
    perm = np.asarray(perm, dtype=np.uint32)
    return EdgeList(g.n, perm[g.src], perm[g.dst], g.name + "/relabelled")


def random_graph(n: int, p: float, seed: int, dup_frac: float = 0.0, loops: int = 0) -> EdgeList:
    """G(n, p) from numpy's PCG64 stream, optionally with repeated pairs (in either
    direction) and self-loops mixed in, to exercise canonicalisation."""
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i, j in itertools.combinations(range(n), 2) if rng.random() < p]
    extra = []
    if pairs and dup_frac > 0:
        for t in rng.choice(len(pairs), size=max(1, int(dup_frac * len(pairs))), replace=True):
            a, b = pairs[int(t)]
            extra.append((b, a) if rng.random() < 0.5 else (a, b))
    for _ in range(loops):
        x = int(rng.integers(0, n))
        extra.append((x, x))
    allp = pairs + extra
    order = rng.permutation(len(allp)) if allp else []
    return _el(n, [allp[int(i)] for i in order], f"G({n},{p},seed={seed})")


def planted_small(n: int, p: float, cliques, seed: int) -> EdgeList:
    """Sparse G(n, p) plus cliques on the given node lists."""
    g = random_graph(n, p, seed)
    pairs = list(zip(g.src.tolist(), g.dst.tolist()))
    for c in cliques:
        pairs += [(a, b) for a, b in itertools.combinations(sorted(c), 2)]
    return _el(n, pairs, f"planted({n},{p},{len(cliques)})")


def hub_bipartite(na: int, nb: int, p: float, seed: int) -> EdgeList:
    """Every node of A = [0, na) joined to every node of B = [na, na + nb), plus
    G(nb, p) inside B (numpy PCG64 stream).  A node of A has degree nb, one of B about
    na + p (nb - 1); when that is larger (na > nb (1 - p) roughly), every node of A
    keeps all of B as its high neighbours: high-neighbourhoods of nb nodes."""
    rng = np.random.default_rng(seed)
    a = np.repeat(np.arange(na, dtype=np.uint64), nb)
    b = np.tile(np.arange(na, na + nb, dtype=np.uint64), na)
    iu, ju = np.triu_indices(nb, 1)
    keep = rng.random(iu.shape[0]) < p
    src = np.concatenate([a, iu[keep].astype(np.uint64) + na]).astype(np.uint32)
    dst = np.concatenate([b, ju[keep].astype(np.uint64) + na]).astype(np.uint32)
    return EdgeList(na + nb, src, dst, f"hub({na},{nb},{p},seed={seed})")
