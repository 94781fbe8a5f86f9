"""GPU parity of the per-node clique-membership counts (kc_count_per_node, Section 3:
the k-cliques that contain each node, summed over the roots' sub-problems) against
the oracle, element by element and bit-exact.  The cases reach every path of the
kernel: one-word local graphs (out-degree <= 64), wide roots whose first-level
candidate sets are compacted at once, wide roots whose candidate sets are split over
several levels, and roots whose bitmaps are larger than the count kernels' LDS arena;
closed forms where the oracle would take too long; full-size workloads on sampled
nodes (recomputed one by one from the plain definition) and on the sum k * q_k."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import graphgen as G
from graphgen import small as S
from paper_1403_0734_amd import kc as K

from gpu_util import announce, device_graph

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "counts.json")))


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    K.load()


def per_node(h, n, k):
    import torch
    c = torch.full((max(n, 1),), -1, dtype=torch.int64, device="cuda:0")
    K.kc_count_per_node(h, k, c.data_ptr())
    torch.cuda.synchronize()
    return c.cpu().numpy().view(np.uint64)[:n]


def oracle_ks(og, budget=1e7):
    """Clique sizes the oracle lists quickly (it visits every k-clique k times)."""
    out = []
    for k in range(1, K.KC_KMAX + 1):
        if k >= 3 and og.count(k) > budget:
            break
        out.append(k)
    return out


CASES = [
    S.complete(5), S.complete(66), S.complete(130), S.complete_multipartite([3, 1, 4, 1, 5, 9, 2, 6]),
    S.turan(40, 7), S.cycle(9), S.star(70), S.empty(7), S.path(12),
    S.random_graph(60, 0.5, 1, dup_frac=0.3, loops=5), S.random_graph(150, 0.6, 2),
    S.random_graph(300, 0.3, 3, dup_frac=0.1, loops=2),
    S.planted_small(400, 0.02, [list(range(0, 60, 2)), list(range(100, 190, 3)), list(range(5, 395, 5))], 4),
    S.disjoint_union(S.complete(20), S.complete_multipartite([4, 4, 4, 4]), S.random_graph(90, 0.4, 5)),
    # wide roots: every node of A keeps B (300 / 600 nodes) as its high neighbours
    S.hub_bipartite(290, 300, 0.05, 1), S.hub_bipartite(580, 600, 0.04, 2),
    G.chung_lu(20000, 2.1, 15.0, 800.0, 9),
]


@pytest.mark.parametrize("el", CASES, ids=lambda e: e.name[:40])
def test_per_node_matches_oracle(el):
    og = O.OracleGraph.from_edgelist(el)
    h = device_graph(el)
    try:
        for k in oracle_ks(og):
            announce(f"per-node {el.name[:40]} k={k}")
            got = per_node(h, el.n, k)
            want = og.count_per_node(k)
            np.testing.assert_array_equal(got, want, err_msg=f"{el.name} k={k}")
            if k >= 3:
                assert int(got.sum(dtype=np.uint64)) == k * K.kc_count(h, k)
    finally:
        K.kc_graph_destroy(h)


@pytest.mark.parametrize("n,ks", [(200, (3, 4, 5)), (1500, (3,))])
def test_per_node_complete_closed_form(n, ks):
    # K_n: every node lies in C(n-1, k-1) k-cliques; with n = 200 the candidate sets
    # of the first three levels hold more than 64 nodes, so the wide levels descend
    h = device_graph(S.complete(n))
    try:
        for k in ks:
            announce(f"per-node K{n} k={k}")
            np.testing.assert_array_equal(per_node(h, n, k), np.full(n, math.comb(n - 1, k - 1), np.uint64))
    finally:
        K.kc_graph_destroy(h)


def _esym(parts, k):
    poly = [1]
    for a in parts:
        nxt = poly + [0]
        for i in range(len(poly)):
            nxt[i + 1] += poly[i] * a
        poly = nxt
    return poly[k] if k < len(poly) else 0


@pytest.mark.parametrize("parts", [[80] * 5, [150, 90, 60, 30, 7, 1]])
def test_per_node_multipartite_closed_form(parts):
    # complete multipartite: a node of block b is in e_{k-1}(sizes of the other blocks)
    el = S.complete_multipartite(parts)
    block = np.repeat(np.arange(len(parts)), parts)
    h = device_graph(el)
    try:
        for k in range(3, 6):
            announce(f"per-node {el.name} k={k}")
            want = np.array([_esym(parts[:b] + parts[b + 1:], k - 1) for b in range(len(parts))], np.uint64)
            np.testing.assert_array_equal(per_node(h, el.n, k), want[block])
    finally:
        K.kc_graph_destroy(h)


def test_per_node_tuned_wave_limit():
    # roots above a lowered one-wave limit keep one-word packed bitmaps instead of rows
    el = S.planted_small(300, 0.05, [list(range(0, 40)), list(range(100, 130))], 8)
    og = O.OracleGraph.from_edgelist(el)
    K.kc_set_tuning(wave_dmax=24)
    try:
        h = device_graph(el)
        try:
            for k in (3, 5, 7):
                np.testing.assert_array_equal(per_node(h, el.n, k), og.count_per_node(k))
        finally:
            K.kc_graph_destroy(h)
    finally:
        K.kc_set_tuning(defaults=True)


def test_per_node_errors():
    el = S.complete(6)
    h = device_graph(el, orient=False)
    import torch
    c = torch.zeros(6, dtype=torch.int64, device="cuda:0")
    try:
        with pytest.raises(K.KcError) as e:
            K.kc_count_per_node(h, 3, c.data_ptr())
        assert e.value.status == K.KC_ESTATE
        K.kc_orient(h)
        for bad in (0, K.KC_KMAX + 1):
            with pytest.raises(K.KcError) as e:
                K.kc_count_per_node(h, bad, c.data_ptr())
            assert e.value.status == K.KC_EINVAL
        with pytest.raises(K.KcError) as e:
            K.kc_count_per_node(h, 3, None)
        assert e.value.status == K.KC_EINVAL
        # a k larger than any clique gives zeros; k = 1 gives ones
        np.testing.assert_array_equal(per_node(h, 6, 7), np.zeros(6, np.uint64))
        np.testing.assert_array_equal(per_node(h, 6, 1), np.ones(6, np.uint64))
    finally:
        K.kc_graph_destroy(h)


def _fullsize(name, make, ks, count, ranks, planted=None):
    """Per-node counts of a benchmark workload: the sum against k * q_k, and the
    counts of sampled nodes against the oracle's plain definition (the cliques in
    the node's neighbourhood): random nodes, nodes at the given positions of the
    degree ranking (per k, as deep into the heavy end as the oracle finishes in
    seconds: the top planted-4M nodes take it about two minutes each at k = 8), and
    members of the first planted clique."""
    gold = GOLD[name]
    announce(f"{name}: generating")
    el = make()
    assert el.digest() == gold["digest"], "generator output changed"
    h = device_graph(el)
    og = O.OracleGraph.from_edgelist(el)
    order = np.argsort(-og.degrees().astype(np.int64), kind="stable")
    rng = np.random.default_rng(11)
    base = [rng.choice(el.n, size=count, replace=False)]
    if planted is not None:
        ps, pd = planted
        base.append(np.unique(np.concatenate([ps[:435], pd[:435]]))[:6])
    try:
        for k in ks:
            announce(f"{name}: per-node k={k}")
            c = per_node(h, el.n, k)
            q = gold["q"][str(k)] if str(k) in gold["q"] else K.kc_count(h, k)
            assert int(c.sum(dtype=np.uint64)) == k * q
            nodes = np.unique(np.concatenate(base + [order[np.asarray(ranks[k], np.int64)]]))
            for v in nodes:
                assert int(c[v]) == og.count_node(int(v), k), (name, k, int(v))
    finally:
        K.kc_graph_destroy(h)


def test_per_node_chung_lu_1m():
    _fullsize("chung_lu_1m", G.workload_chung_lu_1m, (3, 5), 40, {3: [0, 30, 300], 5: [0, 30, 300, 3000]})


def test_per_node_planted_4m():
    # a planted clique's members lie in C(29, k - 1) cliques of it at least
    _fullsize("planted_4m", G.workload_planted, (5, 8), 40, {5: [1000, 3000], 8: [3000]},
              planted=G.planted_cliques(4_000_000, 200, 30, 5))
