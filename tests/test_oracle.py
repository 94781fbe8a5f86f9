"""Pins for the CPU oracle: closed forms, brute force, invariants and published
values.  None of these re-derive a count the way the oracle does (sorted-list
neighbourhood intersection over Gamma+ lists); each checks it against something
the mathematics or the paper fixes independently."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle as O
from graphgen import small as S
import graphgen as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def og(el):
    return O.OracleGraph.from_edgelist(el)


def edge_set(el):
    return {frozenset((int(a), int(b))) for a, b in zip(el.src, el.dst) if a != b}


def brute_cliques(n, edges, k):
    """All k-subsets of the nodes that are cliques (plain definition of q_k)."""
    adj = [set() for _ in range(n)]
    for e in edges:
        a, b = tuple(e)
        adj[a].add(b)
        adj[b].add(a)
    out = []
    for S_ in itertools.combinations(range(n), k):
        if all(b in adj[a] for a, b in itertools.combinations(S_, 2)):
            out.append(S_)
    return out, adj


def prec_min(S_, adj):
    """The smallest node of S in the paper's order: by degree, then by label."""
    return min(S_, key=lambda x: (len(adj[x]), x))


def elementary_symmetric(parts, k):
    """e_k(a_1..a_r): coefficient of x^k in prod (1 + a_i x)."""
    poly = [1]
    for a in parts:
        nxt = poly + [0]
        for i in range(len(poly)):
            nxt[i + 1] += poly[i] * a
        poly = nxt
    return poly[k] if k < len(poly) else 0


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 21, 34])
def test_complete_graph_binomial(n):
    g = og(S.complete(n))
    for k in range(1, 11):
        assert g.count(k) == math.comb(n, k), (n, k)


@pytest.mark.parametrize("parts", [[1, 2, 3, 4, 2], [5, 5, 5], [3, 1, 4, 1, 5, 9, 2], [7, 1], [2] * 9])
def test_complete_multipartite_elementary_symmetric(parts):
    g = og(S.complete_multipartite(parts))
    for k in range(1, 10):
        assert g.count(k) == elementary_symmetric(parts, k), (parts, k)


def test_turan_graph():
    # Turan T(13, 4): parts 4, 3, 3, 3
    g = og(S.turan(13, 4))
    for k in range(1, 6):
        assert g.count(k) == elementary_symmetric([4, 3, 3, 3], k)
    assert g.count(5) == 0


@pytest.mark.parametrize("el", [S.empty(10), S.star(12), S.cycle(4), S.cycle(9), S.path(7)],
                         ids=lambda e: e.name)
def test_triangle_free(el):
    assert og(el).count(3) == 0


def test_triangle_and_small_cases():
    assert og(S.cycle(3)).count(3) == 1
    g = og(S.empty(5))
    assert g.count(1) == 5 and g.count(2) == 0


def test_disjoint_union_adds():
    parts = [S.complete(6), S.complete_multipartite([2, 3, 4]), S.cycle(5), S.complete(9)]
    u = og(S.disjoint_union(*parts))
    for k in range(1, 8):
        assert u.count(k) == sum(og(p).count(k) for p in parts)


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_small_random(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(5, 17))
    p = float(rng.choice([0.3, 0.5, 0.7, 0.9]))
    el = S.random_graph(n, p, seed, dup_frac=0.3, loops=3)
    g = og(el)
    E = edge_set(el)
    assert g.m == len(E)
    for k in range(1, 8):
        cl, adj = brute_cliques(n, E, k) if k >= 1 else ([], None)
        assert g.count(k) == len(cl), (seed, k)
        if k >= 2:
            # per-root counts: each clique belongs to its smallest node in the order
            want = np.zeros(n, np.uint64)
            for S_ in cl:
                want[prec_min(S_, adj)] += 1
            assert np.array_equal(g.count_per_root(k), want), (seed, k)


def test_networkx_clique_census():
    nx = pytest.importorskip("networkx")
    for seed in range(4):
        el = S.random_graph(22, 0.55, 77 + seed)
        G_ = nx.Graph()
        G_.add_nodes_from(range(el.n))
        G_.add_edges_from(zip(el.src.tolist(), el.dst.tolist()))
        census = {}
        for c in nx.enumerate_all_cliques(G_):
            census[len(c)] = census.get(len(c), 0) + 1
        g = og(el)
        for k in range(1, 10):
            assert g.count(k) == census.get(k, 0), (seed, k)


def test_relabelling_invariance():
    el = S.random_graph(30, 0.4, 5)
    rng = np.random.default_rng(9)
    g0 = og(el)
    for t in range(3):
        g1 = og(S.relabel(el, rng.permutation(el.n)))
        for k in range(1, 7):
            assert g0.count(k) == g1.count(k)


# ------------------------------------------------------- order and orientation
def test_canonicalisation_set_semantics():
    el = S.random_graph(40, 0.2, 3, dup_frac=0.8, loops=10)
    g = og(el)
    E = edge_set(el)
    eu, ev = g.canon_edges()
    got = {frozenset((int(a), int(b))) for a, b in zip(eu, ev)}
    assert got == E and len(eu) == len(E)
    assert np.all(eu < ev)
    deg = g.degrees()
    want = np.zeros(el.n, np.int64)
    for e in E:
        for x in e:
            want[x] += 1
    assert np.array_equal(deg.astype(np.int64), want)
    assert int(deg.sum()) == 2 * g.m


@pytest.mark.parametrize("el", [S.random_graph(60, 0.3, 11, dup_frac=0.2, loops=4),
                                S.complete_multipartite([3, 1, 4, 1, 5]),
                                S.star(20)], ids=lambda e: e.name)
def test_orientation_invariants(el):
    g = og(el)
    E = edge_set(el)
    deg = g.degrees()
    hp, hn = g.high_csr()
    dplus = np.diff(hp.astype(np.int64))
    assert int(dplus.sum()) == g.m
    # Theorem I: |Gamma+(u)| <= 2 sqrt(m)
    assert dplus.max(initial=0) <= 2 * math.sqrt(max(g.m, 1))
    # every edge appears once, from its smaller endpoint in the (degree, label) order
    seen = set()
    for u in range(el.n):
        lst = [int(x) for x in hn[hp[u]:hp[u + 1]]]
        keys = [(int(deg[x]), x) for x in lst]
        assert keys == sorted(keys)
        for x in lst:
            assert (int(deg[u]), u) < (int(deg[x]), x)
            e = frozenset((u, x))
            assert e in E and e not in seen
            seen.add(e)
    assert seen == E
    # rank view: rank2id sorted by (degree, label); rows ascending and above the row
    r2i = g.rank2id()
    keys = [(int(deg[x]), int(x)) for x in r2i]
    assert keys == sorted(keys) and sorted(r2i.tolist()) == list(range(el.n))
    optr, ocol = g.rank_csr()
    rank = np.empty(el.n, np.int64)
    rank[r2i] = np.arange(el.n)
    for r in range(el.n):
        row = ocol[optr[r]:optr[r + 1]].astype(np.int64)
        assert np.all(np.diff(row) > 0) and np.all(row > r)
        u = int(r2i[r])
        assert sorted(row.tolist()) == sorted(int(rank[x]) for x in hn[hp[u]:hp[u + 1]])


def test_theorem_one_bound_power_law():
    el = G.chung_lu(20000, 2.1, 20.0, 2000.0, 17)
    g = og(el)
    assert g.max_outdeg() <= 2 * math.sqrt(g.m)


def test_id_out_of_range_rejected():
    with pytest.raises(O.OracleError) as e:
        O.OracleGraph(4, np.array([0, 5], np.uint32), np.array([1, 2], np.uint32))
    assert e.value.status == O.EINVAL


# ---------------------------------------------------------------- colour hash
def test_mix64_published_vectors():
    with open(os.path.join(GOLDEN, "splitmix64_state0.txt")) as f:
        want = [int(x) for x in f.read().split() if not x.startswith("#") and x.strip().isdigit()]
    gamma = 0x9E3779B97F4A7C15
    got = [O.mix64((i * gamma) % 2**64) for i in range(len(want))]
    assert len(want) == 4 and got == want


def test_colour_reduction_range_and_uniformity():
    for c in [1, 2, 3, 7, 8, 10]:
        cols = [O.color(O.hash_root(5, 17, x), c) for x in range(20000)]
        assert min(cols) >= 0 and max(cols) <= c - 1
        freq = np.bincount(cols, minlength=c) / len(cols)
        assert np.all(np.abs(freq - 1.0 / c) < 0.02)
    # the top 32 bits pick the colour: multiply-high
    assert O.color(0xFFFFFFFF00000000, 10) == 9 and O.color(0x00000000FFFFFFFF, 10) == 0


# ---------------------------------------------------------------- colour sampling
@pytest.mark.parametrize("scheme", [O.COLOR_PER_ROOT, O.COLOR_GLOBAL])
def test_colour_one_colour_is_exact(scheme):
    g = og(S.random_graph(40, 0.5, 21))
    for k in range(3, 7):
        assert g.count_colored(k, 1, 123, scheme) == g.count(k)


@pytest.mark.parametrize("seed", range(6))
def test_colour_bruteforce(seed):
    """k-subset form: a clique S with smallest node u survives the per-root colouring
    when every x in S minus u has the same colour col_u(x); it survives the global
    colouring when all of S shares one colour."""
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(8, 16))
    el = S.random_graph(n, 0.75, 40 + seed)
    g = og(el)
    E = edge_set(el)
    for c in [1, 2, 3]:
        hseed = int(rng.integers(0, 2**63))
        for k in range(3, 7):
            cl, adj = brute_cliques(n, E, k)
            per_root = glob = 0
            for S_ in cl:
                u = prec_min(S_, adj)
                if len({O.color(O.hash_root(hseed, u, x), c) for x in S_ if x != u}) == 1:
                    per_root += 1
                if len({O.color(O.hash_node(hseed, x), c) for x in S_}) == 1:
                    glob += 1
            assert g.count_colored(k, c, hseed, O.COLOR_PER_ROOT) == per_root, (seed, c, k)
            assert g.count_colored(k, c, hseed, O.COLOR_GLOBAL) == glob, (seed, c, k)


@pytest.mark.parametrize("scheme", [O.COLOR_PER_ROOT, O.COLOR_GLOBAL])
def test_colour_survival_probability(scheme):
    """Section 6: a k-clique survives the per-root colouring with probability
    c^-(k-2); under one global colouring it needs all k nodes alike, c^-(k-1)."""
    k, c, trials = 4, 3, 6000
    g = og(S.complete(k))
    hits = sum(g.count_colored(k, c, s, scheme) for s in range(trials))
    p = c ** -O.scale_exponent(k, scheme)
    sd = math.sqrt(trials * p * (1 - p))
    assert abs(hits - trials * p) < 5 * sd


@pytest.mark.parametrize("scheme", [O.COLOR_PER_ROOT, O.COLOR_GLOBAL])
def test_colour_estimator_unbiased(scheme):
    """E[raw * c^e] = q_k (Section 6 and Appendix B, colour-sampling analysis)."""
    el = S.random_graph(18, 0.7, 8)
    g = og(el)
    k, c, trials = 4, 2, 3000
    q = g.count(k)
    e = O.scale_exponent(k, scheme)
    est = np.array([g.count_colored(k, c, s, scheme) * c ** e for s in range(trials)], dtype=np.float64)
    se = est.std(ddof=1) / math.sqrt(trials)
    assert abs(est.mean() - q) < 5 * se + 1e-9, (est.mean(), q, se)


# ---------------------------------------------------------------- pair sampling
@pytest.mark.parametrize("el", [S.complete(9), S.random_graph(40, 0.5, 71), S.turan(24, 5),
                                S.complete_multipartite([3, 4, 5, 2])], ids=lambda e: e.name[:30])
def test_pair_sampling_p_one_is_exact(el):
    """p = 1 keeps every pair: the sampled local graphs are the G+(u) themselves, so
    the raw count is q_k (computed by the separate list-merge counter)."""
    g = og(el)
    for k in range(3, 7):
        assert g.count_pair_sampled(k, 1.0, 99) == g.count(k), k


def test_pair_hash_is_the_documented_composition():
    """The pair hash composes the SplitMix64 finaliser (pinned by its published
    vectors) as documented: H2 = mix64(mix64(seed ^ mix64(u << 32 | x)) ^ mix64(y));
    the keep rule (H2 >> 32) < floor(p 2^32) keeps a fraction p of the pairs."""
    rng = np.random.default_rng(7)
    M = 2**64 - 1
    for _ in range(200):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        u, x, y = (int(v) for v in rng.integers(0, 2**32, 3))
        h1 = O.mix64(seed ^ O.mix64(((u << 32) | x) & M))
        assert O.hash_root(seed, u, x) == h1
        assert O.hash_pair(seed, u, x, y) == O.mix64(h1 ^ O.mix64(y))
    for p in [0.1, 0.5, 0.9]:
        t = O.pair_threshold(p)
        kept = sum((O.hash_pair(3, 5, x, x + 1) >> 32) < t for x in range(20000)) / 20000
        assert abs(kept - p) < 0.02, (p, kept)


def test_node_hash_is_the_documented_composition():
    """The global colouring's node hash composes the SplitMix64 finaliser (pinned by
    its published vectors) as documented: H(seed, x) = mix64(seed ^ mix64(x)), with
    the id zero-extended to 64 bits and the colour taken by multiply-high."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        x = int(rng.integers(0, 2**32))
        h = O.hash_node(seed, x)
        assert h == O.mix64(seed ^ O.mix64(x))
        for c in (1, 2, 3, 8, 1000):
            assert O.color(h, c) == ((h >> 32) * c) >> 32
    # the node colour does not depend on anything but (seed, x): two seeds differ
    assert sum(O.hash_node(1, x) == O.hash_node(2, x) for x in range(1000)) == 0


@pytest.mark.parametrize("seed", range(4))
def test_pair_sampling_bruteforce(seed):
    """k-subset form (Section 6, plain pair sampling): a clique S with smallest node
    u survives when every pair {x, y} of S minus u, x before y in the order, is kept:
    (hash_pair(seed, u, x, y) >> 32) < floor(p 2^32)."""
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(9, 15))
    el = S.random_graph(n, 0.8, 90 + seed)
    g = og(el)
    E = edge_set(el)
    for p in [0.3, 0.5, 0.85]:
        t = O.pair_threshold(p)
        hseed = int(rng.integers(0, 2**63))
        for k in range(3, 7):
            cl, adj = brute_cliques(n, E, k)
            order = lambda x: (len(adj[x]), x)
            want = 0
            for S_ in cl:
                u = prec_min(S_, adj)
                rest = sorted((x for x in S_ if x != u), key=order)
                if all((O.hash_pair(hseed, u, x, y) >> 32) < t for x, y in itertools.combinations(rest, 2)):
                    want += 1
            assert g.count_pair_sampled(k, p, hseed) == want, (seed, p, k)


def test_pair_sampling_estimator_unbiased():
    """E[raw / p^C(k-1,2)] = q_k (Section 6: each k-clique survives with probability
    p^((k-1)(k-2)/2), its C(k-1, 2) pairs below the minimum node kept independently)."""
    el = S.random_graph(16, 0.75, 12)
    g = og(el)
    k, p, trials = 4, 0.6, 3000
    q = g.count(k)
    keep = O.pair_threshold(p) / 2**32
    scale = keep ** -math.comb(k - 1, 2)
    est = np.array([g.count_pair_sampled(k, p, s) * scale for s in range(trials)], dtype=np.float64)
    se = est.std(ddof=1) / math.sqrt(trials)
    assert abs(est.mean() - q) < 5 * se + 1e-9, (est.mean(), q, se)


# ---------------------------------------------------------------- work labels
@pytest.mark.parametrize("seed", range(4))
def test_work_counts_cliques_of_high_neighbourhood(seed):
    """Intersections of an unpruned count of (k-1)-cliques in G+(u): one per l-clique
    of G+(u), l = 1..k-2; the word weight charges the 64-bit words above the
    clique's last node in a bitmap row of G+(u)."""
    el = S.random_graph(14, 0.8, 60 + seed)
    g = og(el)
    E = edge_set(el)
    _, adj = brute_cliques(el.n, E, 1)
    hp, hn = g.high_csr()
    for u in range(el.n):
        hi = [int(x) for x in hn[hp[u]:hp[u + 1]]]
        d = len(hi)
        for k in range(3, 8):
            inter = words = 0
            for l in range(1, k - 1):
                for S_ in itertools.combinations(range(d), l):
                    if all(hi[b] in adj[hi[a]] for a, b in itertools.combinations(S_, 2)):
                        inter += 1
                        i = S_[-1]
                        words += ((d - 1) // 64 - (i + 1) // 64 + 1) if i + 1 <= d - 1 else 0
            assert g.work_root(u, k) == (inter, words), (seed, u, k)


def test_work_wide_root_words():
    # a root with 150 high neighbours that form a clique: bitmap rows span 3 words
    el = S.complete(151)
    g = og(el)
    hp, _ = g.high_csr()
    u = int(np.argmax(np.diff(hp.astype(np.int64))))
    d = 150
    inter, words = g.work_root(u, 3)
    assert inter == d
    assert words == sum(((d - 1) // 64 - (i + 1) // 64 + 1) for i in range(d - 1))


# ------------------------------------------------- per-node membership counts
# Section 3 (remark after the round-3 reducers): summing each sub-problem's
# per-node report over all roots gives the k-cliques that contain each node.

@pytest.mark.parametrize("n", [1, 2, 5, 9, 14])
def test_per_node_complete_graph(n):
    g = og(S.complete(n))
    for k in range(1, min(n, 7) + 1):
        np.testing.assert_array_equal(g.count_per_node(k), np.full(n, math.comb(n - 1, k - 1), np.uint64))


@pytest.mark.parametrize("parts", [[1, 2, 3, 4, 2], [5, 5, 5], [3, 1, 4, 1, 5, 9, 2]])
def test_per_node_multipartite_closed_form(parts):
    # a node of block b lies in the k-cliques that take one node from each of k - 1
    # other blocks: e_{k-1} of the other blocks' sizes
    g = og(S.complete_multipartite(parts))
    block = [b for b, s in enumerate(parts) for _ in range(s)]
    for k in range(1, len(parts) + 2):
        want = [elementary_symmetric(parts[:b] + parts[b + 1:], k - 1) for b in block]
        np.testing.assert_array_equal(g.count_per_node(k), np.array(want, np.uint64))


@pytest.mark.parametrize("seed", range(8))
def test_per_node_bruteforce(seed):
    n = 9 + seed
    el = S.random_graph(n, 0.55, 300 + seed, dup_frac=0.1, loops=2)
    g = og(el)
    for k in range(1, 7):
        cl, _ = brute_cliques(n, edge_set(el), k)
        want = np.zeros(n, np.uint64)
        for c in cl:
            for v in c:
                want[v] += 1
        np.testing.assert_array_equal(g.count_per_node(k), want, err_msg=f"k={k}")


@pytest.mark.parametrize("el", [S.random_graph(120, 0.15, 5), S.turan(40, 6),
                                S.planted_small(150, 0.03, [list(range(0, 12)), list(range(40, 49))], 7),
                                S.hub_bipartite(5, 80, 0.2, 3)], ids=lambda e: e.name)
def test_per_node_sums_and_definition(el):
    g = og(el)
    deg = g.degrees()
    for k in range(1, 7):
        c = g.count_per_node(k)
        # every k-clique has k nodes
        assert int(c.sum()) == k * g.count(k), k
        if k == 2:
            np.testing.assert_array_equal(c, deg.astype(np.uint64))
        # the route through the sub-problems agrees with the plain definition
        for v in range(0, el.n, max(1, el.n // 17)):
            assert int(c[v]) == g.count_node(v, k), (k, v)


def test_per_node_disjoint_union():
    a, b = S.complete(6), S.turan(12, 3)
    g = og(S.disjoint_union(a, b))
    c = g.count_per_node(3)
    np.testing.assert_array_equal(c[:6], og(a).count_per_node(3))
    np.testing.assert_array_equal(c[6:], og(b).count_per_node(3))
