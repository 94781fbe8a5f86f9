"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by
element and bit-exact (all results are integers).  Sizes span several tiles and
every tier: wave (out-degree <= 64), workgroup (LDS bitmap) and scratch (global
bitmap), with ragged tails and the degenerate cases."""
import math

import numpy as np
import pytest

import oracle as O
import graphgen as G
from graphgen import small as S
from paper_1403_0734_amd import kc as K

from gpu_util import announce, csr, device_graph, oriented, per_root

pytestmark = pytest.mark.gpu

SMALL = [
    S.complete(5), S.complete(66), S.complete(130), S.complete_multipartite([3, 1, 4, 1, 5, 9, 2, 6]),
    S.turan(40, 7), S.cycle(9), S.star(70), S.empty(7), S.path(12),
    S.random_graph(60, 0.5, 1, dup_frac=0.3, loops=5),
    S.random_graph(150, 0.6, 2), S.random_graph(300, 0.3, 3, dup_frac=0.1, loops=2),
    S.planted_small(400, 0.02, [list(range(0, 60, 2)), list(range(100, 190, 3)), list(range(5, 395, 5))], 4),
    S.disjoint_union(S.complete(20), S.complete_multipartite([4, 4, 4, 4]), S.random_graph(90, 0.4, 5)),
]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    K.load()


def _close(h):
    K.kc_graph_destroy(h)


def bounded_ks(og, lo=1, hi=K.KC_KMAX, budget=2e7):
    """Clique sizes whose enumeration stays cheap: stop after the first k whose
    (k-1)-clique count exceeds the budget (both sides enumerate them)."""
    out = []
    for k in range(lo, hi + 1):
        if k >= 4 and og.count(k - 1) > budget:
            break
        out.append(k)
    return out


MULTI_TILE = [G.chung_lu(50000, 2.1, 20.0, 1500.0, 5), S.random_graph(3000, 0.05, 6, dup_frac=0.2, loops=30)]


# a hub of degree 19999 with the smallest id (every edge keyed by it) and with the
# largest (every edge keyed by a leaf)
HUBS = [S.disjoint_union(S.star(20000), S.random_graph(200, 0.1, 9)),
        S.relabel(S.star(20000), np.arange(20000)[::-1].copy())]


@pytest.mark.parametrize("el", SMALL + MULTI_TILE + HUBS, ids=lambda e: e.name[:40])
def test_csr_and_orientation_match_oracle(el):
    announce(f"csr/orientation {el.name}")
    og = O.OracleGraph.from_edgelist(el)
    h = device_graph(el)
    n, m, dmax = K.kc_graph_info(h)
    assert (n, m) == (og.n, og.m)
    assert dmax == og.max_outdeg()
    # symmetric CSR of the simple graph and degrees
    rp, col, deg = csr(h, n, m)
    eu, ev = og.canon_edges()
    pairs = np.concatenate([np.stack([eu, ev], 1), np.stack([ev, eu], 1)]).astype(np.uint64)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    pairs = pairs[order]
    want_rp = np.zeros(n + 1, np.uint64)
    np.add.at(want_rp, pairs[:, 0].astype(np.int64) + 1, 1)
    want_rp = np.cumsum(want_rp).astype(np.uint64)
    assert np.array_equal(rp, want_rp)
    assert np.array_equal(col, pairs[:, 1].astype(np.uint32))
    assert np.array_equal(deg, og.degrees())
    # oriented CSR in rank space, byte for byte
    optr, ocol, r2i = oriented(h, n, m)
    w_optr, w_ocol = og.rank_csr()
    assert np.array_equal(r2i, og.rank2id())
    assert np.array_equal(optr, w_optr)
    assert np.array_equal(ocol, w_ocol)
    _close(h)


@pytest.mark.parametrize("el", SMALL, ids=lambda e: e.name[:40])
def test_exact_counts_small(el):
    og = O.OracleGraph.from_edgelist(el)
    h = device_graph(el)
    for k in bounded_ks(og):
        announce(f"count {el.name} k={k}")
        assert K.kc_count(h, k) == og.count(k), (el.name, k)
    _close(h)


@pytest.mark.parametrize("el", SMALL[:9] + SMALL[10:13], ids=lambda e: e.name[:40])
def test_per_root_counts_and_work(el):
    og = O.OracleGraph.from_edgelist(el)
    h = device_graph(el)
    for k in [k for k in bounded_ks(og, 3, 7) if k in (3, 4, 5, 7)]:
        announce(f"per-root {el.name} k={k}")
        c, w = per_root(h, el.n, k, with_work=True)
        assert np.array_equal(c, og.count_per_root(k)), (el.name, k)
        inter, _ = og.work_per_root(k)
        assert np.array_equal(w, inter), (el.name, k)
    _close(h)


def test_tier_boundaries_complete_graphs():
    """K_n has out-degrees 0..n-1, so one graph crosses every tier threshold; the
    closed form C(n, k) is the reference (no oracle run needed at this size)."""
    for n, ks in [(40, range(3, 11)), (63, range(3, 7)), (64, range(3, 7)), (65, range(3, 7)),
                  (129, range(3, 6)), (700, [3, 4]), (1300, [3, 4])]:
        h = device_graph(S.complete(n))
        for k in ks:
            announce(f"K{n} k={k}")
            assert K.kc_count(h, k) == math.comb(n, k), (n, k)
        _close(h)


@pytest.mark.parametrize("level2", ["1", "2"])
def test_wide_search_closed_forms(monkeypatch, level2):
    """First-level candidate sets above 128 nodes (the wide depth-first search of the
    workgroup tier, from k = 5): K_400, K_300 and K_260 against C(n, k) (sets that
    still need three nodes are counted lane-parallel at the first level at k = 5, one
    and two levels down at k = 6 and 7), and a complete
    multipartite graph against the elementary symmetric polynomial of its parts; with
    two-level items where the estimate asks for them (1) and for every wide node (2)."""
    monkeypatch.setenv("KC_LEVEL2", level2)
    for n, ks in [(400, [5]), (300, [6]), (260, [7])]:
        h = device_graph(S.complete(n))
        for k in ks:
            announce(f"K{n} k={k} (wide search)")
            assert K.kc_count(h, k) == math.comb(n, k), (n, k)
        _close(h)
    parts = [200, 150, 300, 90, 310]
    h = device_graph(S.complete_multipartite(parts))
    announce("multipartite k=5 (wide search)")
    assert K.kc_count(h, 5) == math.prod(parts)
    _close(h)


@pytest.mark.parametrize("level2", ["1", "0", "2"])
def test_wide_search_dense_random(monkeypatch, level2):
    """A dense G(500, 0.6): out-degrees up to about 275, first-level candidate sets of
    about 165 nodes; totals and per-root counts at k = 5 against the oracle, with the
    heaviest first-level nodes split into two-level items (Section 7) where the estimate
    asks for them (1), never (0), and for every wide node (2)."""
    monkeypatch.setenv("KC_LEVEL2", level2)
    el = S.random_graph(500, 0.6, 8)
    og = O.OracleGraph.from_edgelist(el)
    h = device_graph(el)
    announce(f"G(500, 0.6) k=5 level2={level2}")
    assert K.kc_count(h, 5) == og.count(5)
    c, _ = per_root(h, el.n, 5)
    assert np.array_equal(c, og.count_per_root(5))
    for scheme in (K.KC_COLOR_PER_ROOT, K.KC_COLOR_GLOBAL):
        e = K.kc_count_colored(h, 5, 2, 3, scheme)
        assert e.raw == og.count_colored(5, 2, 3, scheme), scheme
    e = K.kc_count_pair_sampled(h, 5, 0.5, 4)
    assert e.raw == og.count_pair_sampled(5, 0.5, 4)
    _close(h)


@pytest.fixture
def wg_cap():
    """Lowers the workgroup tier's out-degree cap (the wg_dmax tunable) for one test,
    so that roots above it take the scratch tier (bitmaps in global memory)."""
    def set_cap(cap):
        K.kc_set_tuning(wg_dmax=cap)
    yield set_cap
    K.kc_set_tuning(defaults=True)


SCRATCH_GRAPHS = [SMALL[2], SMALL[10], SMALL[11], SMALL[12], MULTI_TILE[0]]


@pytest.mark.parametrize("cache", ["1", "0"])
@pytest.mark.parametrize("cap", [64, 72])
def test_scratch_tier_under_lowered_cap(monkeypatch, wg_cap, cap, cache):
    """The scratch tier (G+(u) bitmap in a global-memory slice per block) on ordinary
    graphs: with the cap at 64 every root above the one-wave tier takes it, at 72 the
    workgroup and scratch tiers share the roots.  Staged into the cache and counted
    from it, or staged per call; exact totals k = 3..8, per-root counts, both
    colourings and (cached) pair sampling against the oracle."""
    monkeypatch.setenv("KC_STAGE_CACHE", cache)
    wg_cap(cap)
    for el in SCRATCH_GRAPHS:
        og = O.OracleGraph.from_edgelist(el)
        h = device_graph(el)
        ks = bounded_ks(og, 3, 8, budget=5e6)
        for k in ks:
            announce(f"scratch cap={cap} cache={cache} {el.name} k={k}")
            assert K.kc_count(h, k) == og.count(k), (el.name, k)
        for scheme in (K.KC_COLOR_PER_ROOT, K.KC_COLOR_GLOBAL):
            for k in ks[:4]:
                e = K.kc_count_colored(h, k, 3, 77, scheme)
                assert e.raw == og.count_colored(k, 3, 77, scheme), (el.name, k, scheme)
        for k in sorted({ks[-1], min(5, ks[-1])}):
            c, _ = per_root(h, el.n, k)
            assert np.array_equal(c, og.count_per_root(k)), (el.name, k)
        if cache == "1":
            for k in ks[:3]:
                e = K.kc_count_pair_sampled(h, k, 0.5, 9)
                assert e.raw == og.count_pair_sampled(k, 0.5, 9), (el.name, k)
        _close(h)


@pytest.mark.parametrize("cache", ["1", "0"])
def test_scratch_tier_natural(monkeypatch, cache):
    """Out-degrees above what LDS holds (about 1280 to 1344 nodes, by k) with the
    default tunables.  K_1400 against C(n, k); a hub graph (every node of A joined to
    every node of B, |A| = 1400, |B| = 1401, G(1401, 0.05) inside B) whose 1400 roots
    each keep 1401 high neighbours, against the oracle: exact k = 3..6, per-root
    counts, both colourings and pair sampling."""
    monkeypatch.setenv("KC_STAGE_CACHE", cache)
    h = device_graph(S.complete(1400))
    assert K.kc_graph_info(h)[2] == 1399
    for k in (3, 4):
        announce(f"K1400 k={k} cache={cache}")
        assert K.kc_count(h, k) == math.comb(1400, k)
    _close(h)
    el = S.hub_bipartite(1400, 1401, 0.05, 3)
    og = O.OracleGraph.from_edgelist(el)
    h = device_graph(el)
    assert K.kc_graph_info(h)[2] == og.max_outdeg() == 1401
    for k in range(3, 7):
        announce(f"hub k={k} cache={cache}")
        assert K.kc_count(h, k) == og.count(k), k
    for k in (4, 6):
        c, _ = per_root(h, el.n, k)
        assert np.array_equal(c, og.count_per_root(k)), k
    for scheme in (K.KC_COLOR_PER_ROOT, K.KC_COLOR_GLOBAL):
        e = K.kc_count_colored(h, 5, 2, 41, scheme)
        assert e.raw == og.count_colored(5, 2, 41, scheme), scheme
    if cache == "1":
        e = K.kc_count_pair_sampled(h, 4, 0.5, 13)
        assert e.raw == og.count_pair_sampled(4, 0.5, 13)
    _close(h)


def test_complete_multipartite_large():
    parts = [200, 150, 300, 90, 310]  # wide roots on every tier; e_4 ~ 1e10 cliques
    h = device_graph(S.complete_multipartite(parts))
    poly = [1]
    for a in parts:
        nxt = poly + [0]
        for i in range(len(poly)):
            nxt[i + 1] += poly[i] * a
        poly = nxt
    for k in range(3, 5):
        announce(f"multipartite k={k}")
        assert K.kc_count(h, k) == poly[k]
    _close(h)


@pytest.mark.parametrize("scheme", [K.KC_COLOR_PER_ROOT, K.KC_COLOR_GLOBAL])
def test_colour_raw_counts_match_oracle(scheme):
    for el in [SMALL[1], SMALL[2], SMALL[10], SMALL[11], SMALL[12]]:
        og = O.OracleGraph.from_edgelist(el)
        h = device_graph(el)
        for k in bounded_ks(og, 3, 6, budget=5e6):
            for c in [1, 2, 3, 8]:
                for seed in [11, 2**63 + 5]:
                    announce(f"colour {el.name} k={k} c={c} scheme={scheme}")
                    e = K.kc_count_colored(h, k, c, seed, scheme)
                    raw = og.count_colored(k, c, seed, scheme)
                    assert e.raw == raw, (el.name, k, c, seed, scheme)
                    exp = k - 2 if scheme == K.KC_COLOR_PER_ROOT else k - 1
                    assert e.scale_exponent == exp
                    assert e.estimate == float(raw * c ** exp)
                    assert bool(e.estimate_fits_u64) == (raw * c ** exp < 2**64)
                    if e.estimate_fits_u64:
                        assert e.estimate_u64 == raw * c ** exp
        _close(h)


@pytest.mark.parametrize("cache", ["1", "0"])
def test_staged_cache_and_per_call_staging(monkeypatch, cache):
    """Counts from the handle's staged G+(u) cache (the default) and with staging on
    every call: exact totals, per-root counts and both colourings, every tier."""
    monkeypatch.setenv("KC_STAGE_CACHE", cache)
    for el in [SMALL[2], SMALL[11], SMALL[12], MULTI_TILE[0]]:
        og = O.OracleGraph.from_edgelist(el)
        h = device_graph(el)
        ks = bounded_ks(og, 3, 7, budget=5e6)
        for k in ks:
            announce(f"stage cache={cache} {el.name} k={k}")
            assert K.kc_count(h, k) == og.count(k), (el.name, k)
        for scheme in (K.KC_COLOR_PER_ROOT, K.KC_COLOR_GLOBAL):
            for k in ks[:3]:
                e = K.kc_count_colored(h, k, 3, 77, scheme)
                assert e.raw == og.count_colored(k, 3, 77, scheme), (el.name, k, scheme)
        c, _ = per_root(h, el.n, ks[-1])
        assert np.array_equal(c, og.count_per_root(ks[-1]))
        _close(h)


ITEM_MODES = {
    "edge-ordered items": {},
    "degree split": {"KC_WORK_ORDER": "0"},
    "degree split, per-call staging": {"KC_STAGE_CACHE": "0", "KC_DEGREE_SPLIT": "5"},
    "whole roots": {"KC_WORK_ORDER": "0", "KC_DEGREE_SPLIT": "0"},
    "two lists split at out-degree 96": {"KC_WG_DSPLIT": "96"},
    "two lists split at out-degree 100, per-call staging": {"KC_WG_DSPLIT": "100", "KC_STAGE_CACHE": "0"},
}


@pytest.mark.parametrize("mode", sorted(ITEM_MODES))
def test_workgroup_items(monkeypatch, mode):
    """The workgroup tier from k = 5 on, as whole roots, split by out-degree, or
    ordered and split by the edges of G+(u) (padded item list): exact totals,
    per-root counts (split roots add their parts) and colourings."""
    for key, val in ITEM_MODES[mode].items():
        monkeypatch.setenv(key, val)
    for el in [SMALL[2], SMALL[12], MULTI_TILE[0]]:
        og = O.OracleGraph.from_edgelist(el)
        h = device_graph(el)
        ks = [k for k in bounded_ks(og, 3, 8, budget=5e6) if k >= 5]
        for k in ks:
            announce(f"items {mode} {el.name} k={k}")
            assert K.kc_count(h, k) == og.count(k), (el.name, k)
        if ks:
            k = ks[0]
            c, _ = per_root(h, el.n, k)
            assert np.array_equal(c, og.count_per_root(k)), (el.name, k)
            for scheme in (K.KC_COLOR_PER_ROOT, K.KC_COLOR_GLOBAL):
                e = K.kc_count_colored(h, k, 2, 5, scheme)
                assert e.raw == og.count_colored(k, 2, 5, scheme), (el.name, k, scheme)
        _close(h)


@pytest.mark.parametrize("dsplit", [None, "0", "300", "850"])
def test_workgroup_split_by_outdegree(monkeypatch, dsplit):
    """Roots of out-degree 900 beside roots below 100 in the workgroup tier: at k >= 5
    the default rule gives the large roots items of their own (one large arena per
    block, few blocks per CU) beside the small roots' (small arena, many blocks),
    launched side by side; forced split points and one list give the same counts."""
    if dsplit is not None:
        monkeypatch.setenv("KC_WG_DSPLIT", dsplit)
    el = S.disjoint_union(S.hub_bipartite(880, 900, 0.03, 21), S.random_graph(300, 0.3, 22))
    og = O.OracleGraph.from_edgelist(el)
    h = device_graph(el)
    assert K.kc_graph_info(h)[2] == og.max_outdeg() > 850
    for k in (5, 6, 7):
        announce(f"split by out-degree {dsplit} k={k}")
        assert K.kc_count(h, k) == og.count(k), k
    c, _ = per_root(h, el.n, 5)
    assert np.array_equal(c, og.count_per_root(5))
    for scheme in (K.KC_COLOR_PER_ROOT, K.KC_COLOR_GLOBAL):
        e = K.kc_count_colored(h, 5, 2, 5, scheme)
        assert e.raw == og.count_colored(5, 2, 5, scheme), scheme
    _close(h)


@pytest.mark.parametrize("p", [1.0, 0.5, 0.2])
def test_pair_sampling_raw_counts_match_oracle(p):
    """Plain pair sampling (Section 6): the raw count of the masked cache equals the
    oracle's, bit for bit, on every tier (K130 has workgroup-tier roots); p = 1 is
    the exact count; the estimate is raw over the exact keep probability."""
    cases = [(SMALL[2], [3, 4]), (SMALL[1], None), (SMALL[10], None), (SMALL[12], None), (MULTI_TILE[0], None)]
    for el, ks in cases:
        og = O.OracleGraph.from_edgelist(el)
        h = device_graph(el)
        for k in ks or [k for k in bounded_ks(og, 3, 5, budget=2e6)]:
            for seed in [3, 2**63 + 17]:
                announce(f"pair sampling {el.name} k={k} p={p}")
                e = K.kc_count_pair_sampled(h, k, p, seed)
                raw = og.count_pair_sampled(k, p, seed)
                assert e.raw == raw, (el.name, k, p, seed)
                ex = (k - 1) * (k - 2) // 2
                assert e.scale_exponent == ex
                keep = O.pair_threshold(p) / 2**32
                assert e.estimate == pytest.approx(raw / keep ** ex, rel=1e-12)
                if p == 1.0:
                    assert raw == og.count(k) and e.estimate_fits_u64 and e.estimate_u64 == raw
        _close(h)


@pytest.mark.parametrize("p", [1.0, 0.5])
def test_pair_sampling_first_call_at_k7(p):
    """Pair sampling as the first k >= 7 call on a fresh handle: the handle's second
    stream (the one-wave tier beside the workgroup tier from k = 7) is created inside
    this call, on a graph with both tiers."""
    el = SMALL[10]
    og = O.OracleGraph.from_edgelist(el)
    h = device_graph(el)
    announce(f"pair sampling, first call at k=7, p={p}")
    e = K.kc_count_pair_sampled(h, 7, p, 5)
    assert e.raw == og.count_pair_sampled(7, p, 5)
    if p == 1.0:
        assert e.raw == og.count(7)
    _close(h)


def test_pair_sampling_needs_the_cache(monkeypatch):
    monkeypatch.setenv("KC_STAGE_CACHE", "0")
    h = device_graph(SMALL[10])
    with pytest.raises(K.KcError) as err:
        K.kc_count_pair_sampled(h, 4, 0.5, 1)
    assert err.value.status == K.KC_ENOMEM
    _close(h)


def test_repeat_runs_identical():
    el = SMALL[12]
    h = device_graph(el)
    for k in [4, 6]:
        vals = {K.kc_count(h, k) for _ in range(3)}
        assert len(vals) == 1
    _close(h)


def test_host_input_path():
    el = SMALL[10]
    og = O.OracleGraph.from_edgelist(el)
    h = K.kc_graph_create(el.src, el.dst, el.m_in, el.n, False, None)
    K.kc_orient(h)
    K.kc_orient(h)  # idempotent
    for k in [3, 4, 5]:
        assert K.kc_count(h, k) == og.count(k)
    _close(h)


def test_error_paths():
    el = S.complete(6)
    h = device_graph(el, orient=False)
    with pytest.raises(K.KcError) as e:
        K.kc_count(h, 3)
    assert e.value.status == K.KC_ESTATE
    K.kc_orient(h)
    for bad_k in [0, -1, K.KC_KMAX + 1]:
        with pytest.raises(K.KcError) as e:
            K.kc_count(h, bad_k)
        assert e.value.status == K.KC_EINVAL
    with pytest.raises(K.KcError) as e:
        K.kc_count_colored(h, 3, 0, 1)
    assert e.value.status == K.KC_EINVAL
    with pytest.raises(K.KcError) as e:
        K.kc_count_colored(h, 3, 2, 1, 7)
    assert e.value.status == K.KC_EINVAL
    _close(h)
    bad = np.array([0, 1, 9], np.uint32)
    with pytest.raises(K.KcError) as e:
        K.kc_graph_create(bad, np.array([1, 2, 3], np.uint32), 3, 5, False, None)
    assert e.value.status == K.KC_EINVAL
    with pytest.raises(K.KcError) as e:
        K.kc_graph_create(None, None, 3, 5, False, None)
    assert e.value.status == K.KC_EINVAL


OVERFLOW_CHILD = """
import sys
sys.path.insert(0, sys.argv[1])
from graphgen import small as S
from paper_1403_0734_amd import kc as K
def graph(el):
    h = K.kc_graph_create(el.src, el.dst, el.m_in, el.n, False, None)
    K.kc_orient(h)
    return h
print("K5", K.kc_count(graph(S.complete(5)), 3), flush=True)
try:
    print("K6", K.kc_count(graph(S.complete(6)), 3), flush=True)
except K.KcError as e:
    print("K6 status", e.status, flush=True)
"""


def test_overflow_is_reported():
    """The carry check of the global sum, forced from the host: the library reads
    KC_TEST_TOTAL_BIAS once per process and starts every total there.  At 2^64 - 11,
    K_5's 10 triangles give 2^64 - 1 exactly and K_6's 20 must report KC_EOVERFLOW.
    Runs in a child process (host input path, default stream) with that variable."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, KC_TEST_TOTAL_BIAS=str(2**64 - 11))
    r = subprocess.run([sys.executable, "-c", OVERFLOW_CHILD, root], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = r.stdout.split("\n")
    assert f"K5 {2**64 - 1}" in lines, r.stdout
    assert f"K6 status {K.KC_EOVERFLOW}" in lines, r.stdout
    h = device_graph(S.complete(5))
    assert K.kc_count(h, 3) == 10  # this process has no bias
    _close(h)


def test_er2000_workload_against_golden():
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "counts.json")))["er2000"]
    el = G.workload_er2000()
    assert el.digest() == gold["digest"]
    h = device_graph(el)
    for k, q in gold["q"].items():
        assert K.kc_count(h, int(k)) == q
    for rec in gold["colour"]:
        e = K.kc_count_colored(h, rec["k"], rec["c"], rec["seed"], rec["scheme"])
        assert e.raw == rec["raw"]
    _close(h)
