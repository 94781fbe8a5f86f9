"""GPU tests of the scheduling and batching layers: neither may change a count.
Learned schedule vs degree schedule vs oracle; batched counts (eager, captured
HIP graph replays, every tunable setting) vs per-graph oracle counts; the
autotuner's cache."""
import os

import numpy as np
import pytest

import oracle as O
import graphgen as G
from graphgen import small as S
from paper_1403_0734_amd import kc as K

from gpu_util import announce, device_graph, per_root

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    import torch
    assert torch.cuda.is_available()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        yield s


def graph_on(el, stream):
    import torch
    dev = torch.device("cuda:0")
    src = torch.from_numpy(el.src.view(np.int32).copy()).to(dev)
    dst = torch.from_numpy(el.dst.view(np.int32).copy()).to(dev)
    torch.cuda.synchronize()
    h = K.kc_graph_create(src.data_ptr(), dst.data_ptr(), el.m_in, el.n, True, stream.cuda_stream)
    K.kc_orient(h)
    return h


def training_graphs():
    return [G.workload_er2000(), G.chung_lu(60000, 2.1, 20.0, 1000.0, 21),
            S.planted_small(3000, 0.004, [list(range(i, i + 25)) for i in range(0, 2500, 500)], 9)]


def test_learned_schedule_counts_equal(stream, tmp_path):
    train = [graph_on(el, stream) for el in training_graphs()]
    wpath = str(tmp_path / "w.bin")
    announce("training the scheduler MLP")
    loss = K.kc_train_schedule(train, 6, 30, 7, wpath)
    assert np.isfinite(loss) and loss < 0.5, loss
    el = S.planted_small(5000, 0.003, [list(range(i, i + 28)) for i in range(0, 4000, 400)], 3)
    og = O.OracleGraph.from_edgelist(el)
    h = graph_on(el, stream)
    for k in range(3, 8):
        announce(f"learned vs degree k={k}")
        K.kc_set_schedule(h, K.KC_SCHED_DEGREE)
        qd = K.kc_count(h, k)
        K.kc_set_schedule(h, K.KC_SCHED_LEARNED, wpath)
        ql = K.kc_count(h, k)
        assert qd == ql == og.count(k), k
        c, _ = per_root(h, el.n, k)
        assert np.array_equal(c, og.count_per_root(k))
    # colour sampling under the learned schedule
    e = K.kc_count_colored(h, 5, 3, 99, K.KC_COLOR_PER_ROOT)
    assert e.raw == og.count_colored(5, 3, 99, O.COLOR_PER_ROOT)
    for g in train + [h]:
        K.kc_graph_destroy(g)


def test_learned_schedule_on_held_out_graph(stream, tmp_path):
    """A schedule trained on other graphs: counts and work labels stay exact."""
    train = [graph_on(el, stream) for el in training_graphs()]
    wpath = str(tmp_path / "w.bin")
    K.kc_train_schedule(train, 6, 30, 11, wpath)
    el = G.chung_lu(80000, 2.1, 20.0, 2000.0, 77)
    h = graph_on(el, stream)
    _, work = per_root(h, el.n, 6, with_work=True)
    og = O.OracleGraph.from_edgelist(el)
    K.kc_set_schedule(h, K.KC_SCHED_LEARNED, wpath)
    assert K.kc_count(h, 6) == og.count(6)
    inter, _ = og.work_per_root(6)
    assert np.array_equal(work, inter)
    for g in train + [h]:
        K.kc_graph_destroy(g)


def test_bad_weight_file(stream, tmp_path):
    h = graph_on(S.complete(8), stream)
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a weight file")
    with pytest.raises(K.KcError) as e:
        K.kc_set_schedule(h, K.KC_SCHED_LEARNED, str(bad))
    assert e.value.status == K.KC_EINVAL
    with pytest.raises(K.KcError) as e:
        K.kc_set_schedule(h, K.KC_SCHED_LEARNED, None)
    assert e.value.status == K.KC_ESTATE
    K.kc_graph_destroy(h)


def batch_graphs():
    gs = []
    for i, n in enumerate([500, 3000, 1200, 20000, 800, 7000]):
        gs.append(G.chung_lu(n, 2.3, 20.0, (20.0 * n) ** 0.5, 100 + i))
    gs += [S.complete(70), S.complete_multipartite([30, 40, 50]), S.empty(5), S.random_graph(200, 0.3, 5),
           S.planted_small(1500, 0.01, [list(range(0, 40)), list(range(500, 530))], 2)]
    return gs


@pytest.mark.parametrize("cache", ["1", "0"])
@pytest.mark.parametrize("k", [3, 5, 6])
def test_batch_matches_per_graph(stream, k, cache, monkeypatch):
    """Batched counts equal per-graph counts: with the plan's union staged once and
    the from-cache kernels captured (default), and staged on every replay."""
    monkeypatch.setenv("KC_STAGE_CACHE", cache)
    els = batch_graphs()
    want = [O.OracleGraph.from_edgelist(el).count(k) for el in els]
    hs = [graph_on(el, stream) for el in els]
    announce(f"batch k={k} cache={cache}")
    for rep in range(3):  # eager + capture, then graph replays
        assert K.kc_count_batch(hs, k) == want, rep
    assert [K.kc_count(h, k) for h in hs] == want
    # a different subset and order re-plans
    sub = [hs[3], hs[0], hs[7]]
    assert K.kc_count_batch(sub, k) == [want[3], want[0], want[7]]
    for h in hs:
        K.kc_graph_destroy(h)


def test_batch_default_stream_and_destroy():
    els = batch_graphs()[:4]
    want = [O.OracleGraph.from_edgelist(el).count(4) for el in els]
    hs = [K.kc_graph_create(el.src, el.dst, el.m_in, el.n, False, None) for el in els]
    for h in hs:
        K.kc_orient(h)
    assert K.kc_count_batch(hs, 4) == want
    assert K.kc_count_batch(hs, 4) == want
    K.kc_graph_destroy(hs[1])  # drops the cached plan
    assert K.kc_count_batch([hs[0], hs[2], hs[3]], 4) == [want[0], want[2], want[3]]
    for h in (hs[0], hs[2], hs[3]):
        K.kc_graph_destroy(h)


TUNING_FIELDS = ["wave_dmax", "wg_blocks_per_cu", "wave_blocks_per_cu", "queue_chunk_div", "wg_dmax", "local_bits"]


@pytest.mark.parametrize("tuning", [(16, 0, 8, 8, 0, 128), (24, 2, 4, 4, 0, 64), (48, 1, 16, 64, 64, 128),
                                    (64, 8, 1, 1, 0, 128), (1, 0, 8, 8, 100, 64)])
def test_tunables_never_change_counts(stream, tuning):
    els = batch_graphs()
    want5 = [O.OracleGraph.from_edgelist(el).count(5) for el in els]
    hs = [graph_on(el, stream) for el in els]
    try:
        K.kc_set_tuning(*tuning)
        assert K.kc_get_tuning() == dict(zip(TUNING_FIELDS, tuning))
        assert K.kc_count_batch(hs, 5) == want5
        assert [K.kc_count(h, 5) for h in hs] == want5
    finally:
        K.kc_set_tuning(defaults=True)
        for h in hs:
            K.kc_graph_destroy(h)


def test_tuning_rejects_bad_values():
    for bad in [(0, 0, 8, 8), (65, 0, 8, 8), (64, 9, 8, 8), (64, 0, 0, 8), (64, 0, 8, 65), (64, 0, 8, 8, 63),
                (64, 0, 8, 8, 65536), (64, 0, 8, 8, 0, 96)]:
        with pytest.raises(K.KcError) as e:
            K.kc_set_tuning(*bad)
        assert e.value.status == K.KC_EINVAL
    K.kc_set_tuning(defaults=True)
    assert K.kc_get_tuning() == dict(zip(TUNING_FIELDS, (64, 0, 8, 8, 0, 128)))


def test_autotune_cache(stream, tmp_path):
    els = batch_graphs()
    want = [O.OracleGraph.from_edgelist(el).count(4) for el in els]
    hs = [graph_on(el, stream) for el in els]
    cache = str(tmp_path / "tune.tsv")
    try:
        announce("autotune")
        best = K.kc_autotune(hs, 4, cache)
        assert best["wave_dmax"] in (24, 48, 64)
        assert os.path.exists(cache)
        line = open(cache).read().strip().split("\t")
        assert len(line) == 2 and "k=4" in line[0]
        K.kc_set_tuning(defaults=True)
        again = K.kc_autotune(hs, 4, cache)  # read back, no timing
        assert again == best
        assert K.kc_get_tuning() == best
        assert K.kc_count_batch(hs, 4) == want
    finally:
        K.kc_set_tuning(defaults=True)
        for h in hs:
            K.kc_graph_destroy(h)
