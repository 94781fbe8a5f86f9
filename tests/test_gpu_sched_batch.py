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
    for k in range(3, 9):
        announce(f"learned vs degree vs edges k={k}")
        K.kc_set_schedule(h, K.KC_SCHED_DEGREE)
        qd = K.kc_count(h, k)
        K.kc_set_schedule(h, K.KC_SCHED_EDGES)
        qe = K.kc_count(h, k)
        K.kc_set_schedule(h, K.KC_SCHED_LEARNED, wpath)
        ql = K.kc_count(h, k)
        assert qd == qe == ql == og.count(k), k
        assert K.kc_count(h, k) == ql  # the learned queue of this k, cached
        c, _ = per_root(h, el.n, k)
        assert np.array_equal(c, og.count_per_root(k))
    # colour sampling under the learned schedule
    e = K.kc_count_colored(h, 5, 3, 99, K.KC_COLOR_PER_ROOT)
    assert e.raw == og.count_colored(5, 3, 99, O.COLOR_PER_ROOT)
    for g in train + [h]:
        K.kc_graph_destroy(g)


@pytest.mark.parametrize("cache", ["1", "0"])
def test_learned_promotion_of_every_candidate(stream, tmp_path, monkeypatch, cache):
    """With a promotion threshold of 0 the learned schedule moves every one-wave root it
    considers into the workgroup tier, whose cached path then reads their staged rows
    (not packed bitmaps); a dense G(500, 0.6) adds wide first-level nodes, each split
    into two-level items of the learned estimate.  Counts, per-root counts and colourings against the
    oracle, staged once or per call."""
    monkeypatch.setenv("KC_STAGE_CACHE", cache)
    monkeypatch.setenv("KC_PROMOTE_LOGWORK", "0")
    monkeypatch.setenv("KC_LEVEL2", "2")
    train = [graph_on(el, stream) for el in training_graphs()[:2]]
    wpath = str(tmp_path / "w.bin")
    K.kc_train_schedule(train, 6, 5, 3, wpath)
    for g in train:
        K.kc_graph_destroy(g)
    for el in [S.planted_small(3000, 0.004, [list(range(i, i + 25)) for i in range(0, 2500, 500)], 9),
               S.random_graph(500, 0.6, 8)]:
        og = O.OracleGraph.from_edgelist(el)
        h = graph_on(el, stream)
        K.kc_set_schedule(h, K.KC_SCHED_LEARNED, wpath)
        ks = [k for k in range(3, 9) if k < 6 or el.n != 500]
        for k in ks:
            announce(f"learned, all promoted, cache={cache} {el.name} k={k}")
            assert K.kc_count(h, k) == og.count(k), (el.name, k)
        k = ks[-1]
        c, _ = per_root(h, el.n, k)
        assert np.array_equal(c, og.count_per_root(k)), (el.name, k)
        e = K.kc_count_colored(h, 5, 3, 8, K.KC_COLOR_PER_ROOT)
        assert e.raw == og.count_colored(5, 3, 8, O.COLOR_PER_ROOT)
        K.kc_graph_destroy(h)


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


# ---------------------------------------------------------------------------
# The MLP's fp32 kernels against torch (fp32 forward, autograd gradient, Adam)

def _mlp_layout(P):
    P = np.asarray(P)
    return (P[0:256].reshape(32, 8), P[256:288], P[288:1312].reshape(32, 32), P[1312:1344], P[1344:1376], P[1376])


def _torch_forward(P, x):
    import torch
    W1, b1, W2, b2, w3, b3 = _mlp_layout(P)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32)
    h1 = torch.relu(t(x) @ t(W1).T + t(b1))
    h2 = torch.relu(h1 @ t(W2).T + t(b2))
    return (h2 @ t(w3) + float(b3)).numpy()


def _write_weights(path, params, norm):
    with open(path, "wb") as f:
        f.write(b"KCMLP001")
        f.write(np.uint32(K.KC_MLP_PARAMS).tobytes())
        f.write(np.asarray(norm, np.float32).tobytes())
        f.write(np.asarray(params, np.float32).tobytes())


def _features_from_oracle(og, k):
    """The eight scheduler features recomputed in float64 from the oracle's Gamma+
    lists and per-root triangle counts (edges of G+(u)), by original id."""
    import math
    hp, hn = og.high_csr()
    dplus = np.diff(hp.astype(np.int64))
    deg = og.degrees().astype(np.float64)
    ep = og.count_per_root(3).astype(np.float64)
    n = og.n
    wed = np.zeros(n)
    mx = np.zeros(n)
    for u in range(n):
        nb = hn[hp[u]:hp[u + 1]]
        if len(nb):
            wed[u] = dplus[nb].sum()
            mx[u] = dplus[nb].max()
    pairs = np.where(dplus >= 2, 0.5 * dplus * (dplus - 1), 0.0)
    dens = np.divide(ep, pairs, out=np.zeros(n), where=pairs > 0)
    lc = np.full(n, -10.0)
    r = k - 1
    for u in range(n):
        if dplus[u] >= r and dens[u] > 0:
            v = (math.lgamma(dplus[u] + 1) - math.lgamma(r + 1) - math.lgamma(dplus[u] - r + 1)
                 + 0.5 * r * (r - 1) * math.log(dens[u]))
            lc[u] = min(max(v, -10.0), 60.0)
    f = np.stack([np.log1p(dplus), np.log1p(wed), np.log1p(mx), np.log1p(deg), np.log1p(ep), dens,
                  np.full(n, k / 10.0), lc], 1)
    return f.astype(np.float32), dplus


def test_mlp_forward_matches_torch(stream, tmp_path):
    """kc_predict_work (features + the fp32 inference kernel) against the oracle's
    features and a torch fp32 forward pass of the same weight file."""
    import torch
    rng = np.random.default_rng(5)
    params = (rng.standard_normal(K.KC_MLP_PARAMS) * 0.3).astype(np.float32)
    norm = np.array([2, 5, 4, 3, 4, 0.3, 0.5, 0, 1, 2, 2, 1, 2, 0.3, 0.2, 5, 3, 2], np.float32)
    wpath = str(tmp_path / "w.bin")
    _write_weights(wpath, params, norm)
    el = S.planted_small(3000, 0.004, [list(range(i, i + 25)) for i in range(0, 2500, 500)], 9)
    og = O.OracleGraph.from_edgelist(el)
    h = graph_on(el, stream)
    K.kc_set_schedule(h, K.KC_SCHED_LEARNED, wpath)
    for k in (4, 7):
        announce(f"MLP forward k={k}")
        pred = torch.zeros(el.n, dtype=torch.float32, device="cuda:0")
        feat = torch.zeros(el.n * 8, dtype=torch.float32, device="cuda:0")
        K.kc_predict_work(h, k, pred.data_ptr(), feat.data_ptr())
        torch.cuda.synchronize()
        f = feat.cpu().numpy().reshape(el.n, 8)
        want_f, dplus = _features_from_oracle(og, k)
        np.testing.assert_allclose(f, want_f, rtol=2e-6, atol=1e-6)
        x = (f - norm[:8]) / norm[8:16]
        y = _torch_forward(params, x) * norm[17] + norm[16]
        active = dplus >= k - 1
        p = pred.cpu().numpy()
        np.testing.assert_allclose(p[active], y[active], rtol=1e-5, atol=1e-5)
        assert np.all(p[~active] == 0)
    K.kc_graph_destroy(h)


def test_mlp_step_matches_torch_autograd(stream):
    """kc_mlp_step (the gradient and Adam kernels of the training loop) against torch
    autograd of 0.5 * mean (y - t)^2 and the Adam update, over three steps with
    batches of 200, 137 and 64 samples (ragged 64-sample blocks)."""
    import torch
    rng = np.random.default_rng(17)
    P = (rng.standard_normal(K.KC_MLP_PARAMS) * 0.3).astype(np.float32)
    dev = torch.device("cuda:0")
    dP = torch.from_numpy(P.copy()).to(dev)
    dM = torch.zeros_like(dP)
    dV = torch.zeros_like(dP)
    dG = torch.zeros_like(dP)
    m = np.zeros(K.KC_MLP_PARAMS)
    v = np.zeros(K.KC_MLP_PARAMS)
    lr = 2e-3
    for step, count in enumerate([200, 137, 64], start=1):
        x = rng.standard_normal((count, 8)).astype(np.float32)
        t = rng.standard_normal(count).astype(np.float32)
        dx = torch.from_numpy(x).to(dev)
        dt = torch.from_numpy(t).to(dev)
        torch.cuda.synchronize()
        p_before = dP.cpu().numpy().astype(np.float32)
        loss = K.kc_mlp_step(dP.data_ptr(), dM.data_ptr(), dV.data_ptr(), step, lr, dx.data_ptr(), dt.data_ptr(),
                             count, dG.data_ptr(), bs_stream(stream))
        torch.cuda.synchronize()
        # torch autograd at the parameters before the step
        tp = torch.tensor(p_before, dtype=torch.float32, requires_grad=True)
        W1 = tp[0:256].reshape(32, 8)
        b1 = tp[256:288]
        W2 = tp[288:1312].reshape(32, 32)
        b2 = tp[1312:1344]
        w3 = tp[1344:1376]
        b3 = tp[1376]
        y = torch.relu(torch.relu(torch.from_numpy(x) @ W1.T + b1) @ W2.T + b2) @ w3 + b3
        tl = 0.5 * ((y - torch.from_numpy(t)) ** 2).mean()
        tl.backward()
        g_ref = tp.grad.numpy()
        g = dG.cpu().numpy()
        np.testing.assert_allclose(g, g_ref, rtol=1e-4, atol=2e-6)
        assert loss == pytest.approx(float(tl), rel=1e-5)
        # Adam from the library's gradient, in float64 with the kernel's fp32 constants
        # (1 - beta2 rounds to 0.00099998713 in fp32)
        f32 = np.float32
        b1, b2 = float(f32(0.9)), float(f32(0.999))
        ob1, ob2 = float(f32(1) - f32(0.9)), float(f32(1) - f32(0.999))
        c1, c2 = float(f32(1) - f32(0.9) ** step), float(f32(1) - f32(0.999) ** step)
        gd = g.astype(np.float64)
        m = b1 * m + ob1 * gd
        v = b2 * v + ob2 * gd * gd
        want = p_before - float(f32(lr)) * (m / c1) / (np.sqrt(v / c2) + 1e-8)
        np.testing.assert_allclose(dP.cpu().numpy(), want, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(dM.cpu().numpy(), m, rtol=1e-5, atol=1e-9)
        np.testing.assert_allclose(dV.cpu().numpy(), v, rtol=1e-5, atol=1e-12)


def bs_stream(stream):
    return stream.cuda_stream


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


@pytest.mark.parametrize("dsplit", [None, "0", "300"])
def test_learned_schedule_split_by_outdegree(stream, tmp_path, monkeypatch, dsplit):
    """The learned queue's workgroup tier in two item lists by out-degree (default
    rule, forced, or one list): roots of out-degree about 900 beside roots below 100."""
    if dsplit is not None:
        monkeypatch.setenv("KC_WG_DSPLIT", dsplit)
    train = [graph_on(el, stream) for el in training_graphs()[:2]]
    wpath = str(tmp_path / "w.bin")
    K.kc_train_schedule(train, 7, 5, 3, wpath)
    el = S.disjoint_union(S.hub_bipartite(880, 900, 0.03, 21), S.random_graph(300, 0.3, 22))
    og = O.OracleGraph.from_edgelist(el)
    h = graph_on(el, stream)
    K.kc_set_schedule(h, K.KC_SCHED_LEARNED, wpath)
    for k in (5, 6, 7):
        announce(f"learned, split by out-degree {dsplit}, k={k}")
        assert K.kc_count(h, k) == og.count(k), k
    c, _ = per_root(h, el.n, 5)
    assert np.array_equal(c, og.count_per_root(5))
    for g in train + [h]:
        K.kc_graph_destroy(g)


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


TUNING_FIELDS = ["wave_dmax", "wg_blocks_per_cu", "wave_blocks_per_cu", "queue_chunk_div", "wg_dmax", "local_bits",
                 "wg_waves"]


@pytest.mark.parametrize("tuning", [(16, 0, 8, 8, 0, 128, 0), (24, 2, 4, 4, 0, 64, 8), (48, 1, 16, 64, 64, 128, 16),
                                    (64, 8, 1, 1, 0, 128, 4), (1, 0, 8, 8, 100, 64, 16)])
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
                (64, 0, 8, 8, 65536), (64, 0, 8, 8, 0, 96), (64, 0, 8, 8, 0, 128, 12)]:
        with pytest.raises(K.KcError) as e:
            K.kc_set_tuning(*bad)
        assert e.value.status == K.KC_EINVAL
    K.kc_set_tuning(defaults=True)
    assert K.kc_get_tuning() == dict(zip(TUNING_FIELDS, (64, 0, 8, 8, 0, 128, 0)))


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
