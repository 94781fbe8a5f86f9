"""Benchmark: k-cliques/s on one MI355X.

A step is one pass of the whole counting path over one synthetic graph already
resident in HBM, on a fresh handle: ingest (simple graph + degrees) ->
orientation -> staging of every G+(u) (the first count) -> exact q_k for every k
(scheduling, per-root counting, reduction) -> one colour-sampled estimate.
``value`` = (sum of q_k over the k counted) / (seconds per step).  The default
workload is the planted-clique Chung-Lu graph (n = 4,000,000, exponent 2.0, mean
degree 30, 200 planted 30-cliques) at k = 3..8.

    python bench.py [--steps K] [--warmup W] [--workload planted_4m] [--ks 3,...,8]
                    [--schedule edges|degree|learned] [--no-cpu-baseline] [--no-extras]

Prints one JSON line.  Only one GPU is used; --gpus above 1 is refused.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "k-cliques/s and s/graph at k=3..8, 1 MI355X; learned vs degree-binned schedule"
# Spec-derived peaks of one MI355X (256 CUs, 2.4 GHz): int32 VALU = 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (one op per lane per clock, not packed); LDS = 256 CUs x 256 B/clock
# (128-bit reads) x 2.4 GHz; HBM3E 8 TB/s.  The on-box microbenchmarks (libkc_peaks) are
# reported beside them, with each fraction against both.
INT_PEAK = 256 * 4 * 16 * 2.4e9
LDS_PEAK = 256 * 256 * 2.4e9
HBM_PEAK = 8.0e12

WORKLOADS = {
    "planted_4m": ("workload_planted", [3, 4, 5, 6, 7, 8]),
    "chung_lu_1m": ("workload_chung_lu_1m", [3, 4, 5, 6]),
    "rmat22": ("workload_rmat22", [3, 4, 5]),
    "er2000": ("workload_er2000", [3, 4]),
}
EXTRAS = ["peaks", "chung_lu_1m", "per_node", "batch", "schedule", "rmat22"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="planted_4m", choices=sorted(WORKLOADS))
    ap.add_argument("--ks", default=None, help="comma-separated clique sizes (default: the workload's)")
    ap.add_argument("--colour", default=None, help="k,c,seed of the colour estimate in each step (default: max k,4,11)")
    ap.add_argument("--schedule", default="edges", choices=["edges", "degree", "learned"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline step")
    ap.add_argument("--extras", default=",".join(EXTRAS), help="comma-separated extra blocks: " + ",".join(EXTRAS))
    ap.add_argument("--batch-graphs", type=int, default=512)
    ap.add_argument("--sched-ks", default="3,4,5,6,7,8")
    ap.add_argument("--rmat-budget", type=float, default=90.0, help="seconds of GPU work for the R-MAT block")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE) and exit")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "hbm_traffic_planted_4m.md"),
                    help="profile summary holding kernels' HBM bytes per launch (rocprofv3 counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the counting path has no multi-GPU mode "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        a = torch.empty(args.copy_calibration << 20, dtype=torch.uint8, device="cuda:0")
        a.fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel()}), flush=True)
        return

    import graphgen as G
    from paper_1403_0734_amd import kc as K

    extras = set() if args.no_extras else {x for x in args.extras.split(",") if x}
    fn_name, default_ks = WORKLOADS[args.workload]
    ks = [int(x) for x in args.ks.split(",")] if args.ks else default_ks
    ck, cc, cseed = ([int(x) for x in args.colour.split(",")] if args.colour else [max(ks), 4, 11])
    stream = torch.cuda.current_stream().cuda_stream
    K.load()

    wpath = None
    if args.schedule == "learned" or "schedule" in extras:
        wpath, train_info = train_schedule(K, torch, G, stream, max(max(ks), 8))

    log(f"generating {args.workload}")
    el = getattr(G, fn_name)()
    dev = torch.device("cuda:0")
    src = torch.from_numpy(el.src.view(np.int32)).to(dev)
    dst = torch.from_numpy(el.dst.view(np.int32)).to(dev)
    torch.cuda.synchronize()
    policy = {"edges": K.KC_SCHED_EDGES, "degree": K.KC_SCHED_DEGREE, "learned": K.KC_SCHED_LEARNED}[args.schedule]

    def step(record=None):
        t0 = time.perf_counter()
        h = K.kc_graph_create(src.data_ptr(), dst.data_ptr(), el.m_in, el.n, True, stream)
        try:
            t1 = time.perf_counter()
            K.kc_orient(h)
            t2 = time.perf_counter()
            K.kc_set_schedule(h, policy, wpath if policy == K.KC_SCHED_LEARNED else None)
            qs = {}
            for i, k in enumerate(ks):
                qs[k] = K.kc_count(h, k)
                if record is not None:
                    record.setdefault(k, []).append(K.kc_last_timings(h))
                    record.setdefault(("tiers", k), []).append(K.kc_last_tier_timings(h))
                    if i == 0:
                        record.setdefault("stage_tiers", []).append(K.kc_last_stage_timings(h))
            est = K.kc_count_colored(h, ck, cc, cseed, K.KC_COLOR_PER_ROOT)
            if record is not None:
                record.setdefault("colour", []).append(K.kc_last_timings(h))
                record.setdefault("ingest_ms", []).append((t1 - t0) * 1e3)
                record.setdefault("orient_ms", []).append((t2 - t1) * 1e3)
            info = K.kc_graph_info(h)
        finally:
            K.kc_graph_destroy(h)
        return qs, est, info

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    rec = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        qs, est, info = step(rec)
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    total_q = sum(qs.values())
    value = total_q / ((t1 - t0) / args.steps)

    # stages of the step (means over the timed steps; HIP events on the library's stream
    # for the counting calls, host clocks around the synchronous ingest and orientation)
    mean = lambda xs: sum(xs) / len(xs)
    stages = {"ingest_ms": mean(rec["ingest_ms"]), "orient_ms": mean(rec["orient_ms"]),
              "staging_ms": mean([t[0] for t in rec[ks[0]]]),
              "staging_tiers_ms": [round(mean([t[i] for t in rec["stage_tiers"]]), 4) for i in range(3)],
              "colour_ms": mean([t[2] for t in rec["colour"]])}
    per_k = {}
    for i, k in enumerate(ks):
        ts = rec[k]
        t_count = mean([t[1] for t in ts])
        per_k[str(k)] = {"q": qs[k], "ms_schedule": round(mean([t[0] for t in ts]), 4) if i else 0.0,
                         "ms_count": round(t_count, 4),
                         "ms_tiers": [round(mean([t[j] for t in rec[("tiers", k)]]), 4) for j in range(3)],
                         "kcliques_per_s_count": qs[k] / (t_count * 1e-3) if t_count > 0 else None}
    stages["counts_ms"] = sum(v["ms_count"] + v["ms_schedule"] for v in per_k.values())

    out = {
        "metric": METRIC, "value": value, "unit": "k-cliques/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": el.name, "n": el.n, "m_in": el.m_in, "m": info[1], "max_outdeg": info[2], "ks": ks,
                   "schedule": args.schedule,
                   "colour_estimate": {"k": ck, "c": cc, "seed": cseed, "scheme": "per_root", "raw": est.raw,
                                       "estimate": est.estimate}},
        "stages": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in stages.items()},
        "per_k": per_k,
    }
    peaks = measure_peaks(torch, stream) if "peaks" in extras else None
    out["roofline"] = roofline(args, K, torch, np, el, src, dst, stream, ks, per_k, stages, policy, wpath, peaks)
    if peaks:
        out["peaks_measured"] = peaks

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(el, ks, qs)
    if "chung_lu_1m" in extras and args.workload != "chung_lu_1m":
        out["chung_lu_1m"] = bench_secondary(K, torch, np, G, stream, "chung_lu_1m")
    if "per_node" in extras:
        out["per_node"] = bench_per_node(K, torch, np, el, src, dst, stream, ks, qs)
    if "batch" in extras and args.batch_graphs > 0:
        out["batch"] = bench_batch(args, K, torch, stream)
        K.kc_set_tuning(defaults=True)  # the batch's tuning does not carry over
    if "schedule" in extras:
        out["schedule"] = bench_schedule(args, K, torch, np, G, stream, wpath, train_info)
    if "rmat22" in extras:
        out["rmat22"] = bench_rmat(args, K, torch, np, G, stream)
    print(json.dumps(out), flush=True)


def device_graph(K, torch, np, el, stream):
    dev = torch.device("cuda:0")
    src = torch.from_numpy(el.src.view(np.int32)).to(dev)
    dst = torch.from_numpy(el.dst.view(np.int32)).to(dev)
    torch.cuda.synchronize()
    h = K.kc_graph_create(src.data_ptr(), dst.data_ptr(), el.m_in, el.n, True, stream)
    K.kc_orient(h)
    return h


def train_schedule(K, torch, G, stream, kmax):
    """The scheduler MLP, trained on the per-root work the exact counter measures on the
    ER 2000 and Chung-Lu 1M graphs (clique sizes 4..kmax), outside every timed region."""
    import tempfile
    import numpy as np
    log("training the scheduler MLP on the ER 2000 and Chung-Lu 1M graphs")
    train = [device_graph(K, torch, np, G.workload_er2000(), stream),
             device_graph(K, torch, np, G.workload_chung_lu_1m(), stream)]
    wpath = os.path.join(tempfile.mkdtemp(), "sched.bin")
    t0 = time.perf_counter()
    loss = K.kc_train_schedule(train, kmax, 20, 1, wpath)
    t_train = time.perf_counter() - t0
    for h in train:
        K.kc_graph_destroy(h)
    return wpath, {"train_loss": loss, "train_seconds": t_train, "train_graphs": ["er2000", "chung_lu_1m"],
                   "train_ks": f"4..{kmax}"}


def measure_peaks(torch, stream):
    """On-box peaks: HBM copy (1 GiB), LDS 128-bit reads, int32 VALU, 64-bit AND+popcount."""
    from paper_1403_0734_amd import peaks as P
    log("peak microbenchmarks")
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    res = {}
    ms, work = P.hbm_copy(a.data_ptr(), b.data_ptr(), nbytes, 10, stream)
    res["hbm_copy_GBps"] = work / (ms * 1e-3) / 1e9
    del a, b
    blocks = 256 * 16
    ms, work = P.lds_read(blocks, 4096, 5, stream)
    res["lds_read_TBps"] = work / (ms * 1e-3) / 1e12
    ms, work = P.valu_int32(blocks, 4096, 5, stream)
    res["valu_int32_Tops"] = work / (ms * 1e-3) / 1e12
    ms, work = P.and_popcount(blocks, 4096, 5, stream)
    res["and_popcount_Twords"] = work / (ms * 1e-3) / 1e12
    res["spec"] = {"hbm_GBps": HBM_PEAK / 1e9, "lds_TBps": LDS_PEAK / 1e12, "valu_int32_Tops": INT_PEAK / 1e12}
    return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in res.items()}


def roofline(args, K, torch, np, el, src, dst, stream, ks, per_k, stages, policy, wpath, peaks):
    """Roofline of the step's dominant kernel (the largest mean launch time over the
    staging pass's tier kernels and every count's tier kernels).

    Count kernels (one-wave / workgroup / scratch tier at clique size k) are bound by
    int32 VALU and LDS: their algorithmic work is the neighbourhood intersections of
    the unpruned depth-first count over the tier's roots, W(u, k) = sum over l = 1..k-2
    of the l-cliques of G+(u) (the per-root work label kc_count_per_root reports), each
    at least one 64-bit AND and popcount (4 int32 ops) reading two 8-byte rows from
    LDS.  Staging kernels are bound by HBM gathers: 4 bytes per out-list element read,
    sum over the tier's roots u of d+(u) + sum over x in Gamma+(u) of d+(x)."""
    cands = [(stages["staging_tiers_ms"][i], "stage", i) for i in range(3)]
    for k in ks:
        for i in range(3):
            cands.append((per_k[str(k)]["ms_tiers"][i], k, i))
    ms, kdom, tier = max(cands, key=lambda c: c[0])
    dev = torch.device("cuda:0")
    h = K.kc_graph_create(src.data_ptr(), dst.data_ptr(), el.m_in, el.n, True, stream)
    K.kc_orient(h)
    n = el.n
    optr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    ocol = torch.zeros(max(el.m_in, 1), dtype=torch.int32, device=dev)
    r2i = torch.zeros(n, dtype=torch.int32, device=dev)
    K.kc_get_oriented(h, optr.data_ptr(), ocol.data_ptr(), r2i.data_ptr())
    wd = K.kc_get_tuning()["wave_dmax"]
    d_rank = np.diff(optr.cpu().numpy())
    tiers_of = lambda d, k: [(d >= max(k - 1, 2)) & (d <= wd), d > wd, np.zeros(d.shape, bool)]
    kk, mode = (3, 1) if kdom == "stage" else (kdom, 2)
    kname = (f"k_count_wave<{kk}, {mode}>" if tier == 0 else
             f"k_count_wg<{kk}, {'true' if tier == 2 else 'false'}, {mode}>")
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        for line in open(args.traffic):
            if line.startswith("    {"):
                traffic = json.loads(line).get(kname)
    if kdom == "stage":
        m = int(optr[-1].item())
        oc = ocol[:m].cpu().numpy().astype(np.int64)
        wedge = np.add.reduceat(d_rank[oc], optr[:-1].cpu().numpy().clip(max=max(m - 1, 0))) if m else np.zeros(n)
        wedge = np.where(d_rank > 0, wedge, 0)
        sel = tiers_of(d_rank, 3)[tier]
        nbytes = 4.0 * float(wedge[sel].sum() + d_rank[sel].sum())
        achieved = nbytes / (ms * 1e-3)
        res = {"bound": "hbm", "kernel": kname, "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
               "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": traffic, "ms_per_launch": ms,
               "work": f"4 B x {nbytes / 4:.6g} out-list elements (roots of the tier)"}
        if peaks:
            res["frac_of_measured"] = achieved / (peaks["hbm_copy_GBps"] * 1e9)
    else:
        K.kc_set_schedule(h, policy, wpath if policy == K.KC_SCHED_LEARNED else None)
        cnt = torch.zeros(n, dtype=torch.int64, device=dev)
        work = torch.zeros(n, dtype=torch.int64, device=dev)
        K.kc_count_per_root(h, kdom, cnt.data_ptr(), work.data_ptr())
        d_id = np.zeros(n, np.int64)
        d_id[r2i.cpu().numpy().view(np.uint32)] = d_rank
        w_id = work.cpu().numpy().astype(np.float64)
        inter = float(w_id[tiers_of(d_id, kdom)[tier]].sum())
        achieved = 4.0 * inter / (ms * 1e-3)
        lds = 16.0 * inter / (ms * 1e-3)
        res = {"bound": "alu", "kernel": kname, "achieved": achieved / 1e12,
               "peak": INT_PEAK / 1e12, "unit": "TOP/s (int32)", "frac": achieved / INT_PEAK, "traffic": traffic,
               "ms_per_launch": ms, "work": f"4 ops x {inter:.6g} intersections (roots of the tier, k={kdom})",
               "lds": {"achieved_TBps": lds / 1e12, "peak_TBps": LDS_PEAK / 1e12, "frac": lds / LDS_PEAK,
                       "work": "16 B (two 64-bit rows) per intersection"}}
        if peaks:
            res["frac_of_measured"] = achieved / (peaks["valu_int32_Tops"] * 1e12)
            res["lds"]["frac_of_measured"] = lds / (peaks["lds_read_TBps"] * 1e12)
        if policy == K.KC_SCHED_LEARNED:
            res["note"] = "tier membership by out-degree; the learned schedule promotes a few one-wave roots"
    K.kc_graph_destroy(h)
    torch.cuda.synchronize()
    return res


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def cpu_baseline(el, ks, qs):
    """The oracle (plain C, OpenMP over roots) on the host cores, on a random sample of
    roots of the same graph: k-cliques found per second over the sampled roots
    (roots are independent, Section 3), sample doubled until it takes 10 s."""
    import numpy as np
    import oracle as O
    import graphgen as G
    threads = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        threads = min(threads, int(omp))
    log(f"cpu baseline: oracle with {threads} threads")
    c0 = time.perf_counter()
    og = O.OracleGraph.from_edgelist(el)
    t_build = time.perf_counter() - c0
    rng = np.random.default_rng(2024)
    size, spent, found = 2000, 0.0, 0
    sample = 0
    while True:
        roots = rng.choice(el.n, size=min(size, el.n), replace=False).astype(np.uint32)
        c1 = time.perf_counter()
        got = sum(int(og.count_roots(roots, k, threads=threads).sum(dtype=np.uint64)) for k in ks)
        dt = time.perf_counter() - c1
        if dt >= 10.0 or size >= el.n or size >= 2_000_000:
            spent, found, sample = dt, got, len(roots)
            break
        size *= 2
    # single-threaded exact counts of the ER 2000 graph (k = 3, 4)
    er = O.OracleGraph.from_edgelist(G.workload_er2000())
    c2 = time.perf_counter()
    er_q = [er.count(k, threads=1) for k in (3, 4)]
    t_er = time.perf_counter() - c2
    return {"value": found / spent if spent > 0 else None, "unit": "k-cliques/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_info(),
            "sample": f"{sample} random roots of {el.name}, exact per-root counts for k={ks}: {found} cliques in "
                      f"{spent:.1f} s (graph build {t_build:.1f} s, not counted)",
            "er2000_single_thread": {"q3": er_q[0], "q4": er_q[1], "seconds": t_er}}


def bench_secondary(K, torch, np, G, stream, name, steps=5):
    """Chung-Lu 1M: the same step (ingest -> orient -> staging -> k = 3..6 -> one
    colour estimate), timed the same way."""
    fn, ks = WORKLOADS[name]
    el = getattr(G, fn)()
    dev = torch.device("cuda:0")
    src = torch.from_numpy(el.src.view(np.int32)).to(dev)
    dst = torch.from_numpy(el.dst.view(np.int32)).to(dev)
    torch.cuda.synchronize()

    def step():
        h = K.kc_graph_create(src.data_ptr(), dst.data_ptr(), el.m_in, el.n, True, stream)
        K.kc_orient(h)
        qs = {k: K.kc_count(h, k) for k in ks}
        K.kc_count_colored(h, max(ks), 4, 11, K.KC_COLOR_PER_ROOT)
        K.kc_graph_destroy(h)
        return qs

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        qs = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"workload": el.name, "ks": ks, "q": {str(k): v for k, v in qs.items()}, "ms_per_step": dt * 1e3,
            "kcliques_per_s": sum(qs.values()) / dt}


def bench_per_node(K, torch, np, el, src, dst, stream, ks, qs, reps=3):
    """Per-node clique-membership counts (kc_count_per_node) on the headline graph at
    every k, beside the total count on the same staged handle: median of reps timed
    calls after one untimed call each; the counts must sum to k * q_k."""
    h = K.kc_graph_create(src.data_ptr(), dst.data_ptr(), el.m_in, el.n, True, stream)
    out = {}
    try:
        K.kc_orient(h)
        c = torch.zeros(el.n, dtype=torch.int64, device="cuda:0")
        for k in ks:
            K.kc_count(h, k)
            K.kc_count_per_node(h, k, c.data_ptr())
            tc, tp = [], []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                q = K.kc_count(h, k)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                K.kc_count_per_node(h, k, c.data_ptr())
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                tc.append((t1 - t0) * 1e3)
                tp.append((t2 - t1) * 1e3)
            total = int(c.cpu().numpy().view(np.uint64).sum(dtype=np.uint64))
            out[str(k)] = {"ms_per_node": round(median(tp), 3), "ms_count": round(median(tc), 3),
                           "ratio": round(median(tp) / median(tc), 2), "sum_is_k_q": total == k * qs[k]}
            log(f"per-node k={k}: {out[str(k)]}")
    finally:
        K.kc_graph_destroy(h)
    return out


def bench_batch(args, K, torch, stream):
    """512 Chung-Lu graphs at k = 5, on equal work both ways:
    - cold: the first kc_count_batch of a plan (concatenation, queue, staging of the
      union, eager run, HIP-graph capture) against one kc_count per graph on fresh,
      unstaged handles (each stages its own graph);
    - warm: a replay of the captured HIP graph (counts from the staged union) against
      one kc_count per graph on handles that have already staged."""
    import numpy as np
    import graphgen as G
    k = 5
    log(f"batch: generating {args.batch_graphs} graphs")
    els = G.workload_batch(args.batch_graphs)
    bs = torch.cuda.Stream()
    with torch.cuda.stream(bs):
        hs = [device_graph(K, torch, np, el, bs.cuda_stream) for el in els]
        log("batch: autotuning")
        tuning = K.kc_autotune(hs, k, os.environ.get("KC_TUNE_CACHE") or None)
        # cold per-graph calls: fresh handles
        for h in hs:
            K.kc_graph_destroy(h)
        hs = [device_graph(K, torch, np, el, bs.cuda_stream) for el in els]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per_graph = [K.kc_count(h, k) for h in hs]
        t_cold_graphs = time.perf_counter() - t0
        t0 = time.perf_counter()
        warm_graphs = [K.kc_count(h, k) for h in hs]
        t_warm_graphs = time.perf_counter() - t0
        # cold batch: a fresh plan
        cold = []
        for _ in range(3):
            hs2 = [device_graph(K, torch, np, el, bs.cuda_stream) for el in els]  # new handles: a new plan
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            batched = K.kc_count_batch(hs2, k)
            cold.append(time.perf_counter() - t0)
            for h in hs2:
                K.kc_graph_destroy(h)
        K.kc_count_batch(hs, k)  # plan for the warm replays
        reps = []
        for _ in range(5):
            t0 = time.perf_counter()
            batched2 = K.kc_count_batch(hs, k)
            reps.append(time.perf_counter() - t0)
        for h in hs:
            K.kc_graph_destroy(h)
    tc, tw = median(cold), median(reps)
    return {"workload": f"{len(els)} Chung-Lu graphs, exponent 2.3, mean 20, n log-uniform in [1000, 200000]",
            "k": k, "nodes": sum(el.n for el in els), "edges_in": sum(el.m_in for el in els),
            "q_total": int(sum(batched)),
            "counts_equal": batched == per_graph == warm_graphs == batched2,
            "cold": {"s_per_batch": tc, "s_per_graph": tc / len(els), "s_per_graph_calls": t_cold_graphs,
                     "speedup": t_cold_graphs / tc},
            "warm": {"s_per_batch": tw, "s_per_graph": tw / len(els), "s_per_graph_calls": t_warm_graphs,
                     "speedup": t_warm_graphs / tw},
            "s_per_graph": tc / len(els), "tuning": tuning}


def bench_schedule(args, K, torch, np, G, stream, wpath, train_info):
    """Plain degree binning (the reference the others are measured against), the
    edge-estimate items and the learned schedule on the planted-clique Chung-Lu 4M
    graph: same kernels and counts, only the queue order, tiers and item split
    differ.  Median of 5 counts after one warm-up count per (policy, k)."""
    ks = [int(x) for x in args.sched_ks.split(",")]
    log("schedule: planted workload")
    el = G.workload_planted()
    h = device_graph(K, torch, np, el, stream)
    res = dict(train_info)
    res.update({"workload": el.name, "per_k": {}})
    names = (("degree", K.KC_SCHED_DEGREE), ("edges", K.KC_SCHED_EDGES), ("learned", K.KC_SCHED_LEARNED))
    tot = {n: 0.0 for n, _ in names}
    for k in ks:
        row = {}
        for name, pol in names:
            K.kc_set_schedule(h, pol, wpath if pol == K.KC_SCHED_LEARNED else None)
            q = K.kc_count(h, k)  # warm-up (builds the policy's cached queue)
            ts = []
            for _ in range(5):
                assert K.kc_count(h, k) == q
                ts.append(K.kc_last_timings(h)[2])
            row[name] = {"q": q, "ms": median(ts)}
            tot[name] += row[name]["ms"]
        row["equal"] = len({row[n]["q"] for n, _ in names}) == 1
        row["learned_vs_degree"] = row["degree"]["ms"] / row["learned"]["ms"]
        row["learned_vs_edges"] = row["edges"]["ms"] / row["learned"]["ms"]
        res["per_k"][str(k)] = row
        log(f"schedule k={k}: " + ", ".join(f"{n} {row[n]['ms']:.2f} ms" for n, _ in names))
    K.kc_graph_destroy(h)
    res["ms_total"] = tot
    res["learned_vs_degree"] = tot["degree"] / tot["learned"]
    res["learned_vs_edges"] = tot["edges"] / tot["learned"]
    return res


def bench_rmat(args, K, torch, np, G, stream):
    """R-MAT scale 22: exact q_k, colour-sampled estimates at c = 2, 4, 8 (seeds 11,
    12, 13, both schemes) and plain pair-sampled estimates at p = 1/c, k = 4..7, with
    the relative error against the exact count where it was counted.  Cells whose
    time, predicted from the same sampler's cell at k - 1, would exceed the budget are
    left out and listed."""
    log("rmat22: generating")
    el = G.workload_rmat22()
    h = device_graph(K, torch, np, el, stream)
    budget = args.rmat_budget
    spent = 0.0
    res = {"workload": el.name, "n": el.n, "exact": {}, "colour": [], "pair": [], "skipped": []}
    t0 = time.perf_counter()
    K.kc_count(h, 3)
    res["staging_s"] = time.perf_counter() - t0
    exact = {}
    last = None
    for k in (4, 5, 6, 7):
        if last is not None and last * 100 > budget - spent:
            res["skipped"].append(f"exact k={k}: predicted above the remaining budget")
            break
        t0 = time.perf_counter()
        exact[k] = K.kc_count(h, k)
        last = time.perf_counter() - t0
        spent += last
        res["exact"][str(k)] = {"q": exact[k], "s": last}
        log(f"rmat22 exact k={k}: {exact[k]} in {last:.2f} s")
    # every sampler at k = 4, then k = 5, ...: a cell runs when its time, predicted as 20x
    # the same sampler's time at k - 1, fits in the remaining budget
    samplers = [("colour", sname, scheme, c) for scheme, sname in ((K.KC_COLOR_GLOBAL, "global"),
                                                                    (K.KC_COLOR_PER_ROOT, "per_root"))
                for c in (8, 4, 2)] + [("pair", "pair", None, c) for c in (8, 4, 2)]
    last = {}
    for k in (4, 5, 6, 7):
        for kind, sname, scheme, c in samplers:
            key = (sname, c)
            if key in last and (last[key] is None or 3 * 20 * last[key] > budget - spent):
                if last[key] is not None:
                    res["skipped"].append(f"{sname} c={c} k>={k}: predicted above the remaining budget")
                last[key] = None
                continue
            cell = ({"scheme": sname, "c": c, "k": k, "runs": []} if kind == "colour" else
                    {"p": 1.0 / c, "k": k, "runs": []})
            t0 = time.perf_counter()
            for seed in (11, 12, 13):
                e = (K.kc_count_colored(h, k, c, seed, scheme) if kind == "colour" else
                     K.kc_count_pair_sampled(h, k, 1.0 / c, seed))
                r = {"seed": seed, "raw": e.raw, "estimate": e.estimate}
                if k in exact:
                    r["rel_error"] = abs(e.estimate - exact[k]) / exact[k]
                cell["runs"].append(r)
            dt = (time.perf_counter() - t0) / 3
            spent += 3 * dt
            last[key] = dt
            cell["s_per_estimate"] = dt
            if k in exact:
                cell["mean_rel_error"] = sum(r["rel_error"] for r in cell["runs"]) / 3
            else:
                est = [r["estimate"] for r in cell["runs"]]
                cell["estimate_mean"] = sum(est) / 3
            res[kind].append(cell)
    res["gpu_seconds"] = spent
    K.kc_graph_destroy(h)
    return res


if __name__ == "__main__":
    main()
