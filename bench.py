"""Benchmark: k-cliques/s on one MI355X.

A step is one pass of the whole counting path over one synthetic graph already
resident in HBM: ingest (simple graph + degrees) -> orientation -> for every k:
schedule + per-root counting + reduction -> one colour-sampled estimate.
``value`` = (sum of q_k over the k counted) / (seconds per step).

    python bench.py [--steps K] [--warmup W] [--workload chung_lu_1m] [--ks 3,4,5,6]

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
INT_PEAK = 256 * 4 * 16 * 2.4e9  # int32 VALU ops/s: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz

WORKLOADS = {
    "chung_lu_1m": ("workload_chung_lu_1m", [3, 4, 5, 6]),
    "er2000": ("workload_er2000", [3, 4]),
    "rmat22": ("workload_rmat22", [4, 5]),
    "planted_4m": ("workload_planted", [3, 4, 5, 6, 7, 8]),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chung_lu_1m", choices=sorted(WORKLOADS))
    ap.add_argument("--ks", default=None, help="comma-separated clique sizes (default: the workload's)")
    ap.add_argument("--colour", default="6,4,11", help="k,c,seed of the colour-sampled estimate in each step")
    ap.add_argument("--schedule", default="degree", choices=["degree", "learned"])
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1403_0734_amd", "sched_weights.bin"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batch (512 graphs, k=5) and schedule-comparison (planted 4M, k=3..8) sections")
    ap.add_argument("--batch-graphs", type=int, default=512)
    ap.add_argument("--tuning", default=None, metavar="WD,WGB,WVB,CD",
                    help="launch tunables for the timed steps (default: the library's)")
    ap.add_argument("--sched-ks", default="3,4,5,6,7,8")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE) and exit")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "count_kernels_chung_lu_1m.md"),
                    help="profile summary holding the count kernels' HBM bytes per launch (rocprofv3 counters)")
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

    fn_name, default_ks = WORKLOADS[args.workload]
    ks = [int(x) for x in args.ks.split(",")] if args.ks else default_ks
    ck, cc, cseed = [int(x) for x in args.colour.split(",")]

    log(f"generating {args.workload}")
    el = getattr(G, fn_name)()
    dev = torch.device("cuda:0")
    src = torch.from_numpy(el.src.view(np.int32)).to(dev)
    dst = torch.from_numpy(el.dst.view(np.int32)).to(dev)
    stream = torch.cuda.current_stream().cuda_stream
    torch.cuda.synchronize()
    lib = K.load()
    if args.tuning:
        K.kc_set_tuning(*[int(x) for x in args.tuning.split(",")])
    policy = K.KC_SCHED_LEARNED if args.schedule == "learned" else K.KC_SCHED_DEGREE

    def step(record=None):
        h = K.kc_graph_create(src.data_ptr(), dst.data_ptr(), el.m_in, el.n, True, stream)
        try:
            K.kc_orient(h)
            if policy != K.KC_SCHED_DEGREE:
                K.kc_set_schedule(h, policy, args.weights)
            qs = {}
            for k in ks:
                qs[k] = K.kc_count(h, k)
                if record is not None:
                    record.setdefault(k, []).append(K.kc_last_timings(h))
                    record.setdefault(("tiers", k), []).append(K.kc_last_tier_timings(h))
            est = K.kc_count_colored(h, ck, cc, cseed, K.KC_COLOR_PER_ROOT)
            if record is not None:
                record.setdefault("colour", []).append(K.kc_last_timings(h))
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

    # per-k count-stage times (HIP events on the library's stream, around the
    # tier kernels of one count): the dominant stage gives the roofline
    per_k = {}
    for k in ks:
        ts = rec[k]
        t_sched = sum(t[0] for t in ts) / len(ts)
        t_count = sum(t[1] for t in ts) / len(ts)
        per_k[str(k)] = {"q": qs[k], "ms_schedule": round(t_sched, 4), "ms_count": round(t_count, 4),
                         "kcliques_per_s_count": qs[k] / (t_count * 1e-3) if t_count > 0 else None}
    kdom = max(ks, key=lambda k: per_k[str(k)]["ms_count"])
    tiers = rec[("tiers", kdom)]
    t_tier = [sum(t[i] for t in tiers) / len(tiers) for i in range(3)]
    for k in ks:
        tk = rec[("tiers", k)]
        per_k[str(k)]["ms_tiers"] = [round(sum(t[i] for t in tk) / len(tk), 4) for i in range(3)]
    # Algorithmic work of the dominant tier kernel: the unpruned depth-first count
    # performs one neighbourhood intersection per l-clique of G+(u), l = 1..k-2
    # (the per-root work label), each at least one 64-bit AND and one 64-bit
    # popcount = 4 int32 VALU ops.  The label is summed over the tier's roots.
    tier_names = ["k_count_wave", "k_count_wg", "k_count_wg (scratch)"]
    dom = max(range(3), key=lambda i: t_tier[i])
    h = K.kc_graph_create(src.data_ptr(), dst.data_ptr(), el.m_in, el.n, True, stream)
    K.kc_orient(h)
    n = el.n
    cnt = torch.zeros(n, dtype=torch.int64, device=dev)
    work = torch.zeros(n, dtype=torch.int64, device=dev)
    K.kc_count_per_root(h, kdom, cnt.data_ptr(), work.data_ptr())
    optr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    r2i = torch.zeros(n, dtype=torch.int32, device=dev)
    K.kc_get_oriented(h, optr.data_ptr(), None, r2i.data_ptr())
    # plain pair sampling (Section 6) on the same graph, outside the timed steps: the
    # colour estimate's k with p = 1/c, the same expected share of pairs
    pk, pp, pseed = ck, 1.0 / cc, 23
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    ps = K.kc_count_pair_sampled(h, pk, pp, pseed)
    tp1 = time.perf_counter()
    pair_sampling = {"k": pk, "p": pp, "seed": pseed, "raw": ps.raw, "estimate": ps.estimate, "exact": qs.get(pk),
                     "rel_error": abs(ps.estimate - qs[pk]) / qs[pk] if qs.get(pk) else None,
                     "colour_rel_error": abs(est.estimate - qs[ck]) / qs[ck] if qs.get(ck) else None,
                     "ms_call": (tp1 - tp0) * 1e3, "ms_mask_and_count": K.kc_last_timings(h)[1]}
    K.kc_graph_destroy(h)
    torch.cuda.synchronize()
    d_rank = np.diff(optr.cpu().numpy())
    d_id = np.zeros(n, np.int64)
    d_id[r2i.cpu().numpy().view(np.uint32)] = d_rank
    w_id = work.cpu().numpy().astype(np.float64)
    wd = K.kc_get_tuning()["wave_dmax"]
    in_tier = [(d_id >= kdom - 1) & (d_id <= wd), d_id > wd, np.zeros(n, bool)]
    inter = float(w_id[in_tier[dom]].sum())
    ms = t_tier[dom]
    achieved = 4.0 * inter / (ms * 1e-3) if ms > 0 else None
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        # the profile summary carries the per-launch bytes as one indented JSON line
        for line in open(args.traffic):
            if line.startswith("    {"):
                traffic = json.loads(line).get(f"{tier_names[dom].split()[0]}<{kdom}>")
    roofline = {"bound": "alu", "kernel": f"{tier_names[dom]}<{kdom}>", "achieved": achieved, "peak": INT_PEAK,
                "unit": "int32 op/s", "frac": (achieved / INT_PEAK) if achieved else None, "traffic": traffic,
                "ms_per_launch": ms, "work": f"4 ops x {inter:.6g} intersections (roots of the tier, k={kdom})"}

    out = {
        "metric": METRIC, "value": value, "unit": "k-cliques/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": el.name, "n": el.n, "m_in": el.m_in, "m": info[1], "max_outdeg": info[2],
                   "ks": ks, "schedule": args.schedule,
                   "colour_estimate": {"k": ck, "c": cc, "seed": cseed, "scheme": "per_root", "raw": est.raw,
                                       "estimate": est.estimate}},
        "per_k": per_k, "roofline": roofline, "pair_sampling": pair_sampling,
    }

    if not args.no_cpu_baseline:
        import oracle as O
        threads = len(os.sched_getaffinity(0))
        threads = min(threads, 16)
        log(f"cpu baseline: oracle with {threads} threads")
        c0 = time.perf_counter()
        og = O.OracleGraph.from_edgelist(el)
        c1 = time.perf_counter()
        cq = {}
        for k in ks:
            cq[k] = og.count(k, threads=threads)
        c2 = time.perf_counter()
        ok = all(cq[k] == qs[k] for k in ks)
        out["cpu_baseline"] = {"value": sum(cq.values()) / (c2 - c0), "unit": "k-cliques/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"whole workload: build + exact q_k for k={ks} "
                                         f"({c1 - c0:.1f}s build, {c2 - c1:.1f}s counts); "
                                         f"counts {'equal' if ok else 'DIFFER'} to the GPU's"}
    if not args.no_extras:
        if args.batch_graphs > 0:
            out["batch"] = bench_batch(args, K, torch, stream)
        K.kc_set_tuning(defaults=True)  # the batch's tuning does not carry over
        out["schedule"] = bench_schedule(args, K, torch, stream)
    print(json.dumps(out), flush=True)


def _device_graph(K, torch, el, stream):
    import numpy as np
    dev = torch.device("cuda:0")
    src = torch.from_numpy(el.src.view(np.int32)).to(dev)
    dst = torch.from_numpy(el.dst.view(np.int32)).to(dev)
    torch.cuda.synchronize()
    h = K.kc_graph_create(src.data_ptr(), dst.data_ptr(), el.m_in, el.n, True, stream)
    K.kc_orient(h)
    return h


def bench_batch(args, K, torch, stream):
    """s/graph for the batch of Chung-Lu graphs at k=5: one batched, graph-captured
    count sequence against one count call per graph."""
    import graphgen as G
    k = 5
    log(f"batch: generating {args.batch_graphs} graphs")
    els = G.workload_batch(args.batch_graphs)
    # a dedicated stream: launches on it can be captured in a HIP graph
    bs = torch.cuda.Stream()
    with torch.cuda.stream(bs):
        hs = [_device_graph(K, torch, el, bs.cuda_stream) for el in els]
        log("batch: autotuning")
        # optional autotune cache file (KC_TUNE_CACHE); without it every run tunes afresh
        tuning = K.kc_autotune(hs, k, os.environ.get("KC_TUNE_CACHE") or None)
        t0 = time.perf_counter()
        per_graph = [K.kc_count(h, k) for h in hs]
        t1 = time.perf_counter()
        t2 = time.perf_counter()
        batched = K.kc_count_batch(hs, k)  # plan (concatenation, queue, staging), eager run, capture
        t_first = time.perf_counter() - t2
        reps = []
        for _ in range(5):
            t2 = time.perf_counter()
            batched = K.kc_count_batch(hs, k)
            reps.append(time.perf_counter() - t2)
        for h in hs:
            K.kc_graph_destroy(h)
    reps.sort()
    tb = reps[len(reps) // 2]
    return {"workload": f"{len(els)} Chung-Lu graphs, exponent 2.3, mean 20, n log-uniform in [1000, 200000]",
            "k": k, "nodes": sum(el.n for el in els), "edges_in": sum(el.m_in for el in els),
            "q_total": int(sum(batched)), "counts_equal": batched == per_graph,
            "s_per_batch": tb, "s_per_graph": tb / len(els),
            "s_per_batch_per_graph_calls": t1 - t0, "speedup_vs_per_graph_calls": (t1 - t0) / tb,
            "s_first_batch_call": t_first,
            "tuning": tuning}


def bench_schedule(args, K, torch, stream):
    """Learned vs degree-binned schedule on the planted-clique Chung-Lu graph:
    same kernels and counts, only the queue order and tiers differ."""
    import tempfile
    import graphgen as G
    ks = [int(x) for x in args.sched_ks.split(",")]
    log("schedule: training the MLP on the ER 2000 and Chung-Lu 1M graphs")
    train = [_device_graph(K, torch, G.workload_er2000(), stream),
             _device_graph(K, torch, G.workload_chung_lu_1m(), stream)]
    wpath = os.path.join(tempfile.mkdtemp(), "sched.bin")
    t0 = time.perf_counter()
    loss = K.kc_train_schedule(train, max(ks), 20, 1, wpath)
    t_train = time.perf_counter() - t0
    for h in train:
        K.kc_graph_destroy(h)
    log("schedule: planted workload")
    el = G.workload_planted()
    h = _device_graph(K, torch, el, stream)
    res = {"workload": el.name, "train_loss": loss, "train_seconds": t_train, "per_k": {}}
    tot = {"degree": 0.0, "learned": 0.0}
    for k in ks:
        row = {}
        for name, pol in (("degree", K.KC_SCHED_DEGREE), ("learned", K.KC_SCHED_LEARNED)):
            K.kc_set_schedule(h, pol, wpath if pol == K.KC_SCHED_LEARNED else None)
            q = K.kc_count(h, k)  # warm-up (builds cached structures)
            ts = []
            for _ in range(3):
                q = K.kc_count(h, k)
                ts.append(K.kc_last_timings(h)[2])
            ts.sort()
            row[name] = {"q": q, "ms": ts[1]}
            tot[name] += ts[1]
        row["equal"] = row["degree"]["q"] == row["learned"]["q"]
        row["speedup"] = row["degree"]["ms"] / row["learned"]["ms"] if row["learned"]["ms"] > 0 else None
        res["per_k"][str(k)] = row
        log(f"schedule k={k}: degree {row['degree']['ms']:.2f} ms, learned {row['learned']['ms']:.2f} ms")
    K.kc_graph_destroy(h)
    res["ms_total_degree"] = tot["degree"]
    res["ms_total_learned"] = tot["learned"]
    res["speedup"] = tot["degree"] / tot["learned"] if tot["learned"] > 0 else None
    return res


if __name__ == "__main__":
    main()
