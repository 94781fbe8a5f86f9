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
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the counting path has no multi-GPU mode in this build "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

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
    # algorithmic work of counting q_k: one neighbourhood intersection per l-clique of
    # every G+(u), l = 1..k-2, i.e. sum_{j=2}^{k-1} q_j intersections, each at least
    # one 64-bit AND and one 64-bit popcount = 4 int32 VALU ops
    inter = info[1] + sum(qs.get(j, 0) for j in range(3, kdom))
    missing = [j for j in range(3, kdom) if j not in qs]
    ms = per_k[str(kdom)]["ms_count"]
    achieved = 4.0 * inter / (ms * 1e-3) if ms > 0 and not missing else None
    roofline = {"bound": "alu", "kernel": f"count stage k={kdom} (k_count_wave/k_count_wg)",
                "achieved": achieved, "peak": INT_PEAK, "unit": "int32 op/s",
                "frac": (achieved / INT_PEAK) if achieved else None, "traffic": None,
                "work": f"4 ops x {inter} intersections"}

    out = {
        "metric": METRIC, "value": value, "unit": "k-cliques/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": el.name, "n": el.n, "m_in": el.m_in, "m": info[1], "max_outdeg": info[2],
                   "ks": ks, "schedule": args.schedule,
                   "colour_estimate": {"k": ck, "c": cc, "seed": cseed, "scheme": "per_root", "raw": est.raw,
                                       "estimate": est.estimate}},
        "per_k": per_k, "roofline": roofline,
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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
