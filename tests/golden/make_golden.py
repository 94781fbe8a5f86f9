"""Write tests/golden/counts.json: exact counts of the benchmark workloads.

Every value comes from the CPU oracle (oracle/) on the seeded generators
(graphgen/); nothing here touches the GPU library.  The digest of each raw
edge list is stored so that a consumer can confirm it regenerated the same bytes.

    python tests/golden/make_golden.py [--only NAME ...]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as G  # noqa: E402
import oracle as O    # noqa: E402

OUT = os.path.join(HERE, "counts.json")

PLAN = {
    "er2000": (G.workload_er2000, [1, 2, 3, 4, 5], [(4, 2), (3, 2)]),
    "chung_lu_1m": (G.workload_chung_lu_1m, [3, 4, 5, 6], [(4, 2), (4, 4), (4, 8), (5, 4), (6, 8)]),
    "planted_4m": (G.workload_planted, [3, 4, 5], [(5, 8)]),
    "rmat22": (G.workload_rmat22, [3, 4], [(4, 8)]),
}
COLOUR_SEED = 11


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name, (fn, ks, colours) in PLAN.items():
        if args.only and name not in args.only:
            continue
        t0 = time.time()
        el = fn()
        g = O.OracleGraph.from_edgelist(el)
        rec = {"digest": el.digest(), "n": g.n, "m_in": el.m_in, "m": g.m,
               "max_outdeg": g.max_outdeg(), "q": {}, "colour": []}
        for k in ks:
            t = time.time()
            rec["q"][str(k)] = g.count(k)
            print(f"{name} k={k} q={rec['q'][str(k)]} ({time.time() - t:.1f}s)", flush=True)
        for k, c in colours:
            for scheme in (O.COLOR_PER_ROOT, O.COLOR_GLOBAL):
                raw = g.count_colored(k, c, COLOUR_SEED, scheme)
                rec["colour"].append({"k": k, "c": c, "seed": COLOUR_SEED, "scheme": scheme, "raw": raw})
                print(f"{name} colour k={k} c={c} scheme={scheme} raw={raw}", flush=True)
        rec["oracle_seconds"] = round(time.time() - t0, 1)
        data[name] = rec
        g.close()
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
