"""Write full-size expected counts for a seeded workload.

Calls only the CPU oracle (and the seeded generator): the stored raw counters
are the paper's Algorithms 1 and 2 run on the regenerated input, tagged with
the sha256 of the input arrays so a test can tell whether it regenerated the
same edge list.

    python tests/golden/make_golden.py [workload] [threads]

``workload``:
  powerlaw, skewed  the named single-graph workloads at every delta of theirs
  batch             a seeded sample of 256 graphs of the 4,096-graph batch
                    (graphgen.batch_sample: the 20 largest, the 10 widest
                    windows, the 10 smallest, the rest uniform), each at its
                    own delta
  serve             the largest serving request graph (graphgen.serve_max,
                    5e7 edges) at delta 60, 3,600 and 86,400
  motif4            four-node three-edge motif counts (oracle.local4) with the
                    raw three-edge counters of the same delta (oracle.alg):
                    the power-law workload at delta 600 and 3,600, the skewed
                    one at delta 600
The file written is ``tests/golden/<workload>_counts.json``.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402

SERVE_DELTAS = [60, 3600, 86400]
MOTIF4 = {"powerlaw": [600, 3600], "skewed": [600]}


def counts_record(g, deltas, threads):
    out = {}
    for delta in deltas:
        t0 = time.time()
        raw = oracle.alg(g.src, g.dst, g.t, delta, n=g.n, threads=threads)
        grid = oracle.merge(raw)
        out[str(delta)] = {"raw": [int(x) for x in raw],
                           "grid": [[int(x) for x in row] for row in grid],
                           "oracle_seconds": round(time.time() - t0, 2)}
        print(f"delta={delta}: {time.time() - t0:.1f}s", flush=True)
    return out


def single(workload, threads):
    if workload == "serve":
        gen, deltas = graphgen.serve_max, SERVE_DELTAS
    else:
        spec = graphgen.CONFIGS[workload]
        gen, deltas = spec["fn"], spec["deltas"]
    t0 = time.time()
    g = gen()
    print(f"generated {workload}: n={g.n} m={g.m} in {time.time() - t0:.1f}s", flush=True)
    rec = {"workload": workload, "n": g.n, "m": g.m, "edge_sha256": graphgen.edge_hash(g),
           "counts": counts_record(g, deltas, threads)}
    return rec


def batch(threads):
    spec = graphgen.batch_spec()
    idx = graphgen.batch_sample(spec)
    rec = {"workload": "batch", "graphs_in_batch": len(spec), "sample": "graphgen.batch_sample",
           "members": []}
    t_all = time.time()
    for k, i in enumerate(idx):
        it = spec[i]
        g = graphgen.batch_graph(it)
        t0 = time.time()
        raw = oracle.alg(g.src, g.dst, g.t, it.delta, n=g.n, threads=threads)
        rec["members"].append({"index": i, "m": g.m, "n": g.n, "delta": it.delta,
                               "edge_sha256": graphgen.edge_hash(g),
                               "raw": [int(x) for x in raw],
                               "oracle_seconds": round(time.time() - t0, 3)})
        if k % 32 == 0:
            print(f"member {k}/{len(idx)} (graph {i}, m={g.m}, delta={it.delta})", flush=True)
    print(f"batch sample: {len(idx)} graphs in {time.time() - t_all:.1f}s", flush=True)
    return rec


def motif4(threads):
    rec = {}
    for workload, deltas in MOTIF4.items():
        t0 = time.time()
        g = graphgen.CONFIGS[workload]["fn"]()
        print(f"generated {workload}: n={g.n} m={g.m} in {time.time() - t0:.1f}s", flush=True)
        counts = {}
        for delta in deltas:
            t0 = time.time()
            f4 = oracle.local4(g.src, g.dst, g.t, delta, n=g.n, threads=threads)
            raw = oracle.alg(g.src, g.dst, g.t, delta, n=g.n, threads=threads)
            counts[str(delta)] = {"f4": [int(x) for x in f4], "raw": [int(x) for x in raw],
                                  "oracle_seconds": round(time.time() - t0, 2)}
            print(f"{workload} delta={delta}: {time.time() - t0:.1f}s", flush=True)
        rec[workload] = {"n": g.n, "m": g.m, "edge_sha256": graphgen.edge_hash(g), "counts": counts}
        del g
    return rec


def main():
    workload = sys.argv[1] if len(sys.argv) > 1 else "powerlaw"
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    if workload == "batch":
        rec = batch(threads)
    elif workload == "motif4":
        rec = motif4(threads)
    else:
        rec = single(workload, threads)
    with open(os.path.join(HERE, f"{workload}_counts.json"), "w") as f:
        json.dump(rec, f, indent=None if workload == "batch" else 1, separators=None)
    if workload != "motif4":
        print(json.dumps({k: v for k, v in rec.items() if k not in ("counts", "members")}))


if __name__ == "__main__":
    main()
