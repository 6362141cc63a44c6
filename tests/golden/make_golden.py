"""Write full-size expected counts for a seeded workload.

Calls only the CPU oracle (and the seeded generator): the stored raw counters
are the paper's Algorithms 1 and 2 run on the regenerated input, tagged with
the sha256 of the input arrays so a test can tell whether it regenerated the
same edge list.

    python tests/golden/make_golden.py [workload] [threads]

``workload`` is ``powerlaw`` (default) or ``skewed``; the file written is
``tests/golden/<workload>_counts.json``.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402


def main():
    workload = sys.argv[1] if len(sys.argv) > 1 else "powerlaw"
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    spec = graphgen.CONFIGS[workload]
    t0 = time.time()
    g = spec["fn"]()
    h = graphgen.edge_hash(g)
    print(f"generated {workload}: n={g.n} m={g.m} in {time.time() - t0:.1f}s", flush=True)
    rec = {"workload": workload, "n": g.n, "m": g.m, "edge_sha256": h, "counts": {}}
    for delta in spec["deltas"]:
        t0 = time.time()
        raw = oracle.alg(g.src, g.dst, g.t, delta, n=g.n, threads=threads)
        grid = oracle.merge(raw)
        rec["counts"][str(delta)] = {"raw": [int(x) for x in raw],
                                     "grid": [[int(x) for x in row] for row in grid],
                                     "oracle_seconds": round(time.time() - t0, 2)}
        print(f"delta={delta}: {time.time() - t0:.1f}s", flush=True)
    with open(os.path.join(HERE, f"{workload}_counts.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: v for k, v in rec.items() if k != "counts"}))


if __name__ == "__main__":
    main()
