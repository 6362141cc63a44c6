"""Write full-size expected counts for the power-law workload.

Calls only the CPU oracle (and the seeded generator): the stored raw counters
are the paper's Algorithms 1 and 2 run on the regenerated input, tagged with
the sha256 of the input arrays so a test can tell whether it regenerated the
same edge list.

    python tests/golden/make_golden.py [threads]
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
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    g = graphgen.powerlaw()
    h = graphgen.edge_hash(g)
    rec = {"workload": "powerlaw", "n": g.n, "m": g.m, "edge_sha256": h, "counts": {}}
    for delta in graphgen.CONFIGS["powerlaw"]["deltas"]:
        t0 = time.time()
        raw = oracle.alg(g.src, g.dst, g.t, delta, n=g.n, threads=threads)
        grid = oracle.merge(raw)
        rec["counts"][str(delta)] = {"raw": [int(x) for x in raw],
                                     "grid": [[int(x) for x in row] for row in grid],
                                     "oracle_seconds": round(time.time() - t0, 2)}
    with open(os.path.join(HERE, "powerlaw_counts.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: v for k, v in rec.items() if k != "counts"}))


if __name__ == "__main__":
    main()
