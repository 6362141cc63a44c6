"""Throughput benchmark: exact 36-motif counting of the power-law workload.

One step = the whole counting path on one synthetic graph already resident
in HBM: build the device graph (validate, time sort, per-node sequences S_u,
node-pair edge sets) from device pointers, count every motif for one delta
(star/pair sweeps, triangle kernel, reduction), copy the 36 counts back.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.  ``value`` = edges counted per second over the K timed
steps (wall clock, bracketed by device synchronisation).  ``roofline`` is
measured for the kernel with the largest share of GPU time, from HIP events
the library records around every launch on the launch stream during the
timed steps; its algorithmic bytes per launch are modelled below.
``cpu_baseline`` is the CPU oracle (test infrastructure, paper's Algorithms
1 and 2, OpenMP over centers) timed on this host on the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "temporal edges/s counted (exact 36 motifs)"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="powerlaw", choices=["powerlaw", "tiny", "batch", "serve"])
    ap.add_argument("--serve-pool", type=int, default=128, help="graphs in the serving pool")
    ap.add_argument("--serve-mhi", type=float, default=5e6,
                    help="largest edge count of a pool graph (log-uniform from 1e3)")
    ap.add_argument("--serve-rates", default="50,100,200,500,1000,2000")
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="arrival window per rate (at most --serve-max requests)")
    ap.add_argument("--serve-max", type=int, default=1000)
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--batch-mhi", type=float, default=2e6,
                    help="largest per-graph edge count of the batch workload (log-uniform from 1e3)")
    ap.add_argument("--procs", type=int, default=16, help="generator processes (batch workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--untraced", action="store_true",
                    help="time the steps without the per-launch event tracer (no roofline)")
    return ap.parse_args()


def algorithmic_bytes(name: str, m: int, info: dict) -> float | None:
    """Minimum bytes one launch of ``name`` must move (reads + writes) on this
    workload.  Radix scatter passes read and write every (key, value) pair
    once; histogram passes read every key once."""
    e2 = 2 * m
    tk = 4 if info["tbits"] <= 32 else 8
    me = info["multi_pair_edges"]
    table = {
        "sort_time_scatter": m * (tk + 12) * 2,      # key + (src, dst, id)
        "sort_time_hist": m * tk,
        "sort_node_scatter": e2 * (4 + 8) * 2,       # node + (rank, other end, dir)
        "sort_node_hist": e2 * 4,
        "sort_pair_scatter": m * (8 + 4) * 2,        # pair key + rank
        "sort_pair_hist": m * 8,
        "fill_seq": e2 * (8 + 8 + 8 + 4 + 4 + 4),    # read value, t; write t, nd, rank, epos
        "rank": m * (tk + 12 + 8 + 4 + 8 + 16 + 8 + 4),
        "windows": e2 * (4 + 8 + 4),                 # center, t -> window length
        "star_prep": 2 * me * (8 + 8 + 8 + 4 + 16),
        "star_pair": me * 2 * (8 + 1 + 8 + 16),
        "tri_flags": m * (8 + 4 + 4 + 4),
        "validate": m * 16,
        "time_keys": m * (16 + tk + 12),
    }
    return table.get(name)


def _gen_batch_member(item):
    import graphgen
    g = graphgen.batch_graph(item)
    return g.src, g.dst, g.t, g.n


def bench_batch(args):
    """Batched vs per-graph counting of many uneven graphs, each with its own
    delta.  Batched step = one build of all graphs (tm_build_batch from
    device pointers) + one count (tm_count_batch, a captured hipGraph) + free.
    Per-graph = tm_build_graph + tm_count + free for every graph in turn.
    Both must give identical counts."""
    import multiprocessing as mp

    import numpy as np
    import torch

    import graphgen
    import paper_2204_09236_amd as tm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = graphgen.batch_spec(seed=3, graphs=args.batch_graphs, m_hi=args.batch_mhi)
    t0 = time.time()
    with mp.get_context("fork").Pool(args.procs) as pool:
        members = pool.map(_gen_batch_member, spec, chunksize=8)
    deltas = np.array([it.delta for it in spec], np.int64)
    G = len(members)
    off = np.zeros(G + 1, np.uint64)
    off[1:] = np.cumsum([mb[0].size for mb in members])
    m_total = int(off[-1])
    print(f"[bench] generated batch: G={G} edges={m_total} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    ncount = np.array([mb[3] for mb in members], np.uint32)
    src = torch.from_numpy(np.concatenate([mb[0] for mb in members])).to(dev)
    dst = torch.from_numpy(np.concatenate([mb[1] for mb in members])).to(dev)
    tt = torch.from_numpy(np.concatenate([mb[2] for mb in members])).to(dev)
    del members
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def batched():
        B = tm.build_batch_arrays(src, dst, tt, off, ncount, stream=stream)
        out = B.count_batch(deltas)
        B.free()
        return out

    for _ in range(args.warmup):
        res_b = batched()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        res_b = batched()
    torch.cuda.synchronize()
    el_b = (time.perf_counter() - t_start) / args.steps
    print(f"[bench] batched: {el_b * 1e3:.1f} ms per batch", file=sys.stderr, flush=True)

    def per_graph():
        outs = []
        for i in range(G):
            a, b = int(off[i]), int(off[i + 1])
            Gi = tm.build_graph(src[a:b], dst[a:b], tt[a:b], n=int(ncount[i]), stream=stream)
            outs.append(Gi.count(int(deltas[i])))
            Gi.free()
        return np.stack(outs)

    res_p = per_graph()  # warm-up pass
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    res_p = per_graph()
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t_start
    same = bool(np.array_equal(res_b, res_p))
    line = {
        "metric": METRIC + ", batched", "value": round(m_total / el_b, 1), "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el_b * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "batch", "graphs": G, "edges": m_total,
                   "m_range": [1000, args.batch_mhi], "delta_range": [60, 86400],
                   "parallelism": "single-gpu"},
        "per_graph": {"value": round(m_total / el_p, 1), "unit": "edges/s",
                      "seconds": round(el_p, 3)},
        "batched_over_per_graph": round(el_p / el_b, 2),
        "identical_counts": same,
        "motif_total": int(res_b.sum()),
    }
    print(json.dumps(line))
    if not same:
        sys.exit(1)


def bench_serve(args):
    """Serving: Poisson arrivals of (pool graph, delta) requests at each rate;
    keyed graphs stay resident after their first request.  Latency = done -
    submit on the server's clock; edges/s = edges of the completed requests /
    (last done - first submit).  Every result is compared with the same
    request counted alone."""
    import math
    import multiprocessing as mp

    import numpy as np
    import torch

    import graphgen
    import paper_2204_09236_amd as tm

    torch.cuda.set_device(0)
    rng = np.random.default_rng(4)
    ms = np.rint(np.exp(rng.uniform(math.log(1e3), math.log(args.serve_mhi), args.serve_pool)))
    kids = np.random.SeedSequence(4).spawn(args.serve_pool)
    spec = [graphgen.BatchItem(int(m), max(3, int(m) // 20), 0, kids[i]) for i, m in enumerate(ms)]
    t0 = time.time()
    with mp.get_context("fork").Pool(args.procs) as pool_:
        pool = pool_.map(_gen_batch_member, spec, chunksize=2)
    print(f"[bench] serving pool: {len(pool)} graphs, {int(ms.sum())} edges, generated in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    rates = [float(r) for r in args.serve_rates.split(",")]
    budget = int(0.7 * torch.cuda.get_device_properties(0).total_memory)
    S = tm.Server(budget, max_inflight=16)
    alone_graphs = {}
    rows = []
    sent = set()
    for rate in rates:
        n_req = int(min(args.serve_max, max(20, rate * args.serve_seconds)))
        gaps = rng.exponential(1.0 / rate, n_req)
        reqs = [(int(rng.integers(0, len(pool))),
                 int(round(math.exp(rng.uniform(math.log(60), math.log(86400))))))
                for _ in range(n_req)]
        outstanding, done = {}, {}
        start = time.perf_counter()
        t_next = start
        for i, (gi, delta) in enumerate(reqs):
            t_next += gaps[i]
            while True:      # poll finished requests until the next arrival
                for tk in list(outstanding):
                    rc, out, times = S.poll(tk)
                    if rc != tm.tm.TM_EAGAIN:
                        done[outstanding.pop(tk)] = (rc, out, times)
                if time.perf_counter() >= t_next:
                    break
                time.sleep(min(2e-4, max(0.0, t_next - time.perf_counter())))
            src, dst, t, n = pool[gi]
            if gi in sent:
                tk = S.submit(delta, key=gi + 1)
            else:
                tk = S.submit(delta, src, dst, t, n=n, key=gi + 1)
                sent.add(gi)
            outstanding[tk] = i
        for tk, i in outstanding.items():
            done[i] = S.wait(tk)
        lat = np.array([(done[i][2][2] - done[i][2][0]) / 1e6 for i in range(n_req)])
        first_submit = min(done[i][2][0] for i in range(n_req))
        last_done = max(done[i][2][2] for i in range(n_req))
        edges = sum(pool[gi][0].size for gi, _ in reqs)
        ok = all(done[i][0] == 0 for i in range(n_req))
        same = ok
        if ok:
            for i, (gi, delta) in enumerate(reqs):
                if gi not in alone_graphs:
                    src, dst, t, n = pool[gi]
                    alone_graphs[gi] = tm.build_graph(src, dst, t, n=n)
                if not np.array_equal(done[i][1], alone_graphs[gi].count(delta)):
                    same = False
                    break
        row = {"rate": rate, "requests": n_req, "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "edges_per_s": round(edges / ((last_done - first_submit) / 1e9), 1),
               "all_ok": ok, "identical_to_alone": same}
        rows.append(row)
        print(f"[bench] serve rate {rate}: {row}", file=sys.stderr, flush=True)
    st = S.stats()
    S.close()
    for G in alone_graphs.values():
        G.free()
    line = {
        "metric": "p50/p99 request latency and edges/s, served (exact 36 motifs)",
        "value": rows[-1]["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": len(rows),
        "warmup": 0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "serve", "pool_graphs": len(pool), "pool_edges": int(ms.sum()),
                   "m_range": [1000, args.serve_mhi], "delta_range": [60, 86400],
                   "budget_bytes": budget, "max_inflight": 16, "parallelism": "single-gpu"},
        "rates": rows, "server_stats": st,
    }
    print(json.dumps(line))
    if not all(r["identical_to_alone"] for r in rows):
        sys.exit(1)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are "
                          "not supported (the path shards by center, see DESIGN.md)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)

    import numpy as np
    import torch

    import graphgen
    import paper_2204_09236_amd as tm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = graphgen.CONFIGS[args.workload]
    delta = spec["deltas"][0]
    t0 = time.time()
    g = spec["fn"]()
    gen_s = time.time() - t0
    print(f"[bench] generated {args.workload}: n={g.n} m={g.m} in {gen_s:.1f}s", file=sys.stderr,
          flush=True)
    src = torch.from_numpy(g.src).to(dev)
    dst = torch.from_numpy(g.dst).to(dev)
    tt = torch.from_numpy(g.t).to(dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step():
        G = tm.build_graph(src, dst, tt, n=g.n, stream=stream)
        out = G.count(delta)
        G.free()
        return out

    for _ in range(args.warmup):
        counts = step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    tm.prof_reset()
    tm.prof_enable(not args.untraced)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        counts = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    tm.prof_enable(False)
    prof = tm.prof_read()
    print("[bench] timed steps done", file=sys.stderr, flush=True)

    ms_per_step = elapsed * 1e3 / args.steps
    value = g.m * args.steps / elapsed

    # graph facts for the byte model
    with tm.build_graph(src, dst, tt, n=g.n, stream=stream) as G:
        info = G.info()
    tspan = int(g.t.max() - g.t.min())
    info["tbits"] = max(tspan.bit_length(), 1)
    kernels = {k: {"launches": v[0], "total_ms": round(v[1], 4),
                   "avg_ms": round(v[1] / max(v[0], 1), 5)} for k, v in prof.items()}
    gpu_ms = sum(v[1] for v in prof.values()) / args.steps
    dominant = max(prof.items(), key=lambda kv: kv[1][1])[0] if prof else None
    roofline = None
    if dominant is not None:
        launches, total_ms = prof[dominant]
        avg_s = total_ms / launches / 1e3
        b = algorithmic_bytes(dominant, g.m, info)
        if b is not None:
            achieved = b / avg_s / 1e9
            roofline = {"kernel": dominant, "bound": "hbm", "achieved": round(achieved, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": None, "bytes_per_launch": b,
                        "avg_launch_ms": round(avg_s * 1e3, 4)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        t0 = time.perf_counter()
        want = oracle.count(g.src, g.dst, g.t, delta, n=g.n, threads=threads)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": round(g.m / cpu_s, 1), "unit": "edges/s", "cores": threads, "kind": "oracle",
               "sample": f"whole {args.workload} workload (m={g.m}, delta={delta}), one run, "
                         f"{cpu_s:.1f} s incl. building S_u and E_(v,w)",
               "matches_gpu": bool(np.array_equal(want, counts))}

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "delta": delta,
                   "parallelism": "single-gpu"},
        "roofline": roofline, "cpu_baseline": cpu,
        "gpu_kernel_ms_per_step": round(gpu_ms, 4),
        "kernels": kernels,
        "motif_total": int(counts.sum()),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
