"""Throughput benchmark: exact 36-motif counting.

Default workload: the power-law graph (1M nodes, 20M edges, delta 3600).  One
step = the whole counting path on one synthetic graph already resident in
HBM: build the device graph (validate, time sort, per-node sequences S_u,
node-pair edge sets) from device pointers, count every motif for each delta
of the workload (star/pair sweeps, triangle kernel, reduction), copy the 36
counts back.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload powerlaw|tiny|skewed|batch|serve|stream]

Prints one JSON line.  ``value`` = edges counted per second over the K timed
steps (m x number of deltas per step, wall clock bracketed by device
synchronisation).  ``roofline`` is measured for the kernel with the largest
share of GPU time: K traced steps first record HIP events around every launch
on its stream (the per-kernel table), then the K timed steps trace only that
kernel, whose launch durations inside the timed region give ``achieved``;
algorithmic bytes per launch come from ``byte_model``; ``traffic`` is the HBM bytes per launch from
rocprofv3 counters, read from the committed summary under profiles/ when it
was taken from the current kernel sources.  ``cpu_baseline`` is the CPU
oracle (test infrastructure: the paper's Algorithms 1 and 2, OpenMP over
centers) timed on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "temporal edges/s counted (exact 36 motifs), %HBM peak; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="powerlaw",
                    choices=["powerlaw", "tiny", "skewed", "batch", "serve", "stream"])
    ap.add_argument("--stream-batch", type=int, default=1_000_000,
                    help="stream workload: edges per append")
    ap.add_argument("--serve-pool", type=int, default=128, help="graphs in the serving pool")
    ap.add_argument("--serve-mhi", type=float, default=5e7,
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
    ap.add_argument("--cpu-sample", type=float, default=0.05,
                    help="skewed workload: fraction of the time span the CPU baseline counts")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner pass before warm-up (library defaults)")
    ap.add_argument("--untraced", action="store_true",
                    help="time the steps without the per-launch event tracer (no roofline)")
    return ap.parse_args()


HUB_MIN_DEFAULT, HUB_CAP, HUB_SLICE = 32, 2048, 512


def window_stats(src, dst, t, delta: int, hub_min: int = HUB_MIN_DEFAULT) -> dict:
    """Delta-window facts of a graph, for the triangle kernels' byte models
    (measurement only, outside the timed region).  Entries of S_u are ordered
    by (node, t, edge id): interleaving the two entries of each edge by edge id
    and sorting stably by (node, t) gives that order.  W(p) = later entries of
    the same S_u within delta; a triangle candidate is an edge with non-empty
    windows after it at both endpoints.  Candidates whose larger window is at
    least hub_min and whose smaller one is below HUB_CAP go to the slice
    kernel: they belong to the position with the larger window (the source
    side on a tie), and each HUB_SLICE-position slice of S holding such
    owners reads the union of their windows once."""
    import torch
    m = src.numel()
    if m == 0:
        return {k: 0 for k in ("sum_w", "max_w", "cand", "sum_cand_w", "sum_cand_prod", "reg_cand",
                                "reg_sum_w", "hub_cand", "hub_probes", "hub_tiles", "hub_union")}
    t0 = t - t.min()
    tb = max(int(t0.max().item() + delta).bit_length(), 1)
    node = torch.stack([src, dst], 1).reshape(-1).long()
    tt = torch.stack([t0, t0], 1).reshape(-1)
    key = (node << tb) | tt
    skey, perm = torch.sort(key, stable=True)
    del key
    R = torch.searchsorted(skey, skey + delta, right=True) - 1
    W = R - torch.arange(2 * m, device=R.device)
    del R, skey
    pos = torch.empty_like(perm)
    pos[perm] = torch.arange(2 * m, device=perm.device)
    ps, pd = pos[0::2], pos[1::2]
    ws, wd = W[ps], W[pd]
    cand = (ws > 0) & (wd > 0)
    big, small = torch.maximum(ws, wd), torch.minimum(ws, wd)
    hub = cand & (big >= hub_min) & (small < HUB_CAP)
    reg = cand & ~hub
    own = torch.where(ws >= wd, ps, pd)[hub]
    ow = big[hub]
    tile = own // HUB_SLICE
    n_tiles = (2 * m + HUB_SLICE - 1) // HUB_SLICE
    lo = torch.full((n_tiles,), 2 * m, dtype=torch.long, device=own.device)
    hi = torch.full((n_tiles,), -1, dtype=torch.long, device=own.device)
    lo.scatter_reduce_(0, tile, own + 1, reduce="amin")
    hi.scatter_reduce_(0, tile, own + ow, reduce="amax")
    used = hi >= 0
    return {"sum_w": int(W.sum().item()), "max_w": int(W.max().item()),
            "cand": int(cand.sum().item()),
            "sum_cand_w": int((ws + wd)[cand].sum().item()),
            "sum_cand_prod": int((ws * wd)[cand].sum().item()),
            "reg_cand": int(reg.sum().item()),
            "reg_sum_w": int((ws + wd)[reg].sum().item()),
            "hub_cand": int(hub.sum().item()),
            "hub_probes": int(small[hub].sum().item()),
            "hub_tiles": int(used.sum().item()),
            "hub_union": int((hi - lo + 1)[used].sum().item())}


def byte_model(m: int, n: int, info: dict, ws: dict | None, passes: dict) -> dict:
    """Algorithmic bytes per launch of each kernel: what its access pattern
    must read and write at least once (reads + writes).  m edges, 2m incident
    entries, n nodes, tk = time-sort key width, me = edges on node pairs with
    >= 2 edges, nm = such pairs.  Radix scatter passes read and write every
    (key, value) pair once; histogram passes read every key once.  The time
    sort of one graph reads the input arrays (src, dst, t: 16 B per edge) in
    its histogram and first pass, and its last pass writes the rank-ordered
    arrays (t, input index, the two node-sort entries, pair key and value:
    64 B per edge).  The node sort's last pass writes the sequence arrays
    (node, t, other end | dir, rank) and each edge's two positions instead
    of the ping-pong buffers."""
    e2 = 2 * m
    tk = 4 if info["tbits"] <= 32 else 8
    me, nm = info["multi_pair_edges"], info["multi_pairs"]
    pn = max(passes["node"], 1)
    node_scatter = (e2 * 40 * (pn - 1) + e2 * (20 + 24)) / pn
    pt = max(passes["time"], 1)
    time_first = 16 + ((tk + 12) if pt > 1 else 64)
    time_scatter = (m * time_first + m * (tk + 12) * 2 * max(pt - 2, 0) +
                    (m * (tk + 12 + 64) if pt > 1 else 0)) / pt
    table = {
        "validate": m * 16,
        "time_keys": m * (16 + tk + 12),   # batches only
        "sort_time_hist": m * 8,
        "sort_time_scatter": time_scatter,
        "sort_node_hist": e2 * 4,
        "sort_node_scatter": node_scatter,
        "offsets_fill": (n + 1) * 4,
        "offsets": e2 * 4 + (n + 1) * 4,
        "sort_pair_hist": m * 8,
        "sort_pair_scatter": m * (8 + 4) * 2,
        "multi_flags": m * (8 + 8),
        "multi_fill": m * 28 + me * (32 + 33) + nm * 12,
        # keys read, window ends and starts written; one graph: the three
        # window bit planes too
        "windows": e2 * 20 + (n + 1) * 4 + e2 / 8 + e2 / 4,
        # per element its record, per side X at p, R + 1 and L, Wf, Lf, result
        "star_prep": me * 32 + 2 * me * 36,
        "star_pair": me * 25 + 2 * me * 16,
        "wlevels": e2 * 4 + e2 / 8 + e2 / 4,
        "tri_flags": m * (8 + 4) + e2 / 8,
        "hub_tiles": e2 / 4 + e2 / HUB_SLICE * 64,
    }
    if ws is not None:
        # per-candidate kernel: its candidates' record and both windows
        # (neighbour | dir and rank, 8 B an entry)
        table["tri_compact"] = m * 8 + ws["reg_cand"] * (8 + 8 + 16)
        table["triangles"] = ws["reg_cand"] * 16 + ws["reg_sum_w"] * 8
        # slice kernel: per owner its W, rank, edge positions and the other
        # W (20 B); per probe one entry of the smaller window; per slice the
        # union of its owners' windows once and a row of 8 counters
        table["tri_hub"] = (ws["hub_cand"] * 20 + ws["hub_probes"] * 8 + ws["hub_union"] * 8 +
                            ws["hub_tiles"] * 64)
    return table


def kernel_table(prof: dict, model: dict) -> tuple[dict, str | None]:
    kernels = {}
    for k, (launches, total_ms) in prof.items():
        row = {"launches": launches, "total_ms": round(total_ms, 4),
               "avg_ms": round(total_ms / max(launches, 1), 5)}
        b = model.get(k)
        if b is not None and total_ms > 0:
            gbs = b / (total_ms / launches / 1e3) / 1e9
            row.update({"bytes_per_launch": int(b), "achieved_GBs": round(gbs, 1),
                        "frac": round(gbs / HBM_PEAK_GBS, 4)})
        kernels[k] = row
    dominant = max(prof.items(), key=lambda kv: kv[1][1])[0] if prof else None
    return kernels, dominant


COUNT_KERNELS = ("windows", "star_prep", "item_counts", "item_pairs", "star_pair", "wlevels",
                 "tri_flags", "tri_compact", "triangles", "hub_tiles", "tri_hub", "graph_tiles",
                 "graph_sums", "graph_sums_fin")


def kernel_sources(kernel: str) -> list[str]:
    """The HIP source files that define a traced kernel."""
    if kernel.startswith("sort_") or kernel.startswith("scan_"):
        return ["prim.hip", "tm_internal.h"]
    if kernel in COUNT_KERNELS:
        return ["count.hip", "tm_internal.h"]
    return ["build.hip", "tm_internal.h"]


def source_digest(kernel: str) -> str:
    """sha256 over the sources of one kernel: a stored counter reading
    applies only to the code it was taken from."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2204_09236_amd", "csrc")
    for f in kernel_sources(kernel):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, workload: str) -> dict | None:
    """HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by
    a copy kernel of known size, read from the committed counter summary of
    (kernel, workload) if it was taken from the current sources."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                a, b = line.split("=", 1)
                kv[a.strip()] = b.strip()
    if kv.get("source_digest") != source_digest(kernel):
        return None
    try:
        return {"bytes": float(kv["traffic_bytes_per_launch"]),
                "fetch_kib": float(kv["fetch_kib_per_launch"]),
                "write_kib": float(kv["write_kib_per_launch"]),
                "copy_factor": float(kv["copy_factor"])}
    except (KeyError, ValueError):
        return None


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
        "metric": METRIC, "value": round(m_total / el_b, 1), "unit": "edges/s",
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


def bench_stream(args):
    """Incremental counting: the power-law graph (20M edges, delta 3,600)
    appended in time order, --stream-batch edges per append (tm_stream_*,
    device pointers).  A step is the whole stream: every append returns the
    instances whose last edge is new.  The totals must equal the stored
    oracle count of the whole graph; the alternative without incremental
    counting, a build and count of the whole prefix after every batch, is
    timed once beside it."""
    import numpy as np
    import torch

    import graphgen
    import paper_2204_09236_amd as tm

    delta = 3600
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = graphgen.powerlaw()
    o = np.argsort(g.t, kind="stable")   # time order; ties keep their id order
    src, dst, tt = (torch.from_numpy(np.ascontiguousarray(a[o])).to(dev) for a in (g.src, g.dst, g.t))
    del o
    m = g.m
    cuts = list(range(0, m, args.stream_batch)) + [m]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def run():
        lat = []
        with tm.Stream(delta, n=g.n, stream=stream) as S:
            for a, b in zip(cuts[:-1], cuts[1:]):
                t0 = time.perf_counter()
                S.append(src[a:b], dst[a:b], tt[a:b])
                lat.append(time.perf_counter() - t0)
            total, _, kept = S.totals()
        return total, lat, kept

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    lats = []
    for _ in range(args.steps):
        total, lat, kept = run()
        lats += lat
    torch.cuda.synchronize()
    el = (time.perf_counter() - t_start) / args.steps
    print(f"[bench] stream: {el * 1e3:.1f} ms per pass", file=sys.stderr, flush=True)
    # without incremental counting: the whole prefix after every batch
    t0 = time.perf_counter()
    for b in cuts[1:]:
        with tm.build_graph(src[:b], dst[:b], tt[:b], n=g.n, stream=stream) as G:
            last = G.count(delta)
    torch.cuda.synchronize()
    el_re = time.perf_counter() - t0
    golden = golden_check("powerlaw", g, [delta], [total])
    same = bool(np.array_equal(total, last))
    lat_ms = np.array(lats) * 1e3
    line = {
        "metric": "appended temporal edges/s counted incrementally (exact 36 motifs)",
        "value": round(m / el, 1), "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "stream", "n": g.n, "m": m, "delta": delta,
                   "edges_per_append": args.stream_batch, "appends": len(cuts) - 1,
                   "parallelism": "single-gpu"},
        "append_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                      "p99": round(float(np.percentile(lat_ms, 99)), 3)},
        "tail_edges_at_end": kept,
        "recount_every_append": {"seconds": round(el_re, 4),
                                 "over_incremental": round(el_re / el, 2)},
        "totals_equal_full_count": same, "golden": golden,
    }
    print(json.dumps(line))
    if not same or (golden is not None and golden.get("match") is False):
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
        "metric": METRIC,
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


COPY_CALIB_BYTES = 256 << 20


def bench_single(args):
    """One graph: a step builds the device graph from device pointers and
    counts every delta of the workload (one for power-law and tiny, three for
    skewed) on it."""
    import numpy as np
    import torch

    import graphgen
    import paper_2204_09236_amd as tm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec = graphgen.CONFIGS[args.workload]
    deltas = list(spec["deltas"])
    t0 = time.time()
    g = spec["fn"]()
    print(f"[bench] generated {args.workload}: n={g.n} m={g.m} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    src = torch.from_numpy(g.src).to(dev)
    dst = torch.from_numpy(g.dst).to(dev)
    tt = torch.from_numpy(g.t).to(dev)
    stream = torch.cuda.current_stream()
    # a plain device copy of known size: the reference reading for the
    # FETCH_SIZE / WRITE_SIZE counters of a profiled run of this script
    ca = torch.ones(COPY_CALIB_BYTES // 4, dtype=torch.int32, device=dev)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    del ca, cb
    torch.cuda.synchronize()

    def step():
        G = tm.build_graph(src, dst, tt, n=g.n, stream=stream)
        outs = [G.count(d) for d in deltas]
        G.free()
        return outs

    # the library's autotuner, once, before warm-up and outside the timed
    # region, at the workload's largest delta (the most work): its choice is
    # kept in the process-wide table keyed by graph shape, so the timed
    # steps' freshly built graphs of this shape count with it
    tuned = None
    if not args.no_autotune:
        G0 = tm.build_graph(src, dst, tt, n=g.n, stream=stream)
        tuned = G0.autotune([max(deltas)])
        G0.free()
        print(f"[bench] autotuned at delta {max(deltas)}: {tuned}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        counts = step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    # every launch traced (events around each kernel): the per-kernel table
    # and the kernel with the largest share of GPU time
    tm.prof_reset()
    tm.prof_enable(not args.untraced)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        counts = step()
    torch.cuda.synchronize()
    tm.prof_enable(False)
    prof = tm.prof_read()
    dominant_name = max(prof.items(), key=lambda kv: kv[1][1])[0] if prof else None
    print("[bench] traced steps done", file=sys.stderr, flush=True)

    # the timed steps trace only that kernel (two events per launch of it),
    # so its launch durations come from the timed region itself
    tm.prof_reset()
    tm.prof_only(dominant_name)
    tm.prof_enable(dominant_name is not None)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        counts = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    tm.prof_enable(False)
    tm.prof_only(None)
    prof_timed = tm.prof_read()
    print("[bench] timed steps done", file=sys.stderr, flush=True)
    ms_per_step = elapsed * 1e3 / args.steps
    value = g.m * len(deltas) * args.steps / elapsed

    # build alone and count alone (outside the timed region above)
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    for _ in range(args.steps):
        tm.build_graph(src, dst, tt, n=g.n, stream=stream).free()
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t_b) * 1e3 / args.steps
    # PCIe-inclusive: the same step from host arrays (the boundary copies them in)
    host_reps = max(1, min(args.steps, 3))
    torch.cuda.synchronize()
    t_h = time.perf_counter()
    for _ in range(host_reps):
        Gh = tm.build_graph(g.src, g.dst, g.t, n=g.n)
        for d in deltas:
            Gh.count(d)
        Gh.free()
    torch.cuda.synchronize()
    host_ms = (time.perf_counter() - t_h) * 1e3 / host_reps
    G = tm.build_graph(src, dst, tt, n=g.n, stream=stream)
    info = G.info()
    count_ms = {}
    for d in deltas:
        G.count(d)
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        for _ in range(args.steps):
            G.count(d)
        torch.cuda.synchronize()
        count_ms[str(d)] = round((time.perf_counter() - t_c) * 1e3 / args.steps, 4)
    # one family at a time (tm_count_masked), as the paper times its
    # pair-only and triangle-only variants
    family_ms = {}
    for name, fam in (("stars+pairs", tm.STARS | tm.PAIRS), ("pairs", tm.PAIRS),
                      ("triangles", tm.TRIANGLES)):
        G.count(deltas[0], families=fam)
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        for _ in range(args.steps):
            G.count(deltas[0], families=fam)
        torch.cuda.synchronize()
        family_ms[name] = round((time.perf_counter() - t_c) * 1e3 / args.steps, 4)
    # every delta of the workload in one call (tm_count_multi)
    multi = None
    if len(deltas) > 1:
        mc = G.count_multi(deltas)
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        for _ in range(args.steps):
            mc = G.count_multi(deltas)
        torch.cuda.synchronize()
        multi = {"deltas": deltas, "ms": round((time.perf_counter() - t_c) * 1e3 / args.steps, 4),
                 "sum_of_single_counts_ms": round(sum(count_ms.values()), 4),
                 "equals_step_counts": bool(all(np.array_equal(mc[i], counts[i])
                                                for i in range(len(deltas))))}
    G.free()

    tspan = int(g.t.max() - g.t.min()) if g.m else 0
    info["tbits"] = max(tspan.bit_length(), 1)
    passes = {"node": (max(int(g.n - 1).bit_length(), 1) + 7) // 8,
              "time": (max(info["tbits"], 1) + 7) // 8}
    wstats = {str(d): window_stats(src, dst, tt, d) for d in deltas}
    torch.cuda.empty_cache()
    # count kernels run once per delta: the model averages their bytes over deltas
    model = byte_model(g.m, g.n, info, None, passes)
    tri = {"tri_compact": 0.0, "triangles": 0.0, "tri_hub": 0.0}
    for d in deltas:
        md = byte_model(g.m, g.n, info, wstats[str(d)], passes)
        for k in tri:
            tri[k] += md[k] / len(deltas)
    model.update(tri)
    kernels, dominant = kernel_table(prof, model)
    roofline = None
    if dominant is not None and dominant in prof_timed:
        # the dominant kernel as measured inside the timed steps
        kd = kernel_table({dominant: prof_timed[dominant]}, model)[0][dominant]
    else:
        kd = None
    if kd is not None and "achieved_GBs" in kd:
        tr = stored_traffic(dominant, args.workload)
        roofline = {"kernel": dominant, "bound": "hbm", "achieved": kd["achieved_GBs"],
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kd["frac"],
                    "traffic": None if tr is None else tr["bytes"],
                    "bytes_per_launch": kd["bytes_per_launch"], "avg_launch_ms": kd["avg_ms"]}
        if tr is not None:
            roofline["traffic_over_algorithmic"] = round(tr["bytes"] / kd["bytes_per_launch"], 3)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, g, deltas, counts)
    golden = golden_check(args.workload, g, deltas, counts)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "deltas": deltas,
                   "parallelism": "single-gpu"},
        "roofline": roofline, "cpu_baseline": cpu, "golden": golden,
        "build_only_ms": round(build_ms, 4), "count_only_ms": count_ms,
        "count_only_family_ms": {"delta": deltas[0], **family_ms},
        "count_multi": multi,
        "autotuned": tuned,
        "pcie_inclusive": {"ms_per_step": round(host_ms, 3),
                           "edges_per_s": round(g.m * len(deltas) / (host_ms / 1e3), 1),
                           "note": "inputs in host memory, copied in by tm_build_graph"},
        "count_only_edges_per_s": {d: round(g.m / (v / 1e3), 1) for d, v in count_ms.items()},
        "gpu_kernel_ms_per_step": round(sum(v[1] for v in prof.values()) / args.steps, 4),
        "graph": {k: info[k] for k in ("multi_pairs", "multi_pair_edges", "max_degree")},
        "window_stats": wstats,
        "kernels": kernels,
        "motif_total": [int(c.sum()) for c in counts],
    }
    print(json.dumps(line))
    if (cpu is not None and not cpu["matches_gpu"]) or (golden is not None and not golden["match"]):
        sys.exit(1)


def golden_check(workload, g, deltas, counts):
    """Compare with the oracle's stored counts for this workload
    (tests/golden/<workload>_counts.json, written by make_golden.py from the
    oracle alone) when the regenerated input has the stored sha256."""
    import numpy as np

    import graphgen
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_counts.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("edge_sha256") != graphgen.edge_hash(g):
        return {"match": None, "note": "input differs from the stored one; not compared"}
    ok = True
    for d, c in zip(deltas, counts):
        want = rec["counts"].get(str(d))
        if want is None or not np.array_equal(np.array(want["grid"], dtype=np.uint64), c):
            ok = False
    return {"match": ok, "deltas": deltas, "source": os.path.relpath(path, ROOT)}


def cpu_baseline(args, g, deltas, counts):
    """The CPU oracle (the paper's Algorithms 1 and 2, OpenMP over centers)
    timed on this host.  Power-law and tiny: the whole workload.  Skewed: a
    bounded sample, the edges of the first --cpu-sample fraction of the time
    span (a temporal slice keeps every window of the slice intact), at the
    smallest delta; counts of the sample are not compared."""
    import numpy as np

    import oracle
    threads = args.cpu_threads or min(16, os.cpu_count() or 1)
    if args.workload != "skewed":
        t0 = time.perf_counter()
        want = [oracle.count(g.src, g.dst, g.t, d, n=g.n, threads=threads) for d in deltas]
        cpu_s = time.perf_counter() - t0
        m = g.m * len(deltas)
        sample = (f"whole {args.workload} workload (m={g.m}, deltas={deltas}), one run each, "
                  f"{cpu_s:.1f} s incl. building S_u and E_(v,w)")
        match = all(np.array_equal(a, b) for a, b in zip(want, counts))
    else:
        lim = int(g.t.min()) + int((int(g.t.max()) - int(g.t.min())) * args.cpu_sample)
        sel = g.t <= lim
        s, d, t = g.src[sel], g.dst[sel], g.t[sel]
        t0 = time.perf_counter()
        oracle.count(s, d, t, deltas[0], n=g.n, threads=threads)
        cpu_s = time.perf_counter() - t0
        m = int(s.size)
        sample = (f"edges with t in the first {args.cpu_sample:.0%} of the span (m={m}), "
                  f"delta={deltas[0]}, {cpu_s:.1f} s incl. building S_u and E_(v,w)")
        match = True
    return {"value": round(m / cpu_s, 1), "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": sample, "matches_gpu": bool(match)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are "
                          "not supported (the path would shard by center)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "stream":
        return bench_stream(args)
    return bench_single(args)


if __name__ == "__main__":
    main()
