"""Throughput benchmark: exact 36-motif counting.

Default workload: the large skewed graph (10M nodes, 300M edges, 20 %
repeated node pairs, a hub of ~1.25M incident edges), counted at delta 600,
3,600 and 86,400.  One step = the whole counting path on the graph already
resident in HBM: build the device graph (validate, time sort, per-node
sequences S_u, node-pair edge sets) from device pointers, count every motif
for each delta of the workload (star/pair sweeps, triangle kernels,
reduction), copy the counts back.  The power-law graph (1M nodes, 20M edges,
delta 3,600) runs after it and is reported under ``extra_workloads``.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload skewed|powerlaw|tiny|batch|serve|stream]

Prints one JSON line.  ``value`` = edges counted per second over the K timed
steps (m x number of deltas per step, wall clock bracketed by device
synchronisation).

Rooflines use the algorithmic bytes of each step of the path (the per-unit
figures below; m edges, n nodes, P distinct node pairs, per delta):
  a1 ingest + validate   16 B per edge read
  a2 S_u build           16 B per edge read, 40 B per edge written, 8 B per node
  a3 node-pair lists     16 B per edge written, 8 B per pair (index)
  a4 star/pair           40 B per edge (every entry read once)
  a5 triangles           16 B per edge (both window sizes of every edge, the
                         candidate test) + 8 B per entry of the union of the
                         candidates' larger windows (read once) + 8 B per entry
                         of each candidate's smaller window
``rows`` gives, per step of the path, the GPU time per step (HIP events
around every launch, traced in a separate pass of K steps), these bytes and
the fraction of the 8 TB/s HBM peak; ``whole_step`` the same for the whole
step over the timed wall clock.  ``roofline`` is for the kernel with the
largest share of GPU time: its row's algorithmic bytes are split over the
row's kernels in proportion to the bytes each one's access pattern moves
(``byte_model``), and the kernel's launch durations come from the timed
steps themselves (it alone is traced there).  ``traffic`` is the HBM bytes
per launch from rocprofv3 counters, read from the committed summary under
profiles/ when it was taken from the current kernel sources.
``cpu_baseline`` is the CPU oracle (test infrastructure: the paper's
Algorithms 1 and 2, OpenMP over centers) timed on this host on a bounded
time slice of the workload, on one thread and on all usable cores, median of
3 runs each, with its counts compared with the GPU's on the same slice.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "temporal edges/s counted (exact 36 motifs), %HBM peak; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0
ROWS = {"a1": "ingest + validate", "a2": "S_u build (time sort, node sort, offsets)",
        "a3": "node-pair lists", "a4": "star/pair (window kernel, sweeps)", "a5": "triangles",
        "a6": "work items (chunks, tiles, hub slices)", "a7": "reduction"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="skewed",
                    choices=["skewed", "powerlaw", "tiny", "batch", "serve", "stream"])
    ap.add_argument("--extra-workloads", default="powerlaw",
                    help="single-graph workloads timed after the main one (comma list, '' for none)")
    ap.add_argument("--stream-batch", type=int, default=1_000_000,
                    help="stream workload: edges per append")
    ap.add_argument("--serve-pool", type=int, default=128, help="graphs in the serving pool")
    ap.add_argument("--serve-mhi", type=float, default=5e7,
                    help="largest edge count of a pool graph (log-uniform from 1e3)")
    ap.add_argument("--serve-rates", default="50,100,200,500,1000,2000")
    ap.add_argument("--serve-seconds", type=float, default=4.0,
                    help="arrival window per rate (at most --serve-max requests)")
    ap.add_argument("--serve-max", type=int, default=2000)
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--batch-mhi", type=float, default=2e6,
                    help="largest per-graph edge count of the batch workload (log-uniform from 1e3)")
    ap.add_argument("--procs", type=int, default=16, help="generator processes (batch and serve)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=float, default=0.0,
                    help="fraction of the time span the CPU baseline counts (0: the workload's default)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner pass before warm-up (library defaults)")
    ap.add_argument("--separate-counts", action="store_true",
                    help="count each delta with its own tm_count call instead of one tm_count_multi")
    ap.add_argument("--untraced", action="store_true",
                    help="time the steps without the per-launch event tracer (no roofline)")
    return ap.parse_args()


HUB_MIN_DEFAULT, HUB_CAP, HUB_SLICE = 32, 2048, 512


def window_stats(src, dst, t, delta: int, hub_min: int = HUB_MIN_DEFAULT) -> dict:
    """Delta-window facts of a graph, for the byte models of the triangle
    kernels and the algorithmic bytes of the triangle step (measurement
    only, outside the timed region).  Entries of S_u are ordered by (node, t,
    edge id): interleaving the two entries of each edge by edge id and sorting
    stably by (node, t) gives that order.  W(p) = later entries of the same
    S_u within delta; a triangle candidate is an edge with non-empty windows
    after it at both endpoints.  ``union`` counts the entries that lie in the
    larger window of at least one candidate, ``sum_cand_min`` the entries of
    the candidates' smaller windows.  Candidates whose larger window is at
    least hub_min and whose smaller one is below HUB_CAP go to the slice
    kernel: they belong to the position with the larger window (the source
    side on a tie), and each HUB_SLICE-position slice of S holding such
    owners reads the union of their windows once."""
    import torch
    m = src.numel()
    keys = ("sum_w", "max_w", "cand", "sum_cand_w", "sum_cand_min", "union", "sum_cand_prod",
            "reg_cand", "reg_sum_w", "hub_cand", "hub_probes", "hub_tiles", "hub_union")
    if m == 0:
        return {k: 0 for k in keys}
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
    own_all = torch.where(ws >= wd, ps, pd)
    # union of the candidates' larger windows (own, own + big]
    diff = torch.zeros(2 * m + 2, dtype=torch.int32, device=W.device)
    oc, bc = own_all[cand], big[cand]
    diff.index_add_(0, oc + 1, torch.ones_like(oc, dtype=torch.int32))
    diff.index_add_(0, oc + bc + 1, torch.full_like(oc, -1, dtype=torch.int32))
    union = int((torch.cumsum(diff, 0) > 0).sum().item())
    del diff, oc, bc
    hub = cand & (big >= hub_min) & (small < HUB_CAP)
    reg = cand & ~hub
    own = own_all[hub]
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
            "sum_cand_min": int(small[cand].sum().item()),
            "union": union,
            "sum_cand_prod": int((ws * wd)[cand].sum().item()),
            "reg_cand": int(reg.sum().item()),
            "reg_sum_w": int((ws + wd)[reg].sum().item()),
            "hub_cand": int(hub.sum().item()),
            "hub_probes": int(small[hub].sum().item()),
            "hub_tiles": int(used.sum().item()),
            "hub_union": int((hi - lo + 1)[used].sum().item())}


def distinct_pairs(src, dst) -> int:
    """Number of distinct unordered node pairs (the index of the pair lists)."""
    import torch
    lo = torch.minimum(src, dst).long()
    hi = torch.maximum(src, dst).long()
    return int(torch.unique(lo * (int(hi.max().item()) + 1) + hi).numel())


def row_bytes(m: int, n: int, pairs: int, wstats: dict, deltas: list[int]) -> dict:
    """Algorithmic bytes of each step of the path for one step of the
    benchmark (every delta of the workload counted once); see the module
    docstring for the per-unit figures."""
    a5 = 0
    for d in deltas:
        ws = wstats[str(d)]
        a5 += 16 * m + 8 * (ws["union"] + ws["sum_cand_min"])
    return {"a1": 16 * m, "a2": 56 * m + 8 * n, "a3": 16 * m + 8 * (pairs + 1),
            "a4": 40 * m * len(deltas), "a5": a5}


def byte_model(m: int, n: int, info: dict, ws: dict | None, passes: dict, levels: int = 1) -> dict:
    """Bytes each kernel's access pattern moves per launch (reads + writes of
    the data it touches, each byte once): the weights that split a row's
    algorithmic bytes over its kernels.  m edges, 2m incident entries, n
    nodes, tk = time-sort key width, me = edges on node pairs with >= 2
    edges, nm = such pairs.  Radix scatter passes read and write every (key,
    value) pair once; histogram passes read every key once.  The time sort
    of one graph reads the input arrays (src, dst, t: 16 B per edge) in its
    histogram and first pass, and its last pass writes the rank-ordered
    arrays (t, input index, the two node-sort entries: 44 B per edge when
    the time span fits 32 bits and the entries carry 12-byte values, else
    52 B).  The
    pair sort reads each edge once from its entry at the smaller node and
    sorts (larger node, (smaller node, rank)) pairs on the node bits.  The node sort's last pass writes the sequence arrays
    (node, t, other end | dir, rank) and each entry's slot instead of the
    ping-pong buffers; each edge's two positions come from a two-pass
    partition of (slot, position) pairs and a bucket fill."""
    e2 = 2 * m
    tk = 4 if info["tbits"] <= 32 else 8
    nv = 12 if info["tbits"] <= 32 else 16   # node-sort value bytes
    rank_out = 12 + 2 * (4 + nv)
    me, nm = info["multi_pair_edges"], info["multi_pairs"]
    pt = max(passes["time"], 1)
    time_first = 16 + ((tk + 12) if pt > 1 else rank_out)
    # "sort_time_scatter": every pass but the last (the first reads the inputs)
    time_scatter = ((m * time_first + m * (tk + 12) * 2 * max(pt - 2, 0)) / (pt - 1)
                    if pt > 1 else 0)
    table = {
        "validate": m * 16,
        "time_keys": m * (16 + tk + 12),   # batches only
        "sort_time_hist": m * 8,
        "sort_time_scatter": time_scatter,
        "sort_time_scatter_last": m * (tk + 12 + rank_out) if pt > 1 else m * (16 + rank_out),
        "sort_node_hist": e2 * 4,
        "sort_node_scatter": e2 * 2 * (4 + nv),
        # the last pass also writes each entry's slot (2r + dir) in entry order
        "sort_node_scatter_last": e2 * (4 + nv + 24),
        # edge positions: (slot, position) pairs partitioned by the slot's
        # high bits (the first pass reads the slots alone), then each bucket
        # filled through LDS, with each edge's record (t, both positions)
        "sort_slot_hist": 0,   # the slots are 0 .. 2m-1: digit counts from 2m alone
        "sort_slot_scatter": e2 * 14,
        "epos_fill": e2 * (8 + 4) + m * (8 + 16),
        "offsets_fill": (n + 1) * 4,
        "offsets": e2 * 4 + (n + 1) * 4,
        "sort_pair_hist": m * 4,
        "sort_pair_scatter": m * (8 + 4) * 2,
        "pair_flags": m * (12 + 1),
        # per edge its pair-flag prefix; per element of a pair with >= 2
        # edges its pair-sort record, its edge record, X at its two entries
        # and at the two nodes' first entries, and its 33 B of output
        "multi_fill": m * 8 + me * (12 + 16 + 16 + 33) + nm * 12,
        # keys read; per window the sizes (4 B) and, for non-empty windows,
        # the two star/pair records (8 B each, with X read next to the entry;
        # counted here as one); one graph: the three window bit planes too
        "windows": e2 * (12 + 12 * levels) + (n + 1) * 4 + e2 / 8 + e2 / 4,
        # per element its record, once for all windows of the pass; per side
        # and window its position and the two window records of its entry
        "star_pair": me * 25 + levels * 2 * me * 24,
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


def split_name(full: str) -> tuple[str, str]:
    """'a2:sort_node_scatter' -> ('a2', 'sort_node_scatter')."""
    if ":" in full:
        r, k = full.split(":", 1)
        return r, k
    return "other", full


def kernel_table(prof: dict, model: dict, rows_alg: dict, steps: int) -> tuple[dict, dict]:
    """Per traced kernel: launches, time, modelled bytes, and its share of its
    row's algorithmic bytes (the row's bytes split over the row's kernels in
    proportion to their modelled bytes per step) with the fraction of peak
    that share reaches.  Also the per-row summary."""
    kernels, per_row_model = {}, {}
    for full, (launches, total_ms) in prof.items():
        r, k = split_name(full)
        b = model.get(k)
        if b is not None:
            per_row_model[r] = per_row_model.get(r, 0.0) + b * launches / steps
    rows = {}
    for full, (launches, total_ms) in prof.items():
        r, k = split_name(full)
        row = {"launches": launches, "total_ms": round(total_ms, 4),
               "avg_ms": round(total_ms / max(launches, 1), 5)}
        b = model.get(k)
        if b is not None and total_ms > 0:
            row["model_bytes_per_launch"] = int(b)
            row["model_GBs"] = round(b / (total_ms / launches / 1e3) / 1e9, 1)
            if r in rows_alg and per_row_model.get(r):
                alg = rows_alg[r] * (b * launches / steps) / per_row_model[r] / (launches / steps)
                gbs = alg / (total_ms / launches / 1e3) / 1e9
                row.update({"alg_bytes_per_launch": int(alg), "achieved_GBs": round(gbs, 1),
                            "frac": round(gbs / HBM_PEAK_GBS, 4)})
        kernels[full] = row
        rr = rows.setdefault(r, {"ms_per_step": 0.0})
        rr["ms_per_step"] += total_ms / steps
    for r, rr in rows.items():
        rr["ms_per_step"] = round(rr["ms_per_step"], 4)
        rr["step"] = ROWS.get(r, "untagged launches")
        if r in rows_alg and rr["ms_per_step"] > 0:
            gbs = rows_alg[r] / (rr["ms_per_step"] / 1e3) / 1e9
            rr.update({"alg_bytes_per_step": int(rows_alg[r]), "achieved_GBs": round(gbs, 1),
                       "frac": round(gbs / HBM_PEAK_GBS, 4)})
    return kernels, rows


COUNT_KERNELS = ("windows", "star_prep", "item_counts", "item_pairs", "star_pair", "wlevels",
                 "tri_flags", "tri_compact", "triangles", "hub_tiles", "tri_hub", "graph_tiles",
                 "graph_sums", "graph_sums_fin")


def kernel_sources(kernel: str) -> list[str]:
    """The HIP source files that define a traced kernel."""
    k = split_name(kernel)[1]
    if k.startswith("sort_") or k.startswith("scan_"):
        return ["prim.hip", "tm_internal.h"]
    if k in COUNT_KERNELS:
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
    fname = kernel.replace(":", ".")
    path = os.path.join(ROOT, "profiles", f"pmc_{fname}_{workload}.txt")
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


COPY_CALIB_BYTES = 256 << 20


def run_single(args, workload: str, full: bool = True) -> dict:
    """One graph: a step builds the device graph from device pointers and
    counts every delta of the workload (one for power-law and tiny, three for
    skewed) on it.  ``full`` adds the CPU baseline, the PCIe-inclusive rate
    and the per-family and per-delta timings."""
    import numpy as np
    import torch

    import graphgen
    import paper_2204_09236_amd as tm

    dev = torch.device("cuda:0")
    spec = graphgen.CONFIGS[workload]
    deltas = list(spec["deltas"])
    t0 = time.time()
    g = spec["fn"]()
    print(f"[bench] generated {workload}: n={g.n} m={g.m} in {time.time() - t0:.1f}s",
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
    multi = len(deltas) > 1 and not args.separate_counts

    def step():
        G = tm.build_graph(src, dst, tt, n=g.n, stream=stream)
        outs = list(G.count_multi(deltas)) if multi else [G.count(d) for d in deltas]
        G.free()
        return outs

    # the library's autotuner, once, before warm-up and outside the timed
    # region, on the step's own count (all of the workload's windows in one
    # pass): its choice is kept in the process-wide table keyed by graph
    # shape, so the timed steps' freshly built graphs of this shape count
    # with it
    tuned = None
    if not args.no_autotune:
        G0 = tm.build_graph(src, dst, tt, n=g.n, stream=stream)
        tuned = G0.autotune_multi(deltas) if multi else G0.autotune([max(deltas)])
        G0.free()
        print(f"[bench] autotuned at deltas {deltas}: {tuned}", file=sys.stderr, flush=True)

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
    # a short spin kernel just outside each end of the timed region: it marks
    # the region in a profiler's kernel trace of this run
    torch.cuda._sleep(1000)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        counts = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    torch.cuda._sleep(1000)
    torch.cuda.synchronize()
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
    extra = {}
    if len(deltas) > 1:
        # every delta in one call (tm_count_multi) against the single counts
        mc = G.count_multi(deltas)
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        for _ in range(args.steps):
            mc = G.count_multi(deltas)
        torch.cuda.synchronize()
        extra["count_multi"] = {
            "deltas": deltas, "ms": round((time.perf_counter() - t_c) * 1e3 / args.steps, 4),
            "sum_of_single_counts_ms": round(sum(count_ms.values()), 4),
            "equals_single_counts": bool(all(np.array_equal(mc[i], G.count(d))
                                              for i, d in enumerate(deltas)))}
    if full:
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
        extra["count_only_family_ms"] = {"delta": deltas[0], **family_ms}
    ehash = graphgen.edge_hash(g)
    extra["four_node"] = four_node(tm, G, g, workload, deltas, args.steps, ehash)
    G.free()
    if full:
        # PCIe-inclusive: the same step from host arrays (the boundary copies them in)
        host_reps = max(1, min(args.steps, 3))
        torch.cuda.synchronize()
        t_h = time.perf_counter()
        for _ in range(host_reps):
            Gh = tm.build_graph(g.src, g.dst, g.t, n=g.n)
            if multi:
                Gh.count_multi(deltas)
            else:
                for d in deltas:
                    Gh.count(d)
            Gh.free()
        torch.cuda.synchronize()
        host_ms = (time.perf_counter() - t_h) * 1e3 / host_reps
        extra["pcie_inclusive"] = {"ms_per_step": round(host_ms, 3),
                                   "edges_per_s": round(g.m * len(deltas) / (host_ms / 1e3), 1),
                                   "note": "inputs in host memory, copied in by tm_build_graph"}

    tspan = int(g.t.max() - g.t.min()) if g.m else 0
    info["tbits"] = max(tspan.bit_length(), 1)
    passes = {"node": (max(int(g.n - 1).bit_length(), 1) + 7) // 8,
              "time": (max(info["tbits"], 1) + 7) // 8}
    wstats = {str(d): window_stats(src, dst, tt, d) for d in deltas}
    pairs = distinct_pairs(src, dst)
    torch.cuda.empty_cache()
    rows_alg = row_bytes(g.m, g.n, pairs, wstats, deltas)
    # count kernels run once per delta: the model averages their bytes over deltas
    levels = len(deltas) if multi else 1
    model = byte_model(g.m, g.n, info, None, passes, levels)
    tri = {"tri_compact": 0.0, "triangles": 0.0, "tri_hub": 0.0}
    for d in deltas:
        md = byte_model(g.m, g.n, info, wstats[str(d)], passes, levels)
        for k in tri:
            tri[k] += md[k] / len(deltas)
    model.update(tri)
    kernels, rows = kernel_table(prof, model, rows_alg, args.steps)
    alg_step = sum(rows_alg.values())
    whole = {"alg_bytes_per_step": int(alg_step), "ms_per_step": round(ms_per_step, 4),
             "achieved_GBs": round(alg_step / (ms_per_step / 1e3) / 1e9, 1),
             "frac": round(alg_step / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    roofline = None
    if dominant_name is not None and dominant_name in prof_timed:
        # the dominant kernel as measured inside the timed steps, with its
        # per-launch algorithmic bytes from the traced pass
        launches, tot = prof_timed[dominant_name]
        kd = kernels.get(dominant_name, {})
        if "alg_bytes_per_launch" in kd and tot > 0:
            avg_ms = tot / launches
            gbs = kd["alg_bytes_per_launch"] / (avg_ms / 1e3) / 1e9
            tr = stored_traffic(dominant_name, workload)
            roofline = {"kernel": dominant_name, "bound": "hbm", "achieved": round(gbs, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "traffic": None if tr is None else tr["bytes"],
                        "alg_bytes_per_launch": kd["alg_bytes_per_launch"],
                        "avg_launch_ms": round(avg_ms, 5), "launches_per_step": launches / args.steps,
                        "model_bytes_per_launch": kd.get("model_bytes_per_launch")}
            if tr is not None:
                roofline["traffic_over_alg"] = round(tr["bytes"] / kd["alg_bytes_per_launch"], 3)
                roofline["traffic_GBs"] = round(tr["bytes"] / (avg_ms / 1e3) / 1e9, 1)

    cpu = None
    if full and not args.no_cpu_baseline:
        cpu = cpu_baseline(args, workload, g, deltas)
    golden = golden_check(workload, g, deltas, counts, ehash)
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": workload, "n": g.n, "m": g.m, "deltas": deltas,
                   "counts_per_step": "tm_count_multi" if multi else "tm_count per delta",
                   "parallelism": "single-gpu"},
        "roofline": roofline, "cpu_baseline": cpu, "golden": golden,
        "rows": rows, "whole_step": whole,
        "build_only_ms": round(build_ms, 4), "count_only_ms": count_ms,
        "count_only_edges_per_s": {d: round(g.m / (v / 1e3), 1) for d, v in count_ms.items()},
        **extra,
        "autotuned": tuned,
        "gpu_kernel_ms_per_step": round(sum(v[1] for v in prof.values()) / args.steps, 4),
        "graph": {**{k: info[k] for k in ("multi_pairs", "multi_pair_edges", "max_degree")},
                  "distinct_pairs": pairs},
        "window_stats": wstats,
        "kernels": kernels,
        "motif_total": [int(c.sum()) for c in counts],
    }
    del src, dst, tt
    torch.cuda.empty_cache()
    return line


def four_node(tm, G, g, workload, deltas, steps, ehash) -> dict:
    """Four-node three-edge motifs (tm_count4) at each delta of the workload:
    the time of one call (which runs the 36-class count its corrections need),
    the time of its own kernels (traced "f4:" launches) and its dominant one,
    and a comparison with the oracle's stored counts
    (tests/golden/motif4_counts.json) where they exist for this input."""
    import numpy as np
    import torch
    golden = {}
    path = os.path.join(ROOT, "tests", "golden", "motif4_counts.json")
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f).get(workload)
        if rec and rec.get("edge_sha256") == ehash:
            golden = rec["counts"]
    out = {}
    for d in deltas:
        f4 = G.count4(d)
        torch.cuda.synchronize()
        reps = max(1, min(steps, 3))
        t0 = time.perf_counter()
        for _ in range(reps):
            G.count4(d)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        tm.prof_only(None)
        tm.prof_reset()
        tm.prof_enable(True)
        G.count4(d)
        tm.prof_enable(False)
        pr = {k: v for k, v in tm.prof_read().items() if k.startswith("f4:")}
        top = max(pr.items(), key=lambda kv: kv[1][1]) if pr else None
        ent = {"ms": round(ms, 3), "edges_per_s": round(g.m / (ms / 1e3), 1),
               "f4_kernels_ms": round(sum(v[1] for v in pr.values()), 3),
               "dominant_kernel": None if top is None else {"name": top[0], "ms": round(top[1][1], 3)},
               "instances": int(f4.sum())}
        if str(d) in golden:
            ent["golden_match"] = bool(np.array_equal(f4, np.array(golden[str(d)]["f4"], dtype=np.uint64)))
        out[str(d)] = ent
    return out


def golden_check(workload, g, deltas, counts, ehash):
    """Compare with the oracle's stored counts for this workload
    (tests/golden/<workload>_counts.json, written by make_golden.py from the
    oracle alone) when the regenerated input has the stored sha256."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", f"{workload}_counts.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("edge_sha256") != ehash:
        return {"match": None, "note": "input differs from the stored one; not compared"}
    ok = True
    for d, c in zip(deltas, counts):
        want = rec["counts"].get(str(d))
        if want is None or not np.array_equal(np.array(want["grid"], dtype=np.uint64), c):
            ok = False
    return {"match": ok, "deltas": deltas, "source": os.path.relpath(path, ROOT)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cores() -> int:
    """Cores this process may run on, at most 16 (the host share that goes
    with one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


CPU_SAMPLE = {"skewed": 0.005, "powerlaw": 0.1, "tiny": 1.0}


def cpu_baseline(args, workload, g, deltas):
    """The CPU oracle (the paper's Algorithms 1 and 2, OpenMP over centers,
    building S_u and E_(v,w) itself) timed on this host on a bounded sample:
    the edges of the first fraction of the time span (a temporal slice keeps
    every window inside it intact), every delta of the workload, three runs
    on one thread and three on all usable cores, median of each.  The GPU
    counts the same slice, and the two are compared."""
    import numpy as np
    import torch

    import oracle
    import paper_2204_09236_amd as tm
    frac = args.cpu_sample or CPU_SAMPLE.get(workload, 0.05)
    lim = int(g.t.min()) + int((int(g.t.max()) - int(g.t.min())) * frac)
    sel = g.t <= lim
    s, d, t = g.src[sel], g.dst[sel], g.t[sel]
    m = int(s.size)
    cores = usable_cores()
    res = {}
    want = None
    for threads in (1, cores):
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            want = [oracle.alg(s, d, t, dl, n=g.n, threads=threads) for dl in deltas]
            runs.append(time.perf_counter() - t0)
        res[threads] = statistics.median(runs)
    with tm.build_graph(torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(),
                        torch.from_numpy(t).cuda(), n=g.n) as G:
        got = [G.count_raw(dl) for dl in deltas]
    match = all(np.array_equal(a, b) for a, b in zip(want, got))
    sample = (f"edges with t in the first {frac:.1%} of the span (m={m} of {g.m}), "
              f"deltas={deltas}, incl. building S_u and E_(v,w); median of 3 runs")
    return {"value": round(m * len(deltas) / res[cores], 1), "unit": "edges/s", "cores": cores,
            "kind": "oracle", "sample": sample,
            "single_thread": {"value": round(m * len(deltas) / res[1], 1), "unit": "edges/s",
                              "cores": 1, "seconds": round(res[1], 3)},
            "all_cores_seconds": round(res[cores], 3),
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "matches_gpu": bool(match)}


def _gen_batch_member(item):
    import graphgen
    g = graphgen.batch_graph(item)
    return g.src, g.dst, g.t, g.n


def bench_batch(args):
    """Batched vs per-graph counting of many uneven graphs, each with its own
    delta.  Batched step = one build of all graphs (tm_build_batch from
    device pointers) + one count (tm_count_batch, a captured hipGraph) + free;
    the build and the count are also timed alone.  Per-graph = tm_build_graph
    + tm_count + free for every graph in turn.  Both must give identical
    counts, and the graphs of the stored oracle sample
    (tests/golden/batch_counts.json) must match it."""
    import multiprocessing as mp

    import numpy as np
    import torch

    import graphgen
    import paper_2204_09236_amd as tm

    dev = torch.device("cuda:0")
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
        out = B.count_batch_raw(deltas)
        B.free()
        return out

    for _ in range(args.warmup):
        raw_b = batched()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        raw_b = batched()
    torch.cuda.synchronize()
    el_b = (time.perf_counter() - t_start) / args.steps
    print(f"[bench] batched: {el_b * 1e3:.1f} ms per batch", file=sys.stderr, flush=True)
    # build alone, count alone
    t_s = time.perf_counter()
    for _ in range(args.steps):
        tm.build_batch_arrays(src, dst, tt, off, ncount, stream=stream).free()
    torch.cuda.synchronize()
    el_build = (time.perf_counter() - t_s) / args.steps
    B = tm.build_batch_arrays(src, dst, tt, off, ncount, stream=stream)
    B.count_batch_raw(deltas)
    torch.cuda.synchronize()
    t_s = time.perf_counter()
    for _ in range(args.steps):
        B.count_batch_raw(deltas)
    torch.cuda.synchronize()
    el_count = (time.perf_counter() - t_s) / args.steps
    B.free()
    # one more batched step with every launch traced: the per-kernel table
    tm.prof_reset()
    tm.prof_enable(True)
    batched()
    torch.cuda.synchronize()
    tm.prof_enable(False)
    prof = tm.prof_read()
    kernels = {k: {"launches": v[0], "total_ms": round(v[1], 4)}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])[:25]}

    def per_graph():
        outs = []
        for i in range(G):
            a, b = int(off[i]), int(off[i + 1])
            Gi = tm.build_graph(src[a:b], dst[a:b], tt[a:b], n=int(ncount[i]), stream=stream)
            outs.append(Gi.count_raw(int(deltas[i])))
            Gi.free()
        return np.stack(outs)

    res_p = per_graph()  # warm-up pass
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    res_p = per_graph()
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t_start
    same = bool(np.array_equal(raw_b, res_p))
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "batch_counts.json")
    if args.batch_graphs == 4096 and args.batch_mhi == 2e6 and os.path.exists(gpath):
        with open(gpath) as f:
            rec = json.load(f)
        bad = [r["index"] for r in rec["members"]
               if not np.array_equal(raw_b[r["index"]], np.array(r["raw"], dtype=np.uint64))]
        golden = {"match": not bad, "graphs_compared": len(rec["members"]), "mismatched": bad[:10],
                  "source": os.path.relpath(gpath, ROOT)}
    line = {
        "metric": METRIC, "value": round(m_total / el_b, 1), "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el_b * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "batch", "graphs": G, "edges": m_total,
                   "m_range": [1000, args.batch_mhi], "delta_range": [60, 86400],
                   "parallelism": "single-gpu"},
        "build_only_ms": round(el_build * 1e3, 3), "count_only_ms": round(el_count * 1e3, 3),
        "per_graph": {"value": round(m_total / el_p, 1), "unit": "edges/s",
                      "seconds": round(el_p, 3)},
        "batched_over_per_graph": round(el_p / el_b, 2),
        "identical_counts": same, "golden": golden,
        "motif_total": int(res_p.sum()),
        "kernels_one_step": kernels,
    }
    print(json.dumps(line))
    if not same or (golden is not None and not golden["match"]):
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
    golden = golden_check("powerlaw", g, [delta], [total], graphgen.edge_hash(g))
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
    """Serving.  Open loop: Poisson arrivals of (pool graph, delta) requests
    at each rate; keyed graphs stay resident after their first request.
    Latency = done - submit on the server's clock; edges/s = edges of the
    completed requests / (last done - first submit), the offered load when
    the server keeps up.  Closed loop (saturation): one list of requests, all
    submitted at once to the server, against the same list run as a plain
    sequential loop of tm_count calls on resident graphs and as a plain loop
    of tm_build_graph + tm_count per request; capacity = edges / wall time.
    Every result is compared with the same request counted alone."""
    import math
    import multiprocessing as mp

    import numpy as np
    import torch

    import graphgen
    import paper_2204_09236_amd as tm

    rng = np.random.default_rng(4)
    spec = graphgen.serve_spec(seed=4, pool=args.serve_pool, m_hi=args.serve_mhi)
    ms = np.array([it.m for it in spec])
    t0 = time.time()
    with mp.get_context("fork").Pool(args.procs) as pool_:
        pool = pool_.map(_gen_batch_member, spec, chunksize=2)
    print(f"[bench] serving pool: {len(pool)} graphs, {int(ms.sum())} edges, generated in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    rates = [float(r) for r in args.serve_rates.split(",")]
    budget = int(0.7 * torch.cuda.get_device_properties(0).total_memory)
    max_inflight = 16
    S = tm.Server(budget, max_inflight=max_inflight)
    alone_graphs = {}
    alone_counts = {}

    def alone(gi, delta):
        if (gi, delta) not in alone_counts:
            if gi not in alone_graphs:
                src, dst, t, n = pool[gi]
                alone_graphs[gi] = tm.build_graph(src, dst, t, n=n)
            alone_counts[(gi, delta)] = alone_graphs[gi].count(delta)
        return alone_counts[(gi, delta)]

    def draw(k):
        return [(int(rng.integers(0, len(pool))),
                 int(round(math.exp(rng.uniform(math.log(60), math.log(86400))))))
                for _ in range(k)]

    rows = []
    sent = set()
    for rate in rates:
        n_req = int(min(args.serve_max, max(20, rate * args.serve_seconds)))
        gaps = rng.exponential(1.0 / rate, n_req)
        reqs = draw(n_req)
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
        same = ok and all(np.array_equal(done[i][1], alone(gi, d)) for i, (gi, d) in enumerate(reqs))
        row = {"rate": rate, "requests": n_req, "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "edges_per_s": round(edges / ((last_done - first_submit) / 1e9), 1),
               "all_ok": ok, "identical_to_alone": same}
        rows.append(row)
        print(f"[bench] serve rate {rate}: {row}", file=sys.stderr, flush=True)

    # closed loop: every pool graph is resident by now (or rebuilt on demand)
    sat_reqs = draw(args.serve_max)
    sat_edges = sum(pool[gi][0].size for gi, _ in sat_reqs)
    for gi, d in sat_reqs:          # the alone results first (not timed)
        alone(gi, d)
    torch.cuda.synchronize()
    t_s = time.perf_counter()
    tks = [S.submit(d, key=gi + 1) if gi in sent else
           S.submit(d, *pool[gi][:3], n=pool[gi][3], key=gi + 1) for gi, d in sat_reqs]
    for gi, _ in sat_reqs:
        sent.add(gi)
    res = [S.wait(tk) for tk in tks]
    el_srv = time.perf_counter() - t_s
    srv_same = all(r[0] == 0 and np.array_equal(r[1], alone(gi, d))
                   for r, (gi, d) in zip(res, sat_reqs))
    torch.cuda.synchronize()
    t_s = time.perf_counter()
    plain = [alone_graphs[gi].count(d) for gi, d in sat_reqs]
    torch.cuda.synchronize()
    el_plain = time.perf_counter() - t_s
    plain_same = all(np.array_equal(a, alone(gi, d)) for a, (gi, d) in zip(plain, sat_reqs))
    n_build = min(len(sat_reqs), 200)
    t_s = time.perf_counter()
    for gi, d in sat_reqs[:n_build]:
        src, dst, t, n = pool[gi]
        with tm.build_graph(src, dst, t, n=n) as Gb:
            Gb.count(d)
    torch.cuda.synchronize()
    el_build = time.perf_counter() - t_s
    build_edges = sum(pool[gi][0].size for gi, _ in sat_reqs[:n_build])
    saturation = {
        "requests": len(sat_reqs), "edges": int(sat_edges),
        "served": {"seconds": round(el_srv, 4), "edges_per_s": round(sat_edges / el_srv, 1),
                   "identical_to_alone": bool(srv_same)},
        "plain_resident": {"seconds": round(el_plain, 4),
                           "edges_per_s": round(sat_edges / el_plain, 1),
                           "identical_to_alone": bool(plain_same),
                           "note": "sequential tm_count calls on graphs built beforehand"},
        "plain_build_and_count": {"requests": n_build, "seconds": round(el_build, 4),
                                  "edges_per_s": round(build_edges / el_build, 1),
                                  "note": "sequential tm_build_graph (host arrays) + tm_count "
                                          "per request"},
        "served_over_plain_resident": round(el_plain / el_srv, 3),
        "served_over_plain_build": round((sat_edges / el_srv) / (build_edges / el_build), 3),
    }
    print(f"[bench] saturation: {saturation}", file=sys.stderr, flush=True)
    st = S.stats()
    S.close()
    for G in alone_graphs.values():
        G.free()
    line = {
        "metric": METRIC,
        "value": saturation["served"]["edges_per_s"], "unit": "edges/s", "n_gpus": 1,
        "steps": len(rows), "warmup": 0, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "serve", "pool_graphs": len(pool), "pool_edges": int(ms.sum()),
                   "m_range": [1000, args.serve_mhi], "delta_range": [60, 86400],
                   "budget_bytes": budget, "max_inflight": max_inflight,
                   "parallelism": "single-gpu"},
        "value_is": "closed-loop served edges/s (capacity)",
        "rates": rows, "requests_total": sum(r["requests"] for r in rows) + len(sat_reqs),
        "saturation": saturation, "server_stats": st,
    }
    print(json.dumps(line))
    if not all(r["identical_to_alone"] for r in rows) or not srv_same or not plain_same:
        sys.exit(1)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are "
                          "not supported (the path would shard by center)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "stream":
        return bench_stream(args)
    line = run_single(args, args.workload, full=True)
    extras = {}
    for w in [x for x in args.extra_workloads.split(",") if x and x != args.workload]:
        ex = run_single(args, w, full=False)
        extras[w] = {k: ex[k] for k in ("value", "unit", "ms_per_step", "config", "roofline", "rows",
                                        "whole_step", "build_only_ms", "count_only_ms", "golden",
                                        "four_node", "motif_total")}
    if extras:
        line["extra_workloads"] = extras
    print(json.dumps(line))
    f4_bad = any(v.get("golden_match") is False
                 for ln in [line, *extras.values()] for v in ln.get("four_node", {}).values())
    bad = (line["cpu_baseline"] is not None and not line["cpu_baseline"]["matches_gpu"]) or \
        (line["golden"] is not None and line["golden"]["match"] is False) or \
        any(e["golden"] is not None and e["golden"]["match"] is False for e in extras.values()) or f4_bad
    if bad:
        sys.exit(1)


if __name__ == "__main__":
    main()
