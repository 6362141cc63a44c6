"""Seeded synthetic temporal edge lists for the motif counter and its tests.

This module only draws random inputs: it holds none of the counting method's
arithmetic, so both the CPU oracle and the HIP path may use it.

An edge list is three numpy arrays ``(src int32[m], dst int32[m], t int64[m])``;
the edge id of row i is i (ties in t are ordered by id).  Node ids are
``0 .. n-1`` and no edge is a self-loop (Definition 1 of the paper: a temporal
edge is a timestamped directed edge between two nodes).

Workloads (shapes follow the paper's public datasets, Table 2, which are not
available here, so these synthetic stand-ins take their place):

* ``tiny``     200 nodes, 5,000 edges, uniform endpoints, t uniform in [0, 1e5],
               delta = 1,000, seed 0.
* ``powerlaw`` 1M nodes, 20M edges, directed Chung-Lu with degree exponent 2.1,
               per-source bursty Pareto(alpha = 1.5) inter-event times over a
               6e7 s span, delta = 3,600, seed 1.
* ``skewed``   10M nodes, 300M edges: 240M Chung-Lu edges with weights
               (i + i0)^-1 (exponent 2.0, i0 solved for an expected top
               out-degree of 1e6) plus 60M repeats of random base edges with
               Poisson-spaced (exponential, mean 3,600 s) later timestamps, span
               1e8 s, delta in {600, 3600, 86400}, seed 2.
* ``batch``    G graphs with m log-uniform in [1e3, 2e6], n = max(3, m // 20),
               Chung-Lu 2.1 + Pareto times over 6e7 s, per-graph delta
               log-uniform in [60, 86400], seed 3.  Each graph has its own
               spawned seed so any one of them can be rebuilt alone.
* ``serve``    a pool of graphs with m log-uniform in [1e3, 5e7], n = m // 20,
               generated like the batch members, seed 4; requests draw a pool
               graph and a delta log-uniform in [60, 86400].  ``serve_max`` is
               a request graph at the top of that range (5e7 edges, 2.5M
               nodes, seed 40).
"""
from __future__ import annotations

import hashlib
import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

__all__ = [
    "EdgeList", "tiny", "powerlaw", "skewed", "batch_spec", "batch_graph",
    "small_random", "chung_lu_pareto", "edge_hash", "CONFIGS", "batch_sample",
    "serve_spec", "serve_max",
]


@dataclass
class EdgeList:
    src: np.ndarray   # int32[m]
    dst: np.ndarray   # int32[m]
    t: np.ndarray     # int64[m]
    n: int            # node count (ids are < n)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def edge_hash(g: EdgeList) -> str:
    """sha256 over the raw arrays: identifies a generated input exactly."""
    h = hashlib.sha256()
    for a in (g.src, g.dst, g.t):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(str(g.n).encode())
    return h.hexdigest()


# --------------------------------------------------------------------------
# building blocks

def _inverse_cdf_sample(rng: np.random.Generator, weights: np.ndarray, size: int) -> np.ndarray:
    """Draw ``size`` indices with probability proportional to ``weights``.

    The uniforms are drawn from ``rng`` in order, chunk by chunk; the
    lookups of a group of chunks run on threads (numpy releases the GIL in
    searchsorted), which changes nothing in the result."""
    cdf = np.cumsum(weights, dtype=np.float64)
    cdf /= cdf[-1]
    out = np.empty(size, dtype=np.int32)
    step = 1 << 24                     # bounded temporaries for the 300M-edge case
    last = weights.shape[0] - 1
    workers = max(1, min(16, os.cpu_count() or 1))

    def lookup(job):
        b, u = job
        idx = np.searchsorted(cdf, u, side="right")
        np.minimum(idx, last, out=idx)
        out[b:b + idx.shape[0]] = idx

    starts = list(range(0, size, step))
    with ThreadPoolExecutor(workers) as ex:
        for g in range(0, len(starts), workers):
            jobs = [(b, rng.random(min(step, size - b))) for b in starts[g:g + workers]]
            list(ex.map(lookup, jobs))
    return out


def _chung_lu(rng: np.random.Generator, n: int, m: int, w_out: np.ndarray,
              w_in: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Directed Chung-Lu multigraph: src ~ w_out, dst ~ w_in, self-loops redrawn."""
    src = _inverse_cdf_sample(rng, w_out, m)
    dst = _inverse_cdf_sample(rng, w_in, m)
    while True:
        bad = np.flatnonzero(src == dst)
        if bad.size == 0:
            break
        dst[bad] = _inverse_cdf_sample(rng, w_in, bad.size)
    return src, dst


def _bursty_times(rng: np.random.Generator, src: np.ndarray, n: int, span: int,
                  alpha: float) -> np.ndarray:
    """Per-source renewal process with Pareto(alpha) gaps.

    Node u with k_u out-edges gets gaps x_u * (1 + Lomax(alpha)) (a classic
    Pareto with scale x_u), x_u chosen so that k_u mean gaps cover the span, a
    uniform random phase, and times wrapped into [0, span).
    """
    m = src.shape[0]
    order = np.argsort(src, kind="stable")
    s_sorted = src[order]
    counts = np.bincount(src, minlength=n).astype(np.int64)
    starts = np.concatenate(([0], np.cumsum(counts)[:-1]))
    k = counts[s_sorted].astype(np.float64)
    mean_gap = span / k
    xm = mean_gap * (alpha - 1.0) / alpha
    gaps = xm * (rng.pareto(alpha, m) + 1.0)
    del k, xm, mean_gap
    # cumulative time inside each source's run of edges
    cs = np.cumsum(gaps)
    first = starts[s_sorted]
    base = np.where(first > 0, cs[np.maximum(first - 1, 0)], 0.0)
    local = cs - base
    del cs, base, gaps, first
    phase = rng.random(n) * span
    tt = np.floor(phase[s_sorted] + local).astype(np.int64) % span
    t = np.empty(m, dtype=np.int64)
    t[order] = tt
    return t


def chung_lu_pareto(seed, n: int, m: int, gamma: float = 2.1, span: int = 60_000_000,
                    alpha: float = 1.5) -> EdgeList:
    """Directed Chung-Lu (out and in weights (i+1)^(-1/(gamma-1)), the in
    weights under an independent random permutation of the nodes) with bursty
    per-source Pareto timestamps."""
    rng = np.random.default_rng(seed)
    n = int(n)
    base = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    w_out = base
    w_in = base[rng.permutation(n)]
    src, dst = _chung_lu(rng, n, m, w_out, w_in)
    t = _bursty_times(rng, src, n, span, alpha)
    return EdgeList(src, dst, t, n)


# --------------------------------------------------------------------------
# named workloads

def tiny(seed: int = 0, n: int = 200, m: int = 5000, tmax: int = 100_000) -> EdgeList:
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n - 1, m).astype(np.int32)
    dst = (dst + (dst >= src)).astype(np.int32)       # uniform over nodes != src
    t = rng.integers(0, tmax + 1, m).astype(np.int64)
    return EdgeList(src, dst, t, n)


def powerlaw(seed: int = 1, n: int = 1_000_000, m: int = 20_000_000) -> EdgeList:
    return chung_lu_pareto(seed, n, m, gamma=2.1, span=60_000_000, alpha=1.5)


def _solve_offset(n: int, m_base: int, top: float) -> float:
    """i0 such that m_base * (1/i0) / sum_i 1/(i+i0) equals ``top``."""
    lo, hi = 1.0, 1e4
    i = np.arange(n, dtype=np.float64)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        val = m_base / mid / np.sum(1.0 / (i + mid))
        if val > top:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def skewed(seed: int = 2, n: int = 10_000_000, m: int = 300_000_000,
           repeat_frac: float = 0.2, span: int = 100_000_000,
           repeat_mean: float = 3600.0, top_degree: float = 1e6) -> EdgeList:
    rng = np.random.default_rng(seed)
    m_rep = int(round(m * repeat_frac))
    m_base = m - m_rep
    i0 = _solve_offset(n, m_base, top_degree)
    base = 1.0 / (np.arange(n, dtype=np.float64) + i0)
    w_out = base
    w_in = base[rng.permutation(n)]
    src, dst = _chung_lu(rng, n, m_base, w_out, w_in)
    t = _bursty_times(rng, src, n, span, 1.5)
    pick = rng.integers(0, m_base, m_rep)
    gap = np.rint(rng.exponential(repeat_mean, m_rep)).astype(np.int64)
    t_rep = np.minimum(t[pick] + gap, span - 1)
    src = np.concatenate((src, src[pick]))
    dst = np.concatenate((dst, dst[pick]))
    t = np.concatenate((t, t_rep))
    del pick, gap, t_rep
    perm = rng.permutation(m)
    return EdgeList(src[perm].astype(np.int32), dst[perm].astype(np.int32),
                    t[perm].astype(np.int64), n)


@dataclass
class BatchItem:
    m: int
    n: int
    delta: int
    seed: np.random.SeedSequence


def batch_spec(seed: int = 3, graphs: int = 4096, m_lo: float = 1e3,
               m_hi: float = 2e6, d_lo: float = 60.0, d_hi: float = 86400.0) -> list[BatchItem]:
    rng = np.random.default_rng(seed)
    ms = np.rint(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), graphs))).astype(np.int64)
    ds = np.rint(np.exp(rng.uniform(math.log(d_lo), math.log(d_hi), graphs))).astype(np.int64)
    kids = np.random.SeedSequence(seed).spawn(graphs)
    return [BatchItem(int(mg), max(3, int(mg) // 20), int(dg), kids[i])
            for i, (mg, dg) in enumerate(zip(ms, ds))]


def batch_graph(item: BatchItem) -> EdgeList:
    return chung_lu_pareto(item.seed, item.n, item.m, gamma=2.1, span=60_000_000, alpha=1.5)


def batch_sample(spec: list[BatchItem], k: int = 256, seed: int = 30) -> list[int]:
    """Indices of a seeded sample of a batch that spans its whole range: the
    20 largest graphs, the 10 with the widest windows, the 10 smallest, and
    the rest drawn uniformly from the others (sorted, no repeats)."""
    ms = np.array([it.m for it in spec])
    ds = np.array([it.delta for it in spec])
    pick: list[int] = []
    for idx in (np.argsort(-ms, kind="stable")[:20], np.argsort(-ds, kind="stable")[:10],
                np.argsort(ms, kind="stable")[:10]):
        pick += [int(i) for i in idx if int(i) not in pick]
    rest = np.array([i for i in range(len(spec)) if i not in set(pick)])
    rng = np.random.default_rng(seed)
    extra = rng.choice(rest, size=max(0, min(k - len(pick), rest.size)), replace=False)
    return sorted(pick + [int(i) for i in extra])


def serve_spec(seed: int = 4, pool: int = 128, m_lo: float = 1e3,
               m_hi: float = 5e7) -> list[BatchItem]:
    """The serving pool: graphs with m log-uniform in [m_lo, m_hi], n = m // 20
    (delta is drawn per request, not per graph)."""
    rng = np.random.default_rng(seed)
    ms = np.rint(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), pool)))
    kids = np.random.SeedSequence(seed).spawn(pool)
    return [BatchItem(int(m), max(3, int(m) // 20), 0, kids[i]) for i, m in enumerate(ms)]


def serve_max(seed: int = 40, m: int = 50_000_000) -> EdgeList:
    """A serving request graph at the top of the request-size range."""
    return chung_lu_pareto(seed, m // 20, m, gamma=2.1, span=60_000_000, alpha=1.5)


def small_random(rng: np.random.Generator, n: int, m: int, t_values: int | None = None,
                 tmax: int = 1000, multi: float = 0.0) -> EdgeList:
    """Tiny adversarial graph for exhaustive checks.

    ``t_values`` forces timestamps onto that many distinct values (many ties);
    ``multi`` is the fraction of rows that repeat an earlier row's endpoints
    (multi-edges, possibly with equal timestamps)."""
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n - 1, m).astype(np.int32)
    dst = (dst + (dst >= src)).astype(np.int32)
    if multi > 0 and m > 1:
        rep = np.flatnonzero(rng.random(m) < multi)
        rep = rep[rep > 0]
        srcs = rng.integers(0, rep, rep.size) if rep.size else rep
        src[rep] = src[srcs]
        dst[rep] = dst[srcs]
    if t_values:
        vals = np.sort(rng.integers(0, tmax + 1, t_values))
        t = vals[rng.integers(0, t_values, m)].astype(np.int64)
    else:
        t = rng.integers(0, tmax + 1, m).astype(np.int64)
    return EdgeList(src, dst, t, n)


CONFIGS = {
    "tiny": dict(fn=tiny, deltas=[1000]),
    "powerlaw": dict(fn=powerlaw, deltas=[3600]),
    "skewed": dict(fn=skewed, deltas=[600, 3600, 86400]),
}
