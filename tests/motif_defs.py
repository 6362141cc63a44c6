"""Shared test helpers: counter indices, the toy graph, graph transforms.

The counter index layout is the paper's: Star[Type,d1,d2,d3] (Section IV-A,
quadruple counter), Pair[d1,d2,d3] (triple counter), Tri[Type,d_i,d_j,d_k]
(Section IV-B), with o = 0 and in = 1, concatenated into 56 raw cells.

The 36-cell motif layout M_ij used by the library and the oracle: the paper's
Figure 2 is missing from the available text, and its text pins only these
cells: M24 = Star[I,in,o,in] (Section IV-A), M63 = Star[III,o,o,in], M46 and
M65 through the instances named in Section III, M25 through the three-view
example of Section IV-B, M26 = the time-respecting 3-cycle (the only motif the
2SCENT baseline finds, Section V-D), M55 / M56 / M65 through the isomorphic pair
cells of Section IV-A (M66 is the remaining pair class), and M13, M53 are star
motifs (Section V-C).  The remaining cells follow one convention that honours
all of them (``GRID`` below is the specification both implementations are
checked against).
"""
from __future__ import annotations

import os

import numpy as np

O, IN = 0, 1
TYPES = {"I": 0, "II": 1, "III": 2}
D = {"o": O, "in": IN}


def i_star(ty, a, b, c):
    return TYPES.get(ty, ty) * 8 + D.get(a, a) * 4 + D.get(b, b) * 2 + D.get(c, c)


def i_pair(a, b, c):
    return 24 + D.get(a, a) * 4 + D.get(b, b) * 2 + D.get(c, c)


def i_tri(ty, a, b, c):
    return 32 + TYPES.get(ty, ty) * 8 + D.get(a, a) * 4 + D.get(b, b) * 2 + D.get(c, c)


def cell(row, col):
    """Flat index of M_{row,col} (1-based) in the 36-vector / 6x6 grid."""
    return 6 * (row - 1) + (col - 1)


# ---- the 36-cell layout, written out as the specification -------------------
# key: ("star", type, d1, d2, d3) | ("pair", d2, d3) | ("tri", a, b, c)
def _spec_grid():
    g = {}
    for ty in range(3):
        for d1 in range(2):
            for d2 in range(2):
                for d3 in range(2):
                    row = 1 + 2 * ty + (d3 == IN)
                    col = 1 + 2 * (d2 == O) + (d1 == IN)
                    g[("star", ty, d1, d2, d3)] = cell(row, col)
    g[("pair", O, O)] = cell(5, 5)
    g[("pair", IN, IN)] = cell(5, 6)
    g[("pair", IN, O)] = cell(6, 5)
    g[("pair", O, IN)] = cell(6, 6)
    rowmap = {(True, True): 1, (False, False): 2, (False, True): 3, (True, False): 4}
    for a in range(2):
        for b in range(2):
            for c in range(2):
                g[("tri", a, b, c)] = cell(rowmap[(a == b, c == b)], 5 + (b == O))
    return g


GRID = _spec_grid()


def canon_from_raw(raw) -> np.ndarray:
    """Class counts in canonical order [Star 24 | pair class 4 | tri class 8]
    from the paper's raw counters: stars one-to-one, the pair class is the
    view from the first edge's source (Pair[o,.,.]), the triangle class is the
    Type-I view Tri[I,a,b,c]."""
    raw = np.asarray(raw, dtype=np.uint64)
    out = np.zeros(36, dtype=np.uint64)
    out[:24] = raw[:24]
    out[24:28] = raw[24:28]            # Pair[o][d2][d3]
    out[28:36] = raw[32:40]            # Tri[I][a][b][c]
    return out


def grid_from_canon(canon) -> np.ndarray:
    canon = np.asarray(canon, dtype=np.uint64)
    out = np.zeros(36, dtype=np.uint64)
    for ty in range(3):
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    out[GRID[("star", ty, a, b, c)]] += canon[ty * 8 + a * 4 + b * 2 + c]
    for b in range(2):
        for c in range(2):
            out[GRID[("pair", b, c)]] += canon[24 + b * 2 + c]
    for a in range(2):
        for b in range(2):
            for c in range(2):
                out[GRID[("tri", a, b, c)]] += canon[28 + a * 4 + b * 2 + c]
    return out.reshape(6, 6)


# ---- the paper's toy graph (Figure 1, recovered from the text) --------------
TOY_NODES = "abcde"


def load_toy():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "toy_graph.txt")
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            a, b, t = line.split()
            rows.append((TOY_NODES.index(a), TOY_NODES.index(b), int(t)))
    src = np.array([r[0] for r in rows], np.int32)
    dst = np.array([r[1] for r in rows], np.int32)
    t = np.array([r[2] for r in rows], np.int64)
    return src, dst, t


def edges(rows, names=TOY_NODES):
    """Tiny graph from rows like ('a', 'c', 4)."""
    src = np.array([names.index(r[0]) if isinstance(r[0], str) else r[0] for r in rows], np.int32)
    dst = np.array([names.index(r[1]) if isinstance(r[1], str) else r[1] for r in rows], np.int32)
    t = np.array([r[2] for r in rows], np.int64)
    return src, dst, t


# ---- transforms used by invariance tests ------------------------------------
def relabel(src, dst, t, n, rng):
    perm = rng.permutation(n).astype(np.int32)
    return perm[src], perm[dst], t


def reverse_edges(src, dst, t):
    return dst.copy(), src.copy(), t.copy()


def reverse_time(src, dst, t):
    """t -> -t and id -> m-1-id, so the (t, id) order is exactly reversed."""
    return src[::-1].copy(), dst[::-1].copy(), (-t[::-1]).copy()


def canon_edge_reversal(c):
    """Class counts of the edge-reversed graph: Star[T,d] -> Star[T,not d],
    pair classes fixed, Tri(a,b,c) -> (not a, not b, not c)."""
    c = np.asarray(c)
    out = np.zeros_like(c)
    for ty in range(3):
        for a in range(2):
            for b in range(2):
                for d in range(2):
                    out[ty * 8 + (1 - a) * 4 + (1 - b) * 2 + (1 - d)] = c[ty * 8 + a * 4 + b * 2 + d]
    out[24:28] = c[24:28]
    for a in range(2):
        for b in range(2):
            for d in range(2):
                out[28 + (1 - a) * 4 + (1 - b) * 2 + (1 - d)] = c[28 + a * 4 + b * 2 + d]
    return out


def canon_time_reversal(c):
    """Class counts of the time-reversed graph: Star[I,d1,d2,d3] <->
    Star[III,d3,d2,d1], Star[II,d1,d2,d3] -> Star[II,d3,d2,d1], pair class
    (d2,d3) -> (d2,o) if d3 = o else (not d2, in), Tri(a,b,c) -> (not a, c, b)."""
    c = np.asarray(c)
    out = np.zeros_like(c)
    tmap = {0: 2, 1: 1, 2: 0}
    for ty in range(3):
        for a in range(2):
            for b in range(2):
                for d in range(2):
                    out[tmap[ty] * 8 + d * 4 + b * 2 + a] = c[ty * 8 + a * 4 + b * 2 + d]
    for b in range(2):
        for d in range(2):
            nb, nd = (b, O) if d == O else (1 - b, IN)
            out[24 + nb * 2 + nd] += c[24 + b * 2 + d]
    for a in range(2):
        for b in range(2):
            for d in range(2):
                out[28 + (1 - a) * 4 + d * 2 + b] = c[28 + a * 4 + b * 2 + d]
    return out


def disjoint_union(g1, g2, n1):
    s1, d1, t1 = g1
    s2, d2, t2 = g2
    return (np.concatenate([s1, s2 + n1]).astype(np.int32),
            np.concatenate([d1, d2 + n1]).astype(np.int32),
            np.concatenate([t1, t2]).astype(np.int64))
