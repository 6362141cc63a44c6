"""Pins for the four-node motif oracle (oracle/tm_motif4.c).

The paper leaves higher-order motifs to future work (Section VI); the
definition is the paper's Definitions 2-3 and Problem 1 with four nodes.  The
oracle's two enumerations are checked against:
  * hand-worked cases (tests/golden/motif4_cases.json, reasoning in the file);
  * closed forms on stars built edge by edge;
  * each other on random graphs with ties and multi-edges;
  * identities with the three-node oracle: every chronological triple of one
    node's edges inside delta is a four-node star, a three-node star at that
    center or a two-node pair (seen from each of its nodes), and every
    (middle edge, edge at its source, edge at its target) choice is a path, a
    triangle (three choices each), a three-node star (two) or a pair (six);
  * invariants: edge reversal, time reversal, relabelling.
"""
import json
import os
from math import comb

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def arrays(edges):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    return e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.int64)


def random_graph(seed, n, m, tmax, multi=0.3):
    """Small random temporal graph with forced ties and repeated node pairs."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n - 1, m).astype(np.int32)
    dst[dst >= src] += 1
    rep = rng.random(m) < multi
    j = rng.integers(0, m, m)
    flip = rng.random(m) < 0.5
    src[rep] = np.where(flip[rep], dst[j[rep]], src[j[rep]])
    dst[rep] = np.where(flip[rep], src[j[rep]], dst[j[rep]])
    bad = src == dst
    dst[bad] = (src[bad] + 1) % n
    t = rng.integers(0, tmax, m).astype(np.int64)
    return src, dst, t


def both(src, dst, t, delta, n=None):
    b = oracle.brute4(src, dst, t, delta, n=n)
    lo = oracle.local4(src, dst, t, delta, n=n, threads=2)
    np.testing.assert_array_equal(b, lo)
    return b


# ------------------------------------------------------------ worked cases

CASES = json.load(open(os.path.join(HERE, "golden", "motif4_cases.json")))["cases"]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_hand_worked_cases(case):
    src, dst, t = arrays(case["edges"])
    want = np.zeros(32, dtype=np.uint64)
    for k, v in case["expect"].items():
        want[int(k)] = v
    np.testing.assert_array_equal(both(src, dst, t, case["delta"]), want)


def test_empty_and_tiny():
    for edges in ([], [[0, 1, 0]], [[0, 1, 0], [1, 2, 1]]):
        src, dst, t = arrays(edges)
        np.testing.assert_array_equal(both(src, dst, t, 5, n=3), np.zeros(32, np.uint64))


def test_rejects_invalid():
    with pytest.raises(oracle.OracleError):
        oracle.local4(*arrays([[0, 0, 1]]), 5, n=2)
    with pytest.raises(oracle.OracleError):
        oracle.brute4(*arrays([[0, 1, 1]]), -1, n=2)


# ------------------------------------------------------------ closed forms

def test_star_out_then_in():
    """Center 0 sends to k leaves, then receives from k more, all inside
    delta: (o,o,o) and (in,in,in) C(k,3), (o,o,in) and (o,in,in) C(k,2) k, the
    rest 0; no paths."""
    k = 7
    edges = [[0, 1 + i, 1 + i] for i in range(k)] + [[1 + k + i, 0, 1 + k + i] for i in range(k)]
    src, dst, t = arrays(edges)
    got = both(src, dst, t, 100)
    want = np.zeros(32, np.uint64)
    want[0b000] = comb(k, 3)
    want[0b001] = comb(k, 2) * k
    want[0b011] = k * comb(k, 2)
    want[0b111] = comb(k, 3)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("delta", [0, 1, 2, 5, 30])
def test_star_window_closed_form(delta):
    """k out-edges of one center at times 0..k-1: the triples inside delta
    number sum_i C(min(delta, k-1-i), 2)."""
    k = 25
    src, dst, t = arrays([[0, 1 + i, i] for i in range(k)])
    got = both(src, dst, t, delta)
    want = np.zeros(32, np.uint64)
    want[0] = sum(comb(min(delta, k - 1 - i), 2) for i in range(k))
    np.testing.assert_array_equal(got, want)


def test_path_chain_closed_form():
    """The chain 0->1->2->...->L at times 1..L with delta = 2: the paths are
    the L-2 runs of three consecutive edges, each read from its first edge,
    middle second, all forward (class 8 + 8 + 7); no stars."""
    L = 12
    src, dst, t = arrays([[i, i + 1, i + 1] for i in range(L)])
    got = both(src, dst, t, 2)
    want = np.zeros(32, np.uint64)
    want[23] = L - 2
    np.testing.assert_array_equal(got, want)


# ------------------------------------------------------- the two enumerations

@pytest.mark.parametrize("seed", range(8))
def test_brute_equals_local(seed):
    n = [5, 6, 8, 12, 20, 6, 9, 15][seed]
    src, dst, t = random_graph(100 + seed, n, 60 + 10 * seed, 40)
    for delta in (0, 3, 10, 40):
        both(src, dst, t, delta, n=n)


# ---------------------------------------------- identities with the 36 classes

def per_center_pairs(src, dst, t, delta, n):
    """sum over nodes c and edges e of c of C(w, 2), w = the later edges of c
    (chronological order) with t <= t(e) + delta."""
    order = np.lexsort((np.arange(src.size), t))
    total = 0
    for c in range(n):
        sel = order[(src[order] == c) | (dst[order] == c)]
        tc = t[sel]
        for i in range(tc.size):
            w = int(np.searchsorted(tc, tc[i] + delta, side="right")) - i - 1
            total += comb(w, 2)
    return total


def middle_edge_choices(src, dst, t, delta):
    """Number of (e, x, y): x != e an edge at src(e), y != e an edge at
    dst(e), x != y, the three inside delta."""
    m = src.size
    total = 0
    for e in range(m):
        s, d = src[e], dst[e]
        xs = [x for x in range(m) if x != e and s in (src[x], dst[x])]
        ys = [y for y in range(m) if y != e and d in (src[y], dst[y])]
        for x in xs:
            for y in ys:
                if x == y:
                    continue
                ts = (t[e], t[x], t[y])
                if max(ts) - min(ts) <= delta:
                    total += 1
    return total


@pytest.mark.parametrize("seed", range(5))
def test_identities_with_three_node_classes(seed):
    n = [6, 8, 10, 7, 12][seed]
    src, dst, t = random_graph(300 + seed, n, 45, 30)
    for delta in (0, 4, 15):
        f4 = both(src, dst, t, delta, n=n)
        _, canon = oracle.brute(src, dst, t, delta, n=n)
        stars3, pairs, tris = int(canon[:24].sum()), int(canon[24:28].sum()), int(canon[28:].sum())
        assert int(f4[:8].sum()) + stars3 + 2 * pairs == per_center_pairs(src, dst, t, delta, n)
        assert (int(f4[8:].sum()) + 3 * tris + 2 * stars3 + 6 * pairs
                == middle_edge_choices(src, dst, t, delta))


# ------------------------------------------------------------- invariants

def path_index(r, f1, f2, f3):
    return 8 + r * 8 + f1 * 4 + f2 * 2 + f3


@pytest.mark.parametrize("seed", range(4))
def test_edge_reversal(seed):
    """Reversing every edge flips every direction bit: star d -> 1-d, path
    f -> 1-f (the reading end is the same edge)."""
    src, dst, t = random_graph(500 + seed, 9, 70, 30)
    a = both(src, dst, t, 8, n=9)
    b = both(dst, src, t, 8, n=9)
    for i in range(8):
        assert b[7 - i] == a[i]
    for r in range(3):
        for f in range(8):
            assert b[path_index(r, 0, 0, 0) + (7 - f)] == a[path_index(r, 0, 0, 0) + f]


@pytest.mark.parametrize("seed", range(4))
def test_time_reversal(seed):
    """t -> -t with the input order reversed (so ties reverse too) reverses
    the chronological order: star (d1,d2,d3) -> (d3,d2,d1); a path's middle
    position r -> 2-r, its other end becomes the reading end (every bit
    flips) and E1, E3 swap."""
    src, dst, t = random_graph(700 + seed, 9, 70, 30)
    a = both(src, dst, t, 8, n=9)
    b = both(src[::-1].copy(), dst[::-1].copy(), (-t[::-1]).copy(), 8, n=9)
    for d1 in range(2):
        for d2 in range(2):
            for d3 in range(2):
                assert b[d3 * 4 + d2 * 2 + d1] == a[d1 * 4 + d2 * 2 + d3]
    for r in range(3):
        for f1 in range(2):
            for f2 in range(2):
                for f3 in range(2):
                    assert (b[path_index(2 - r, 1 - f3, 1 - f2, 1 - f1)]
                            == a[path_index(r, f1, f2, f3)])


def test_relabelling():
    src, dst, t = random_graph(900, 11, 80, 25)
    perm = np.random.default_rng(1).permutation(11).astype(np.int32)
    np.testing.assert_array_equal(both(src, dst, t, 6, n=11),
                                  both(perm[src], perm[dst], t, 6, n=11))


def test_local_threads_agree():
    src, dst, t = random_graph(1234, 300, 6000, 2000, multi=0.2)
    a = oracle.local4(src, dst, t, 60, threads=1)
    b = oracle.local4(src, dst, t, 60, threads=4)
    np.testing.assert_array_equal(a, b)
