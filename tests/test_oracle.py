"""Pins for the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself:
  * values the paper prints for its toy graph (Sections III, IV-A, IV-B);
  * the brute-force enumeration of the definition (Definitions 2-3) on small
    random graphs with forced timestamp ties and multi-edges;
  * closed forms on hand-built pairs, stars and triangles;
  * labelled census identities (every class reached equally often);
  * invariants that hold at any size (relabelling, delta-monotonicity,
    edge reversal, time reversal, time shift/scale, disjoint union).
"""
from math import comb

import numpy as np
import pytest

import graphgen
import oracle
from motif_defs import (GRID, IN, O, canon_edge_reversal, canon_from_raw, canon_time_reversal,
                        cell, disjoint_union, edges, grid_from_canon, i_pair, i_star, i_tri,
                        load_toy, relabel, reverse_edges, reverse_time)

A, B, C, Dn, E = range(5)


def only(raw, expected: dict):
    """raw must equal ``expected`` (index -> value) and be zero elsewhere."""
    want = np.zeros(56, dtype=np.uint64)
    for k, v in expected.items():
        want[k] = v
    np.testing.assert_array_equal(raw, want)


# --------------------------------------------------------------------------
# values printed in the paper for its toy graph

def test_toy_star_center_a_paper_example():
    """Section IV-A walks FAST-Star through center a at delta = 10 s and
    finds exactly four instances: Star[III,o,o,in], Star[III,o,o,o],
    Star[II,o,in,o] and Star[II,o,o,o] (no pair instance at a)."""
    src, dst, t = load_toy()
    raw = oracle.alg_centers(src, dst, t, 10, [A], n=5)
    star_pair = raw.copy()
    star_pair[32:] = 0
    only(star_pair, {i_star("III", "o", "o", "in"): 1, i_star("III", "o", "o", "o"): 1,
                     i_star("II", "o", "in", "o"): 1, i_star("II", "o", "o", "o"): 1})


def test_toy_triangle_center_e_paper_example():
    """Section IV-B walks FAST-Tri through center e at delta = 10 s: one
    Tri[III,o,o,o] (e_i = (1,d,o), e_j = (6,c,o), e_k = d->c at 10) and one
    Type-II instance (e_i = (6,c,o), e_j = (14,d,in), e_k = d->c at 10).
    The text prints the latter as Tri[II,o,in,o]; with e_k's direction taken
    relative to v = e_i.v = c as the same section defines it, d->c enters c,
    so the cell is Tri[II,o,in,in] (the printed third index is a typo)."""
    src, dst, t = load_toy()
    raw = oracle.alg_centers(src, dst, t, 10, [E], n=5)
    tri = raw.copy()
    tri[:32] = 0
    only(tri, {i_tri("III", "o", "o", "o"): 1, i_tri("II", "o", "in", "in"): 1})


def test_three_views_of_one_triangle():
    """Section IV-B: <(a,c,8), (d,a,9), (c,d,17)> is one instance of M25 that
    FAST-Tri records as Tri[III,o,in,o] from a, Tri[II,in,o,in] from c and
    Tri[I,o,in,o] from d."""
    src, dst, t = edges([("a", "c", 8), ("d", "a", 9), ("c", "d", 17)])
    big = 100
    assert oracle.alg_centers(src, dst, t, big, [A], n=5)[i_tri("III", "o", "in", "o")] == 1
    assert oracle.alg_centers(src, dst, t, big, [C], n=5)[i_tri("II", "in", "o", "in")] == 1
    assert oracle.alg_centers(src, dst, t, big, [Dn], n=5)[i_tri("I", "o", "in", "o")] == 1
    raw = oracle.alg(src, dst, t, big, n=5)
    assert raw[32:].sum() == 3
    grid = oracle.merge(raw)
    assert grid[1, 4] == 1 and grid.sum() == 1          # M25


@pytest.mark.parametrize("rows,row,col", [
    # Section III names these three instances in the toy graph
    ([("a", "c", 4), ("a", "c", 8), ("d", "a", 9)], 6, 3),     # M63
    ([("e", "c", 6), ("d", "c", 10), ("d", "e", 14)], 4, 6),   # M46
    ([("d", "e", 14), ("e", "d", 18), ("d", "e", 21)], 6, 5),  # M65
])
def test_named_instances(rows, row, col):
    src, dst, t = edges(rows)
    grid = oracle.count(src, dst, t, 100, n=5)
    want = np.zeros((6, 6), dtype=np.uint64)
    want[row - 1, col - 1] = 1
    np.testing.assert_array_equal(grid, want)
    _, canon = oracle.brute(src, dst, t, 100, n=5)
    np.testing.assert_array_equal(grid_from_canon(canon), want)


def test_m24_is_star_type1_in_o_in():
    """Section IV-A: Star[I,in,o,in] records M24 (first edge isolated and
    into the center, then out to and back in from another node)."""
    src, dst, t = edges([(1, 0, 1), (0, 2, 2), (2, 0, 3)])
    raw = oracle.alg(src, dst, t, 10, n=3)
    only(raw, {i_star("I", "in", "o", "in"): 1})
    assert oracle.merge(raw)[1, 3] == 1


def test_toy_full_brute_equals_alg():
    src, dst, t = load_toy()
    for delta in (0, 1, 5, 10, 20, 100):
        raw = oracle.alg(src, dst, t, delta, n=5)
        braw, canon = oracle.brute(src, dst, t, delta, n=5)
        np.testing.assert_array_equal(raw, braw)
        np.testing.assert_array_equal(oracle.merge(raw), grid_from_canon(canon))


def _toy_instances():
    """The hand enumeration of every instance of the toy graph at delta = 10
    (tests/golden/toy_delta10_instances.txt)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "toy_delta10_instances.txt")
    out = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                w = line.split()
                out.append(([int(x[1:]) - 1 for x in w[:3]], w[3], w[4:]))
    return out


def test_toy_graph_all_instances_at_delta_10():
    """The toy graph of Figure 1 at delta = 10 s holds exactly 27 instances
    (19 stars, 1 pair, 7 triangles), including every instance the paper
    names in Sections III, IV-A and IV-B.  Each listed triple, counted on its
    own, is exactly one instance of its listed class; the whole graph counts
    exactly the listed instances, cell by cell."""
    src, dst, t = load_toy()
    inst = _toy_instances()
    assert len(inst) == 27
    assert [k for _, k, _ in inst].count("star") == 19
    assert [k for _, k, _ in inst].count("pair") == 1
    assert [k for _, k, _ in inst].count("tri") == 7
    assert len({tuple(e) for e, _, _ in inst}) == 27
    want = np.zeros(36, dtype=np.uint64)
    for e3, kind, f in inst:
        assert t[e3[2]] - t[e3[0]] <= 10
        if kind == "star":
            key = ("star", TYPES_[f[1]], D_[f[2]], D_[f[3]], D_[f[4]])
        elif kind == "pair":
            assert f[0] == "o"
            key = ("pair", D_[f[1]], D_[f[2]])
        else:
            key = ("tri", D_[f[0]], D_[f[1]], D_[f[2]])
        one = np.zeros(36, dtype=np.uint64)
        one[GRID[key]] = 1
        sel = np.array(e3)
        np.testing.assert_array_equal(oracle.count(src[sel], dst[sel], t[sel], 10, n=5).reshape(-1),
                                      one, err_msg=f"E{e3[0] + 1} E{e3[1] + 1} E{e3[2] + 1}")
        if kind == "star":
            center = "abcde".index(f[0])
            raw = oracle.alg_centers(src[sel], dst[sel], t[sel], 10, [center], n=5)
            assert raw[i_star(f[1], f[2], f[3], f[4])] == 1 and raw[:24].sum() == 1
        want[GRID[key]] += 1
    grid = oracle.count(src, dst, t, 10, n=5)
    np.testing.assert_array_equal(grid.reshape(-1), want)
    # the same 6 x 6, written out
    np.testing.assert_array_equal(grid, np.array([[0, 2, 0, 0, 0, 2],
                                                  [0, 1, 3, 0, 1, 1],
                                                  [2, 1, 1, 0, 0, 0],
                                                  [1, 2, 1, 0, 2, 1],
                                                  [0, 1, 1, 0, 0, 0],
                                                  [1, 1, 1, 0, 1, 0]], dtype=np.uint64))
    assert int(grid.sum()) == 27
    _, canon = oracle.brute(src, dst, t, 10, n=5)
    np.testing.assert_array_equal(grid_from_canon(canon).reshape(-1), want)


TYPES_ = {"I": 0, "II": 1, "III": 2}
D_ = {"o": O, "in": IN}


# --------------------------------------------------------------------------
# brute force of the definition vs the paper's algorithms

@pytest.mark.parametrize("seed", range(40))
def test_brute_vs_alg_random(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 9))
    m = int(rng.integers(0, 70))
    tv = int(rng.integers(1, 12)) if seed % 2 == 0 else None
    g = graphgen.small_random(rng, n, m, t_values=tv, tmax=int(rng.integers(1, 60)),
                              multi=0.3 if seed % 3 == 0 else 0.0)
    span = int(g.t.max() - g.t.min()) if m else 0
    for delta in sorted({0, 1, max(span // 3, 0), span, span + 5}):
        raw = oracle.alg(g.src, g.dst, g.t, delta, n=n)
        braw, canon = oracle.brute(g.src, g.dst, g.t, delta, n=n)
        np.testing.assert_array_equal(raw, braw, err_msg=f"seed {seed} delta {delta}")
        np.testing.assert_array_equal(canon_from_raw(raw), canon)
        np.testing.assert_array_equal(oracle.merge(raw), grid_from_canon(canon))


def test_brute_vs_alg_tiny_config():
    g = graphgen.tiny()
    raw = oracle.alg(g.src, g.dst, g.t, 1000, n=g.n)
    braw, canon = oracle.brute(g.src, g.dst, g.t, 1000, n=g.n)
    np.testing.assert_array_equal(raw, braw)
    np.testing.assert_array_equal(oracle.merge(raw), grid_from_canon(canon))


def test_brute_vs_alg_dense_ties():
    """A denser graph where many instances exist and timestamps tie a lot."""
    rng = np.random.default_rng(7)
    g = graphgen.small_random(rng, 12, 400, t_values=40, tmax=2000, multi=0.2)
    for delta in (0, 30, 200):
        raw = oracle.alg(g.src, g.dst, g.t, delta, n=12)
        braw, canon = oracle.brute(g.src, g.dst, g.t, delta, n=12)
        assert canon.sum() > 100
        np.testing.assert_array_equal(raw, braw)


# --------------------------------------------------------------------------
# closed forms

def test_pair_run_closed_form():
    """n edges u->v at t = 1..n, window w: every instance is M55 and there are
    sum_i C(min(w, n-i), 2) of them (E1 at time i, E2 and E3 any two of the
    min(w, n-i) later edges inside the window)."""
    for n_e, w in [(10, 3), (25, 7), (12, 100)]:
        src = np.zeros(n_e, np.int32)
        dst = np.ones(n_e, np.int32)
        t = np.arange(1, n_e + 1, dtype=np.int64)
        grid = oracle.count(src, dst, t, w, n=2)
        want = np.zeros((6, 6), np.uint64)
        want[4, 4] = sum(comb(min(w, n_e - i), 2) for i in range(1, n_e + 1))
        np.testing.assert_array_equal(grid, want)


def test_pair_alternating_closed_form():
    """Alternating directions u->v, v->u, ... at t = 1..n, all inside delta:
    for indices i < j < k, seen from p = src(E_i), E_j leaves p iff j - i is
    even and E_k leaves p iff k - i is even; count index triples per class."""
    n_e = 11
    src = np.array([0 if k % 2 == 0 else 1 for k in range(n_e)], np.int32)
    dst = 1 - src
    t = np.arange(1, n_e + 1, dtype=np.int64)
    want = np.zeros((6, 6), np.uint64)
    for i in range(n_e):
        for j in range(i + 1, n_e):
            for k in range(j + 1, n_e):
                d2 = O if (j - i) % 2 == 0 else IN
                d3 = O if (k - i) % 2 == 0 else IN
                want.flat[GRID[("pair", d2, d3)]] += 1
    np.testing.assert_array_equal(oracle.count(src, dst, t, 1000, n=2), want)


def test_star_blocks_closed_form():
    """Center 0, L leaves, r edges 0 -> leaf each, leaf blocks in time order,
    all inside delta: Star[I,o,o,o] = Star[III,o,o,o] = C(L,2) r C(r,2),
    Star-II = 0, M55 = L C(r,3), no triangles."""
    for L, r in [(3, 2), (4, 3), (5, 4)]:
        rows = []
        tt = 1
        for leaf in range(1, L + 1):
            for _ in range(r):
                rows.append((0, leaf, tt))
                tt += 1
        src, dst, t = edges(rows)
        raw = oracle.alg(src, dst, t, 10 ** 6, n=L + 1)
        s = comb(L, 2) * r * comb(r, 2)
        p = L * comb(r, 3)
        only(raw, {i_star("I", "o", "o", "o"): s, i_star("III", "o", "o", "o"): s,
                   i_pair("o", "o", "o"): p, i_pair("in", "in", "in"): p})


def test_triangle_cycle_and_variant():
    """x->y@1, y->z@2, z->x@3 within delta is one time-respecting cycle (M26);
    the same edges at times 1, 3, 2 are one M25; beyond delta, nothing."""
    src, dst, t = edges([(0, 1, 1), (1, 2, 2), (2, 0, 3)])
    g = oracle.count(src, dst, t, 2, n=3)
    assert g[1, 5] == 1 and g.sum() == 1
    assert oracle.count(src, dst, t, 1, n=3).sum() == 0
    src, dst, t = edges([(0, 1, 1), (1, 2, 3), (2, 0, 2)])
    g = oracle.count(src, dst, t, 2, n=3)
    assert g[1, 4] == 1 and g.sum() == 1


# --------------------------------------------------------------------------
# labelled census: every class is reached equally often

def test_census_pairs():
    """The 8 orientation patterns of 3 time-ordered edges on 2 nodes give each
    of the 4 pair motifs exactly twice."""
    tot = np.zeros((6, 6), np.uint64)
    for bits in range(8):
        rows = [((bits >> k) & 1, 1 - ((bits >> k) & 1), k + 1) for k in range(3)]
        tot += oracle.count(*edges(rows), 10, n=2)
    for key in [("pair", O, O), ("pair", O, IN), ("pair", IN, O), ("pair", IN, IN)]:
        assert tot.flat[GRID[key]] == 2
    assert tot.sum() == 8


def test_census_stars():
    """Center 0, leaf 1 with two edges and leaf 2 with one: 3 positions of the
    lone edge x 8 orientations = 24 graphs, each star motif exactly once."""
    tot = np.zeros((6, 6), np.uint64)
    raw_tot = np.zeros(56, np.uint64)
    for lone in range(3):
        for bits in range(8):
            rows = []
            for k in range(3):
                leaf = 2 if k == lone else 1
                out = (bits >> k) & 1 == 0
                rows.append((0, leaf, k + 1) if out else (leaf, 0, k + 1))
            src, dst, t = edges(rows)
            raw = oracle.alg(src, dst, t, 10, n=3)
            raw_tot += raw
            tot += oracle.merge(raw)
    np.testing.assert_array_equal(raw_tot[:24], np.ones(24, np.uint64))
    assert raw_tot[24:].sum() == 0
    for key, c in GRID.items():
        if key[0] == "star":
            assert tot.flat[c] == 1


def test_census_triangles():
    """Three node pairs of a triangle in all 3! time orders x 2^3 orientations
    = 48 labelled graphs; the symmetric group acts freely, so each of the 8
    triangle motifs appears exactly 6 times."""
    import itertools
    pairs = [(0, 1), (0, 2), (1, 2)]
    tot = np.zeros((6, 6), np.uint64)
    for order in itertools.permutations(range(3)):
        for bits in range(8):
            rows = []
            for pos, pi in enumerate(order):
                a, b = pairs[pi]
                if (bits >> pi) & 1:
                    a, b = b, a
                rows.append((a, b, pos + 1))
            tot += oracle.count(*edges(rows), 10, n=3)
    for key, c in GRID.items():
        if key[0] == "tri":
            assert tot.flat[c] == 6
    assert tot.sum() == 48


# --------------------------------------------------------------------------
# invariants (hold at any size)

def _mid_graph(seed, n=40, m=1500):
    rng = np.random.default_rng(seed)
    return graphgen.small_random(rng, n, m, t_values=300, tmax=5000, multi=0.25)


@pytest.mark.parametrize("seed", [1, 2])
def test_invariants(seed):
    g = _mid_graph(seed)
    n = g.n
    delta = 120
    base = oracle.alg(g.src, g.dst, g.t, delta, n=n)
    cb = canon_from_raw(base)
    rng = np.random.default_rng(seed)
    # node relabelling
    np.testing.assert_array_equal(oracle.alg(*relabel(g.src, g.dst, g.t, n, rng), delta, n=n), base)
    # time shift and scale (with delta)
    np.testing.assert_array_equal(oracle.alg(g.src, g.dst, g.t + 123456789, delta, n=n), base)
    np.testing.assert_array_equal(oracle.alg(g.src, g.dst, g.t * 7, delta * 7, n=n), base)
    # edge reversal
    rev = oracle.alg(*reverse_edges(g.src, g.dst, g.t), delta, n=n)
    np.testing.assert_array_equal(canon_from_raw(rev), canon_edge_reversal(cb))
    # time reversal
    trev = oracle.alg(*reverse_time(g.src, g.dst, g.t), delta, n=n)
    np.testing.assert_array_equal(canon_from_raw(trev), canon_time_reversal(cb))
    # delta monotone
    prev = np.zeros(36, np.uint64)
    for d in (0, 10, 60, 120, 500, 5000):
        cur = oracle.merge(oracle.alg(g.src, g.dst, g.t, d, n=n)).ravel()
        assert (cur >= prev).all()
        prev = cur
    # disjoint union adds
    h = _mid_graph(seed + 10, n=30, m=900)
    u = disjoint_union((g.src, g.dst, g.t), (h.src, h.dst, h.t), n)
    both = oracle.alg(*u, delta, n=n + 30)
    np.testing.assert_array_equal(both, base + oracle.alg(h.src, h.dst, h.t, delta, n=30))


def test_time_reversal_maps_m13_to_m53():
    """Time reversal swaps Star-I and Star-III; M13 = Star[I,o,o,o] and
    M53 = Star[III,o,o,o] are a reversal pair (the paper's WikiTalk counts
    for them are nearly equal, Section V-C)."""
    c = np.zeros(36, np.uint64)
    c[i_star("I", "o", "o", "o")] = 1
    r = canon_time_reversal(c)
    assert r[i_star("III", "o", "o", "o")] == 1 and r.sum() == 1
    assert GRID[("star", 0, O, O, O)] == cell(1, 3)
    assert GRID[("star", 2, O, O, O)] == cell(5, 3)


# --------------------------------------------------------------------------
# layout anchors, merge self-checks and input validation

def test_oracle_layout_matches_spec():
    for key, c in GRID.items():
        if key[0] == "star":
            assert oracle.layout_star(*key[1:]) == c
        elif key[0] == "pair":
            assert oracle.layout_pair(*key[1:]) == c
        else:
            assert oracle.layout_tri(*key[1:]) == c
    assert sorted(GRID.values()) == list(range(36))


def test_layout_anchors():
    assert GRID[("star", 0, IN, O, IN)] == cell(2, 4)      # M24
    assert GRID[("star", 2, O, O, IN)] == cell(6, 3)       # M63
    assert GRID[("tri", O, IN, O)] == cell(2, 5)           # M25
    assert GRID[("tri", IN, O, IN)] == cell(2, 6)          # M26
    assert GRID[("tri", O, O, IN)] == cell(4, 6)           # M46
    assert GRID[("pair", O, O)] == cell(5, 5)              # M55
    assert GRID[("pair", IN, IN)] == cell(5, 6)            # M56
    assert GRID[("pair", IN, O)] == cell(6, 5)             # M65
    assert GRID[("pair", O, IN)] == cell(6, 6)             # M66


def test_merge_rejects_broken_symmetry():
    raw = np.zeros(56, np.uint64)
    raw[i_pair("o", "o", "o")] = 1                         # missing mirror view
    with pytest.raises(oracle.OracleError):
        oracle.merge(raw)
    raw = np.zeros(56, np.uint64)
    raw[i_tri("I", "o", "o", "o")] = 1                     # orbit incomplete
    with pytest.raises(oracle.OracleError):
        oracle.merge(raw)


@pytest.mark.parametrize("bad", ["selfloop", "range", "neg", "time"])
def test_validation(bad):
    src = np.array([0, 1, 2], np.int32)
    dst = np.array([1, 2, 0], np.int32)
    t = np.array([1, 2, 3], np.int64)
    if bad == "selfloop":
        dst[0] = 0
    elif bad == "range":
        dst[1] = 7
    elif bad == "neg":
        src[2] = -1
    else:
        t[1] = 1 << 62
    with pytest.raises(oracle.OracleError):
        oracle.alg(src, dst, t, 5, n=3)
    with pytest.raises(oracle.OracleError):
        oracle.brute(src, dst, t, 5, n=3)


def test_empty_and_tiny():
    e = np.zeros(0, np.int32)
    assert oracle.alg(e, e, np.zeros(0, np.int64), 5, n=3).sum() == 0
    src, dst, t = edges([(0, 1, 1), (1, 0, 2)])
    assert oracle.alg(src, dst, t, 5, n=2).sum() == 0
    with pytest.raises(oracle.OracleError):
        oracle.alg(src, dst, t, -1, n=2)
