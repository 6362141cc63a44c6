"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Counts are integers, so the bar is bit-exact equality of all 56 raw counters
(and hence of the 36 motif counts) on the same seeded inputs.
"""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from motif_defs import edges, load_toy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2204_09236_amd as p
    return p


def case(msg):
    print(f"[case] {msg}", flush=True)


def gpu_raw(tm, src, dst, t, delta, n=None, **kw):
    with tm.build_graph(src, dst, t, n=n) as g:
        return g.count_raw(delta, **kw)


# hub_min settings every check runs: the default threshold, every triangle
# candidate through the slice kernel (1: any non-empty larger window), and
# the slice kernel off
HUB_SETTINGS = (0, 1, 0xFFFFFFFF)


def check(tm, src, dst, t, deltas, n=None, label=""):
    with tm.build_graph(src, dst, t, n=n) as g:
        for d in deltas:
            case(f"{label} m={len(src)} n={n} delta={d}")
            want = oracle.alg(src, dst, t, d, n=n)
            for hub in HUB_SETTINGS:
                got = g.count_raw(d, hub_min=hub)
                np.testing.assert_array_equal(got, want, err_msg=f"{label} delta={d} hub_min={hub}")
            np.testing.assert_array_equal(g.count(d), oracle.merge(want))


def test_toy_graph(tm):
    src, dst, t = load_toy()
    check(tm, src, dst, t, [0, 1, 5, 10, 20, 100], n=5, label="toy")


@pytest.mark.parametrize("seed", range(24))
def test_random_small(tm, seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(3, 10))
    m = int(rng.integers(3, 80))
    g = graphgen.small_random(rng, n, m, t_values=int(rng.integers(1, 15)) if seed % 2 else None,
                              tmax=int(rng.integers(1, 80)), multi=0.3 if seed % 3 == 0 else 0.0)
    span = int(g.t.max() - g.t.min())
    check(tm, g.src, g.dst, g.t, sorted({0, 1, span // 3, span, span + 7}), n=n,
          label=f"small seed={seed}")


@pytest.mark.parametrize("seed,n,m,tv", [(1, 30, 3000, 200), (2, 200, 20000, None),
                                          (3, 12, 5000, 50), (4, 1000, 60000, 5000)])
def test_random_medium(tm, seed, n, m, tv):
    rng = np.random.default_rng(seed)
    g = graphgen.small_random(rng, n, m, t_values=tv, tmax=100000, multi=0.2)
    check(tm, g.src, g.dst, g.t, [0, 50, 1000, 20000], n=n, label=f"medium seed={seed}")


def test_tiny_config(tm):
    g = graphgen.tiny()
    check(tm, g.src, g.dst, g.t, [1000], n=g.n, label="tiny config")


def test_sequences_match_definition(tm):
    """S_u = every node's incident edges in (t, id) order (byte for byte)."""
    rng = np.random.default_rng(11)
    g = graphgen.small_random(rng, 50, 4000, t_values=300, tmax=10000, multi=0.3)
    case("sequences m=4000")
    with tm.build_graph(g.src, g.dst, g.t, n=50) as G:
        seq = G.sequences()
    m = g.m
    ids = np.arange(m)
    node = np.concatenate([g.src, g.dst]).astype(np.int64)
    nbr = np.concatenate([g.dst, g.src]).astype(np.int64)
    dr = np.concatenate([np.zeros(m), np.ones(m)]).astype(np.uint8)
    tt = np.concatenate([g.t, g.t])
    eid = np.concatenate([ids, ids])
    order = np.lexsort((eid, tt, node))
    off = np.searchsorted(node[order], np.arange(51))
    np.testing.assert_array_equal(seq["off"], off)
    np.testing.assert_array_equal(seq["t"], tt[order])
    np.testing.assert_array_equal(seq["nbr"], nbr[order])
    np.testing.assert_array_equal(seq["dir"], dr[order])
    np.testing.assert_array_equal(seq["id"], eid[order])


def test_partitioning_invariance(tm):
    """Chunk size of the node-pair sweeps and the lane/wave split of the
    triangle kernel change the schedule, never the counts."""
    rng = np.random.default_rng(21)
    g = graphgen.small_random(rng, 20, 6000, t_values=400, tmax=20000, multi=0.5)
    want = oracle.alg(g.src, g.dst, g.t, 800, n=20)
    with tm.build_graph(g.src, g.dst, g.t, n=20) as G:
        for rc in (1, 2, 3, 7, 64, 1 << 30):
            for lm in (1, 4, 64, 1 << 30):
                case(f"partition run_chunk={rc} tri_lane_max={lm}")
                np.testing.assert_array_equal(G.count_raw(800, run_chunk=rc, tri_lane_max=lm), want)
        for hub in (1, 2, 3, 8, 50, 200, 0xFFFFFFFF):
            case(f"partition hub_min={hub}")
            np.testing.assert_array_equal(G.count_raw(800, hub_min=hub), want)


def test_hub_pair_long_run(tm):
    """One node pair with 8,000 edges inside one window (a long E_(v,w))
    plus background edges: exercises chunking with large delta-halos."""
    rng = np.random.default_rng(31)
    k = 8000
    src = np.where(rng.random(k) < 0.5, 0, 1).astype(np.int32)
    dst = (1 - src).astype(np.int32)
    t = rng.integers(0, 3000, k).astype(np.int64)
    bg = graphgen.small_random(rng, 40, 3000, tmax=3000)
    s = np.concatenate([src, bg.src]); d = np.concatenate([dst, bg.dst])
    tt = np.concatenate([t, bg.t])
    check(tm, s, d, tt, [100, 5000], n=40, label="hub pair")


def test_star_hub(tm):
    """A center with 6,000 edges to 150 leaves plus edges among the leaves."""
    rng = np.random.default_rng(32)
    k = 6000
    leaf = rng.integers(1, 151, k).astype(np.int32)
    out = rng.random(k) < 0.5
    src = np.where(out, 0, leaf).astype(np.int32)
    dst = np.where(out, leaf, 0).astype(np.int32)
    t = rng.integers(0, 50000, k).astype(np.int64)
    bg = graphgen.small_random(rng, 151, 8000, tmax=50000)
    s = np.concatenate([src, bg.src]); d = np.concatenate([dst, bg.dst])
    tt = np.concatenate([t, bg.t])
    # at delta 50000 the center's window spans ~6,000 entries: the slice
    # kernel's union windows take several LDS segments
    check(tm, s, d, tt, [0, 300, 5000, 50000], n=151, label="star hub")


def test_all_timestamps_equal(tm):
    rng = np.random.default_rng(41)
    g = graphgen.small_random(rng, 15, 600, multi=0.3)
    t = np.full(g.m, 77, np.int64)
    check(tm, g.src, g.dst, t, [0, 10], n=15, label="all ties")


def test_fewer_than_three_edges(tm):
    for rows in ([], [(0, 1, 5)], [(0, 1, 5), (1, 0, 6)]):
        src, dst, t = edges(rows) if rows else (np.zeros(0, np.int32),) * 2 + (np.zeros(0, np.int64),)
        case(f"m={len(rows)}")
        assert gpu_raw(tm, src, dst, t, 10, n=2).sum() == 0
    src, dst, t = edges([(0, 1, 1), (1, 2, 2), (2, 0, 3)])
    np.testing.assert_array_equal(gpu_raw(tm, src, dst, t, 2, n=3), oracle.alg(src, dst, t, 2, n=3))


def test_isolated_nodes_and_large_ids(tm):
    rng = np.random.default_rng(51)
    g = graphgen.small_random(rng, 60, 5000, t_values=500, tmax=5000, multi=0.2)
    ids = np.sort(rng.choice(1 << 26, 60, replace=False)).astype(np.int32)
    src, dst = ids[g.src], ids[g.dst]
    n = (1 << 26) + 5
    check(tm, src, dst, g.t, [0, 200], n=n, label="sparse ids")


def test_negative_and_extreme_times(tm):
    rng = np.random.default_rng(52)
    g = graphgen.small_random(rng, 25, 3000, t_values=200, tmax=4000, multi=0.2)
    big = (1 << 62) - 10_000
    for shift in (-big, big - 5000, -(1 << 40)):
        t = g.t + shift
        check(tm, g.src, g.dst, t, [0, 100, 3000], n=25, label=f"t shift {shift}")


def test_device_pointer_input(tm):
    import torch
    rng = np.random.default_rng(61)
    g = graphgen.small_random(rng, 100, 20000, t_values=2000, tmax=100000, multi=0.2)
    dev = torch.device("cuda:0")
    s = torch.from_numpy(g.src).to(dev)
    d = torch.from_numpy(g.dst).to(dev)
    t = torch.from_numpy(g.t).to(dev)
    case("device pointers m=20000")
    with tm.build_graph(s, d, t, n=100) as G:
        got = G.count_raw(2000)
    np.testing.assert_array_equal(got, oracle.alg(g.src, g.dst, g.t, 2000, n=100))


def test_invalid_inputs(tm):
    src, dst, t = edges([(0, 1, 1), (1, 2, 2), (2, 0, 3)])
    for s, d, tt, n in [(src, np.array([1, 1, 0], np.int32), t, 3),          # self-loop
                        (src, np.array([1, 5, 0], np.int32), t, 3),          # id >= n
                        (np.array([-1, 1, 2], np.int32), dst, t, 3),         # negative id
                        (src, dst, np.array([1, 1 << 62, 3], np.int64), 3)]:  # |t| too big
        case("invalid input")
        with pytest.raises(tm.TMError) as ei:
            tm.build_graph(s, d, tt, n=n)
        assert ei.value.code == -1
    with tm.build_graph(src, dst, t, n=3) as G:
        with pytest.raises(tm.TMError):
            G.count(-1)


def test_lookback_giveup_fails_cleanly(tm):
    """Every radix-sort tile gives up its look-back wait at once (forced from
    the host): the sorts then leave some output positions unwritten, with
    stale contents, and the build must stop with TM_EINTERNAL while every
    kernel stays in bounds (node offsets are not written from keys >= n).
    The next build with the normal bound is exact again."""
    g = graphgen.chung_lu_pareto(31, 20_000, 200_000)
    case("forced look-back give-up m=200000")
    tm.debug_lookback_giveup(True)
    try:
        for _ in range(2):
            with pytest.raises(tm.TMError) as ei:
                tm.build_graph(g.src, g.dst, g.t, n=g.n)
            assert ei.value.code == -6
    finally:
        tm.debug_lookback_giveup(False)
    case("build after the forced give-up")
    with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
        np.testing.assert_array_equal(G.count_raw(3600), oracle.alg(g.src, g.dst, g.t, 3600, n=g.n))


@pytest.mark.parametrize("m", [12, 9000, 20_000, 200_000, 5_000_000])
def test_edge_index_by_partition(tm, m):
    """Each edge's two positions built by the partition of (slot, position)
    pairs and the bucket fill (taken by graphs whose index outgrows the
    last-level cache), forced at small sizes: no sort pass (under 2^15
    slots), one pass, two passes; ragged last buckets."""
    if m == 12:
        src, dst, t = load_toy()
        n = 5
    else:
        g = graphgen.chung_lu_pareto(40 + m % 97, max(3, m // 20), m)
        src, dst, t, n = g.src, g.dst, g.t, g.n
    tm.debug_force_edge_sort(True)
    try:
        check(tm, src, dst, t, [0, 3600, 86400] if m > 12 else [10], n=n, label=f"edge index m={m}")
        if m == 200_000:
            case("edge index with forced look-back give-up")
            tm.debug_lookback_giveup(True)
            try:
                with pytest.raises(tm.TMError) as ei:
                    tm.build_graph(src, dst, t, n=n)
                assert ei.value.code == -6
            finally:
                tm.debug_lookback_giveup(False)
    finally:
        tm.debug_force_edge_sort(False)


def test_repeatable(tm):
    rng = np.random.default_rng(71)
    g = graphgen.small_random(rng, 300, 50000, t_values=5000, tmax=200000, multi=0.3)
    case("repeat m=50000")
    with tm.build_graph(g.src, g.dst, g.t, n=300) as G:
        a = G.count_raw(4000)
        b = G.count_raw(4000)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("delta", [3600, 86400, 1_000_000])
def test_powerlaw_scaled(tm, delta):
    """The power-law generator at 1/50 scale (20K nodes, 400K edges)."""
    g = graphgen.chung_lu_pareto(101, 20_000, 400_000)
    check(tm, g.src, g.dst, g.t, [delta], n=g.n, label="powerlaw/50")


def test_skewed_scaled(tm):
    """The skewed generator (repeats, hub) at 1/1000 scale."""
    g = graphgen.skewed(seed=102, n=10_000, m=300_000, top_degree=1000)
    check(tm, g.src, g.dst, g.t, [600, 3600, 86400], n=g.n, label="skewed/1000")


def test_skewed_hub_heavy(tm):
    """The skewed generator at 1/100 scale (100K nodes, 3M edges, 20 % repeats)
    with a hub of ~1.2e5 incident edges: long node-pair runs that the hub
    split cuts into many chunks, and wide triangle windows at delta 86400."""
    g = graphgen.skewed(seed=103, n=100_000, m=3_000_000, top_degree=100_000)
    check(tm, g.src, g.dst, g.t, [600, 3600, 86400], n=g.n, label="skewed/100 hub-heavy")


def test_powerlaw_full_size(tm):
    """The benchmark workload at full size (1M nodes, 20M edges, delta 3600),
    built from device pointers on the current stream as bench.py does, against
    the oracle's counts stored by tests/golden/make_golden.py (or the oracle
    run here if this host regenerates a different edge list)."""
    import torch
    rec = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "powerlaw_counts.json")))
    g = graphgen.powerlaw()
    same_input = graphgen.edge_hash(g) == rec["edge_sha256"]
    dev = torch.device("cuda:0")
    s, d, t = (torch.from_numpy(a).to(dev) for a in (g.src, g.dst, g.t))
    for key, val in rec["counts"].items():
        delta = int(key)
        case(f"powerlaw full m={g.m} delta={delta} stored={same_input}")
        with tm.build_graph(s, d, t, n=g.n) as G:
            got = G.count_raw(delta)
        if same_input:
            want = np.array(val["raw"], dtype=np.uint64)
        else:
            want = oracle.alg(g.src, g.dst, g.t, delta, n=g.n, threads=min(16, os.cpu_count()))
        np.testing.assert_array_equal(got, want)


def test_skewed_full_size(tm):
    """The large skewed workload at full size (10M nodes, 300M edges, 20 %
    repeated pairs, a hub of ~1e6 edges; delta 600 / 3,600 / 86,400), built
    from device pointers as bench.py does, against the oracle's counts stored
    by tests/golden/make_golden.py; at delta 86,400 also with the hub slice
    kernel off; the four-node motif counts at delta 600.  Skipped when this host regenerates a different edge list
    (the oracle takes minutes on it)."""
    import torch
    rec = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "skewed_counts.json")))
    case("skewed full: generating 300M edges")
    g = graphgen.skewed()
    if graphgen.edge_hash(g) != rec["edge_sha256"]:
        pytest.skip("the regenerated skewed edge list differs from the stored one")
    dev = torch.device("cuda:0")
    s, d, t = (torch.from_numpy(a).to(dev) for a in (g.src, g.dst, g.t))
    n = g.n
    del g
    with tm.build_graph(s, d, t, n=n) as G:
        for key, val in rec["counts"].items():
            delta = int(key)
            case(f"skewed full m=300000000 delta={delta}")
            want = np.array(val["raw"], dtype=np.uint64)
            np.testing.assert_array_equal(G.count_raw(delta), want, err_msg=f"delta={delta}")
            if delta == 86400:
                case("skewed full delta=86400 hub pass off")
                np.testing.assert_array_equal(G.count_raw(delta, hub_min=tm.HUB_OFF), want)
        # all windows in one pass, as the benchmark counts them
        deltas = [int(k) for k in rec["counts"]]
        case(f"skewed full, windows {deltas} in one pass")
        multi = G.count_multi_raw(deltas)
        for i, key in enumerate(rec["counts"]):
            np.testing.assert_array_equal(multi[i], np.array(rec["counts"][key]["raw"], dtype=np.uint64),
                                          err_msg=f"one pass, delta={key}")
        # four-node motifs (tm_count4) against the oracle's stored counts
        rec4 = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                           "motif4_counts.json")))["skewed"]
        assert rec4["edge_sha256"] == rec["edge_sha256"]
        for key, val in rec4["counts"].items():
            case(f"skewed full four-node motifs delta={key}")
            got, raw = G.count4(int(key), with_raw=True)
            np.testing.assert_array_equal(got, np.array(val["f4"], dtype=np.uint64))
            np.testing.assert_array_equal(raw, np.array(val["raw"], dtype=np.uint64))
    del s, d, t
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# batches: many graphs, one build, one count, per-graph delta

def _batch_graphs(seed, G, lo=0, hi=400):
    rng = np.random.default_rng(seed)
    graphs, deltas = [], []
    for i in range(G):
        m = int(rng.integers(lo, hi))
        n = int(rng.integers(2, 25))
        g = graphgen.small_random(rng, n, m, t_values=int(rng.integers(1, 60)) if i % 2 else None,
                                  tmax=int(rng.integers(1, 3000)), multi=0.3 if i % 3 == 0 else 0.0)
        graphs.append((g.src, g.dst, g.t, n if i % 4 else 0))
        deltas.append(int(rng.integers(0, 400)))
    return graphs, deltas


@pytest.mark.parametrize("seed,G", [(1, 1), (2, 7), (3, 64), (4, 300)])
def test_batch_matches_oracle_per_graph(tm, seed, G):
    graphs, deltas = _batch_graphs(seed, G)
    case(f"batch G={G} seed={seed}")
    with tm.build_batch(graphs) as B:
        assert B.num_graphs == G
        raw = B.count_batch_raw(deltas)
        grids = B.count_batch(deltas)
        # every candidate through the hub slices (tiles never cross graphs)
        raw_hub = B.count_batch_raw_ex(deltas, use_graph=False, hub_min=1)
    for i, (s, d, t, n) in enumerate(graphs):
        want = oracle.alg(s, d, t, deltas[i], n=n or None)
        np.testing.assert_array_equal(raw[i], want, err_msg=f"graph {i}")
        np.testing.assert_array_equal(raw_hub[i], want, err_msg=f"graph {i} hub_min=1")
        np.testing.assert_array_equal(grids[i], oracle.merge(want))


def test_batch_equals_single_graph_counts(tm):
    """A graph counted alone and the same graph inside a batch of uneven
    graphs (with empty and tiny members) give identical counts."""
    graphs, deltas = _batch_graphs(9, 40, lo=0, hi=2000)
    graphs.append((np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), 5))
    deltas.append(10)
    big = graphgen.chung_lu_pareto(77, 3000, 60_000)
    graphs.insert(5, (big.src, big.dst, big.t, big.n))
    deltas.insert(5, 86400)
    with tm.build_batch(graphs) as B:
        raw = B.count_batch_raw(deltas)
    for i, (s, d, t, n) in enumerate(graphs):
        case(f"batch member {i} alone m={len(s)}")
        with tm.build_graph(s, d, t, n=n or None) as G1:
            np.testing.assert_array_equal(G1.count_raw(deltas[i]), raw[i], err_msg=f"graph {i}")


def test_batch_device_pointers_and_repeat(tm):
    import torch
    graphs, deltas = _batch_graphs(12, 100, lo=50, hi=1500)
    src = np.concatenate([g[0] for g in graphs]); dst = np.concatenate([g[1] for g in graphs])
    t = np.concatenate([g[2] for g in graphs])
    off = np.zeros(len(graphs) + 1, np.uint64)
    off[1:] = np.cumsum([len(g[0]) for g in graphs])
    ncount = np.array([g[3] for g in graphs], np.uint32)
    dev = torch.device("cuda:0")
    case("batch device pointers G=100")
    with tm.build_batch_arrays(torch.from_numpy(src).to(dev), torch.from_numpy(dst).to(dev),
                               torch.from_numpy(t).to(dev), off, ncount) as B:
        a = B.count_batch_raw(deltas)
        b = B.count_batch_raw(deltas)
        c = B.count_batch_raw([0] * len(graphs))
    np.testing.assert_array_equal(a, b)
    for i, (s, d, tt, n) in enumerate(graphs):
        np.testing.assert_array_equal(a[i], oracle.alg(s, d, tt, deltas[i], n=n or None))
        np.testing.assert_array_equal(c[i], oracle.alg(s, d, tt, 0, n=n or None))


def test_batch_invalid_member(tm):
    graphs, deltas = _batch_graphs(13, 5, lo=10, hi=50)
    s, d, t, n = graphs[3]
    d = d.copy()
    d[0] = s[0]                                     # self-loop in graph 3
    graphs[3] = (s, d, t, n)
    case("batch invalid member")
    with pytest.raises(tm.TMError) as ei:
        tm.build_batch(graphs)
    assert ei.value.code == -1 and "graph 3" in str(ei.value)


def test_batch_graph_replays_match_eager(tm):
    """The captured hipGraph of a batch count, replayed several times with
    other eager GPU work and synchronisations in between, gives the eager
    result on every replay."""
    import torch
    graphs, deltas = _batch_graphs(21, 80, lo=20, hi=1500)
    rng = np.random.default_rng(5)
    with tm.build_batch(graphs) as B:
        for rep in range(4):
            ds = deltas if rep % 2 == 0 else list(rng.integers(0, 600, len(graphs)))
            case(f"graph replay {rep}")
            replay = B.count_batch_raw_ex(ds, use_graph=True)
            x = torch.randn(1 << 20, device="cuda")          # unrelated eager work
            _ = (x * 2).sum().item()
            torch.cuda.synchronize()
            eager = B.count_batch_raw_ex(ds, use_graph=False)
            np.testing.assert_array_equal(replay, eager)
            if rep == 0:
                for i, (s, d, t, n) in enumerate(graphs):
                    np.testing.assert_array_equal(replay[i], oracle.alg(s, d, t, ds[i], n=n or None))
        for rc, lm, hub in ((3, 16, 0), (1, 1, 0), (0, 0, 1), (0, 0, 0xFFFFFFFF)):
            case(f"graph replay params {rc} {lm} {hub}")
            np.testing.assert_array_equal(B.count_batch_raw_ex(deltas, rc, lm, True, hub_min=hub),
                                          B.count_batch_raw_ex(deltas, rc, lm, False, hub_min=hub))


def test_autotune_then_count(tm):
    g = graphgen.chung_lu_pareto(88, 5000, 150_000)
    with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
        case("autotune")
        best = G.autotune([86400])
        assert best["run_chunk"] in (2, 4, 8)
        assert best["tri_lane_max"] in (8, 32, 64, 256, 1024)
        assert best["hub_min"] in (16, 32, 64, 128, 256, 1024, 0xFFFFFFFF)
        assert best["ms"] > 0
        np.testing.assert_array_equal(G.count_raw(86400), oracle.alg(g.src, g.dst, g.t, 86400, n=g.n))


def test_autotune_multi_then_count(tm):
    """The several-window autotuner (k = 3, and k = 6 > four levels: the
    largest four are timed) keeps a valid choice; counts after it still equal
    the oracle's; a batch and bad arguments are rejected."""
    g = graphgen.chung_lu_pareto(89, 5000, 150_000)
    deltas = [600, 3600, 86400]
    with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
        for ds in (deltas, [0, 10, 60, 600, 3600, 86400]):
            case(f"autotune_multi {ds}")
            best = G.autotune_multi(ds)
            assert best["run_chunk"] in (2, 4, 8)
            assert best["tri_lane_max"] in (8, 32, 64, 256, 1024)
            assert best["hub_min"] in (16, 32, 64, 128, 256, 1024, 0xFFFFFFFF)
            assert best["ms"] > 0
        raw = G.count_multi_raw(deltas)
        for i, d in enumerate(deltas):
            np.testing.assert_array_equal(raw[i], oracle.alg(g.src, g.dst, g.t, d, n=g.n))
        for bad in ([], [-1, 5]):
            with pytest.raises(tm.TMError):
                G.autotune_multi(bad)
    src, dst, t = np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32), np.array([1, 2, 3])
    with tm.build_batch([(src, dst, t, 3), (src, dst, t, 3)]) as B:
        with pytest.raises(tm.TMError):
            B.autotune_multi([5, 10])


# motif-family masks (tm_count_masked): the selected cells equal the full
# count, the others are zero
STAR_CELLS = [(r, c) for r in range(6) for c in range(4)]
PAIR_CELLS = [(r, c) for r in (4, 5) for c in (4, 5)]
TRI_CELLS = [(r, c) for r in range(4) for c in (4, 5)]


@pytest.mark.parametrize("families", [1, 2, 3, 4, 5, 6, 7])
def test_masked_counts(tm, families):
    rng = np.random.default_rng(900 + families)
    g = graphgen.small_random(rng, 40, 3000, t_values=300, multi=0.3)
    big = graphgen.chung_lu_pareto(901, 20_000, 400_000)
    for src, dst, t, n, deltas in [(g.src, g.dst, g.t, g.n, [0, 5, 40]),
                                   (big.src, big.dst, big.t, big.n, [3600, 86400])]:
        with tm.build_graph(src, dst, t, n=n) as G:
            for d in deltas:
                case(f"masked families={families} m={len(src)} delta={d}")
                full = G.count(d)
                got = G.count(d, families=families)
                want = np.zeros_like(full)
                for bit, cells in ((1, STAR_CELLS), (2, PAIR_CELLS), (4, TRI_CELLS)):
                    if families & bit:
                        for rc in cells:
                            want[rc] = full[rc]
                np.testing.assert_array_equal(got, want)
                if d == deltas[0]:
                    np.testing.assert_array_equal(full, oracle.count(src, dst, t, d, n=n))


def test_masked_rejects_bad_families(tm):
    g = graphgen.chung_lu_pareto(902, 100, 1000)
    with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
        for bad in (0, 8, 9):
            with pytest.raises(tm.TMError) as ei:
                G.count(100, families=bad)
            assert ei.value.code == -1


# several windows in one call (tm_count_multi): each equals its own count
def test_count_multi_matches_oracle_per_delta(tm):
    rng = np.random.default_rng(71)
    g = graphgen.small_random(rng, 30, 4000, t_values=500, tmax=20000, multi=0.4)
    deltas = [0, 800, 50, 800, 20000, 3]           # any order, repeats allowed
    case(f"count_multi k={len(deltas)}")
    with tm.build_graph(g.src, g.dst, g.t, n=30) as G:
        raw = G.count_multi_raw(deltas)
        grids = G.count_multi(deltas)
    for i, d in enumerate(deltas):
        want = oracle.alg(g.src, g.dst, g.t, d, n=30)
        np.testing.assert_array_equal(raw[i], want, err_msg=f"delta={d}")
        np.testing.assert_array_equal(grids[i], oracle.merge(want))


def test_count_multi_equals_single_counts_skewed(tm):
    g = graphgen.skewed(seed=104, n=10_000, m=300_000, top_degree=1000)
    deltas = [600, 3600, 86400]
    case("count_multi skewed/1000")
    with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
        multi = G.count_multi_raw(deltas)
        for i, d in enumerate(deltas):
            np.testing.assert_array_equal(multi[i], G.count_raw(d), err_msg=f"delta={d}")
    np.testing.assert_array_equal(multi[1], oracle.alg(g.src, g.dst, g.t, 3600, n=g.n))


def test_count_multi_hub_heavy(tm):
    """Several windows in one pass on the hub-heavy skewed graph (1/100
    scale): the hub slice kernel and the per-candidate kernel both file
    their matches under window levels."""
    g = graphgen.skewed(seed=103, n=100_000, m=3_000_000, top_degree=100_000)
    deltas = [86400, 600, 3600]
    case("count_multi skewed/100 hub-heavy")
    with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
        multi = G.count_multi_raw(deltas)
    for i, d in enumerate(deltas):
        np.testing.assert_array_equal(multi[i], oracle.alg(g.src, g.dst, g.t, d, n=g.n),
                                      err_msg=f"delta={d}")


def test_count_multi_five_windows(tm):
    """Five windows: a pass of four and a pass of one, with equal windows
    inside a pass, against single counts and the oracle."""
    g = graphgen.chung_lu_pareto(105, 20_000, 400_000)
    deltas = [3600, 5, 86400, 600, 3600]
    case("count_multi powerlaw/50 k=5")
    with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
        multi = G.count_multi_raw(deltas)
        for i, d in enumerate(deltas):
            np.testing.assert_array_equal(multi[i], G.count_raw(d), err_msg=f"delta={d}")
    np.testing.assert_array_equal(multi[2], oracle.alg(g.src, g.dst, g.t, 86400, n=g.n))


def test_count_multi_rejects(tm):
    rng = np.random.default_rng(72)
    g = graphgen.small_random(rng, 8, 200)
    case("count_multi errors")
    with tm.build_graph(g.src, g.dst, g.t, n=8) as G:
        with pytest.raises(tm.TMError):
            G.count_multi([])
        with pytest.raises(tm.TMError):
            G.count_multi([10, -1])
    graphs, deltas = _batch_graphs(5, 3)
    with tm.build_batch(graphs) as B:
        with pytest.raises(tm.TMError):
            B.count_multi([10])


def test_hub_threshold_at_and_above_segment_cap(tm):
    """hub_min at and above the 2,048-entry LDS segment (the window levels
    then test W >= 2048 before W >= hub_min): a 6,000-edge center whose
    window at delta 50,000 spans several segments, leaves with small
    windows."""
    rng = np.random.default_rng(33)
    k = 6000
    leaf = rng.integers(1, 151, k).astype(np.int32)
    out = rng.random(k) < 0.5
    src = np.where(out, 0, leaf).astype(np.int32)
    dst = np.where(out, leaf, 0).astype(np.int32)
    t = rng.integers(0, 50000, k).astype(np.int64)
    bg = graphgen.small_random(rng, 151, 8000, tmax=50000)
    s = np.concatenate([src, bg.src]); d = np.concatenate([dst, bg.dst])
    tt = np.concatenate([t, bg.t])
    want = oracle.alg(s, d, tt, 50000, n=151)
    with tm.build_graph(s, d, tt, n=151) as G:
        for hub in (2047, 2048, 2049, 3000, 5000):
            case(f"hub_min={hub} delta=50000")
            np.testing.assert_array_equal(G.count_raw(50000, hub_min=hub), want)
