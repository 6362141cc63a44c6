"""The allocation-free count (tm_count_noalloc) against tm_count.

Counts are integers: the bar is equality of all 36 motif counts.  Two calls
in a row on one device share the library's fixed workspace; the second has
a smaller input, so any state the first call left behind would show."""
import numpy as np
import pytest

import graphgen
import oracle

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


def test_noalloc_matches_count_two_calls(tm):
    big = graphgen.chung_lu_pareto(61, 50_000, 1_000_000)
    small = graphgen.chung_lu_pareto(62, 3_000, 40_000)
    with tm.build_graph(big.src, big.dst, big.t, n=big.n) as Gb, \
            tm.build_graph(small.src, small.dst, small.t, n=small.n) as Gs:
        for G, g, delta, name in ((Gb, big, 86400, "first, 1e6 edges"),
                                  (Gs, small, 3600, "second, 4e4 edges")):
            case(f"no-alloc {name}")
            want = G.count(delta)
            before = tm.debug_alloc_calls()
            got = G.count_noalloc(delta)
            assert tm.debug_alloc_calls() == before
            np.testing.assert_array_equal(got, want)
        np.testing.assert_array_equal(Gs.count_noalloc(3600),
                                      oracle.count(small.src, small.dst, small.t, 3600, n=small.n))


def test_noalloc_edge_cases(tm):
    # fewer than three edges: zeros; delta out of range: refused
    g = graphgen.chung_lu_pareto(63, 100, 2)
    with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
        case("no-alloc m=2")
        np.testing.assert_array_equal(G.count_noalloc(10), np.zeros((6, 6), np.uint64))
        with pytest.raises(tm.TMError) as ei:
            G.count_noalloc(-1)
        assert ei.value.code == -1
    # a batch is refused
    graphs = [(g.src, g.dst, g.t, g.n)] * 2
    with tm.build_batch(graphs) as B:
        with pytest.raises(tm.TMError) as ei:
            B.count_noalloc(10)
        assert ei.value.code == -1


def test_noalloc_refuses_too_large_workspace(tm):
    # about 9e6 edges need more workspace than the fixed array holds
    g = graphgen.chung_lu_pareto(64, 400_000, 9_000_000)
    with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
        case("no-alloc too large")
        with pytest.raises(tm.TMError) as ei:
            G.count_noalloc(3600)
        assert ei.value.code == -2
        # and the fixed workspace still serves a graph that fits
    s = graphgen.chung_lu_pareto(65, 2_000, 30_000)
    with tm.build_graph(s.src, s.dst, s.t, n=s.n) as Gs:
        np.testing.assert_array_equal(Gs.count_noalloc(600), Gs.count(600))
