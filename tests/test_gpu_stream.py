"""GPU tests of incremental counting (tm_stream_*): per append, the
instances whose last edge is new equal the oracle's count of the prefix up
to that batch minus its count of the prefix before it (exact integers); the
running totals equal the oracle's count of everything appended."""
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


def time_ordered(g):
    """The edge list sorted by time (stable): a stream that never goes back."""
    o = np.argsort(g.t, kind="stable")
    return g.src[o], g.dst[o], g.t[o]


def run_stream(tm, src, dst, t, cuts, delta, n):
    """Append the batches [cuts[i], cuts[i+1]) and check each against the
    oracle's prefix difference, then the totals against the whole list."""
    prev = np.zeros(56, dtype=np.uint64)
    with tm.Stream(delta, n=n) as S:
        for a, b in zip(cuts[:-1], cuts[1:]):
            got = S.append(src[a:b], dst[a:b], t[a:b])
            cur = oracle.alg(src[:b], dst[:b], t[:b], delta, n=n)
            want = oracle.merge(cur - prev) if b > a else np.zeros((6, 6), np.uint64)
            np.testing.assert_array_equal(got, want, err_msg=f"batch [{a}, {b}) delta={delta}")
            prev = cur
        total, edges, kept = S.totals()
    np.testing.assert_array_equal(total, oracle.merge(oracle.alg(src, dst, t, delta, n=n)))
    assert edges == len(src) and kept <= len(src)
    return kept


@pytest.mark.parametrize("delta", [0, 40, 300, 5000])
def test_stream_batches_match_prefix_differences(tm, delta):
    rng = np.random.default_rng(61)
    g = graphgen.small_random(rng, 25, 3000, t_values=600, tmax=6000, multi=0.3)
    src, dst, t = time_ordered(g)
    cuts = np.unique(np.concatenate(([0, len(src)], rng.integers(0, len(src), 12)))).tolist()
    case(f"stream small delta={delta} batches={len(cuts) - 1}")
    run_stream(tm, src, dst, t, cuts, delta, n=25)


def test_stream_ties_across_batches(tm):
    """Batches that share timestamps at their boundary (t equal across the
    cut), one-edge batches and an empty batch."""
    rng = np.random.default_rng(62)
    g = graphgen.small_random(rng, 12, 800, t_values=40, tmax=400, multi=0.5)
    src, dst, t = time_ordered(g)
    cuts = [0, 1, 2, 2, 50, 51, 300, 301, 302, 800]
    case("stream ties and tiny batches")
    run_stream(tm, src, dst, t, cuts, 30, n=12)


def test_stream_drops_old_edges(tm):
    """A long stream with a short delta keeps only the recent tail, and the
    counts stay exact."""
    g = graphgen.chung_lu_pareto(63, 2000, 60_000, span=2_000_000)
    src, dst, t = time_ordered(g)
    cuts = list(range(0, len(src), 6000)) + [len(src)]
    case("stream tail trimming, m=60000")
    kept = run_stream(tm, src, dst, t, cuts, 3600, n=g.n)
    assert kept < len(src) // 2


def test_stream_device_batches(tm):
    import torch
    g = graphgen.chung_lu_pareto(64, 3000, 80_000)
    src, dst, t = time_ordered(g)
    dev = torch.device("cuda:0")
    cuts = [0, 10_000, 30_000, 55_000, 80_000]
    case("stream device-pointer batches")
    with tm.Stream(86400, n=g.n) as S:
        for a, b in zip(cuts[:-1], cuts[1:]):
            S.append(*(torch.from_numpy(x[a:b]).to(dev) for x in (src, dst, t)))
        total, edges, _ = S.totals()
    assert edges == len(src)
    np.testing.assert_array_equal(total, oracle.merge(oracle.alg(src, dst, t, 86400, n=g.n)))


def test_stream_rejects_and_stays_unchanged(tm):
    rng = np.random.default_rng(65)
    g = graphgen.small_random(rng, 10, 400, tmax=1000)
    src, dst, t = time_ordered(g)
    case("stream rejections")
    with tm.Stream(100, n=10) as S:
        S.append(src[:200], dst[:200], t[:200])
        # going back in time
        with pytest.raises(tm.TMError) as ei:
            S.append(src[200:], dst[200:], t[200:] - 500)
        assert ei.value.code == -1
        # a self-loop in the batch
        bad = dst[200:].copy()
        bad[3] = src[203]
        with pytest.raises(tm.TMError):
            S.append(src[200:], bad, t[200:])
        # an id beyond n
        big = dst[200:].copy()
        big[0] = 10
        with pytest.raises(tm.TMError):
            S.append(src[200:], big, t[200:])
        S.append(src[200:], dst[200:], t[200:])
        total, edges, _ = S.totals()
    assert edges == len(src)
    np.testing.assert_array_equal(total, oracle.merge(oracle.alg(src, dst, t, 100, n=10)))
    with pytest.raises(tm.TMError):
        tm.Stream(-1)
