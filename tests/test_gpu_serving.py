"""GPU tests of the serving loop: every result equals the same request
counted alone (exact integers, tolerance 0), whatever else is in flight."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

GB = 1 << 30


@pytest.fixture(scope="module")
def tm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2204_09236_amd as p
    return p


def case(msg):
    print(f"[case] {msg}", flush=True)


def _pool(seed, k):
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(k):
        m = int(np.exp(rng.uniform(np.log(300), np.log(60000))))
        g = graphgen.chung_lu_pareto(seed * 1000 + i, max(3, m // 20), m)
        pool.append(g)
    return pool


def test_server_mix_equals_alone(tm):
    pool = _pool(1, 12)
    rng = np.random.default_rng(2)
    reqs = []
    for i in range(150):
        gi = int(rng.integers(0, len(pool)))
        delta = int(np.exp(rng.uniform(np.log(60), np.log(86400))))
        keyed = i % 3 != 0
        reqs.append((gi, delta, keyed))
    case("server mix 150 requests")
    sent = set()
    with tm.Server(64 * GB, max_inflight=8) as S:
        tickets = []
        for gi, delta, keyed in reqs:
            g = pool[gi]
            if keyed:
                if gi in sent:
                    tk = S.submit(delta, key=gi + 1)
                else:
                    tk = S.submit(delta, g.src, g.dst, g.t, n=g.n, key=gi + 1)
                    sent.add(gi)
            else:
                tk = S.submit(delta, g.src, g.dst, g.t, n=g.n)
            tickets.append(tk)
        results = []
        for tk in tickets:
            rc, out, times = S.wait(tk)
            assert rc == 0, (rc, tm.last_error())
            assert times[0] <= times[1] <= times[2]
            results.append(out)
        st = S.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    alone = {}
    for (gi, delta, _), got in zip(reqs, results):
        if (gi, delta) not in alone:
            g = pool[gi]
            with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
                alone[(gi, delta)] = G.count(delta)
        np.testing.assert_array_equal(got, alone[(gi, delta)])
    # and alone == oracle for a few
    for (gi, delta) in list(alone)[:5]:
        g = pool[gi]
        np.testing.assert_array_equal(alone[(gi, delta)], oracle.count(g.src, g.dst, g.t, delta, n=g.n))


def test_server_invalid_request_is_isolated(tm):
    pool = _pool(3, 6)
    bad = pool[2]
    bad_dst = bad.dst.copy()
    bad_dst[5] = bad.src[5]                         # self-loop
    case("server invalid member")
    with tm.Server(64 * GB, max_inflight=1) as S:
        # max_inflight=1 keeps the first request running so the rest are
        # admitted together as one union batch
        first = S.submit(500, pool[0].src, pool[0].dst, pool[0].t, n=pool[0].n)
        tks = []
        for i, g in enumerate(pool[1:]):
            dst = bad_dst if g is bad else g.dst
            tks.append((g, dst, S.submit(3600, g.src, dst, g.t, n=g.n)))
        assert S.wait(first)[0] == 0
        for g, dst, tk in tks:
            rc, out, _ = S.wait(tk)
            if dst is bad_dst:
                assert rc == -1
            else:
                assert rc == 0
                np.testing.assert_array_equal(out, oracle.count(g.src, g.dst, g.t, 3600, n=g.n))


def test_server_budget_and_backpressure(tm):
    g = graphgen.chung_lu_pareto(5, 5000, 100_000)
    case("server budget")
    with tm.Server(1 << 20, max_inflight=4) as S:    # 1 MiB: nothing fits
        rc, _, _ = S.wait(S.submit(100, g.src, g.dst, g.t, n=g.n))
        assert rc == -2                              # TM_ENOMEM
    case("server back-pressure")
    big = graphgen.chung_lu_pareto(6, 50_000, 2_000_000)
    refused = 0
    with tm.Server(64 * GB, max_inflight=1, max_queue=1) as S:
        # one resident graph; edge-less submits take microseconds, each count
        # milliseconds, so a burst overruns the one-slot queue
        assert S.wait(S.submit(86400, big.src, big.dst, big.t, n=big.n, key=9))[0] == 0
        tks = []
        for _ in range(50):
            try:
                tks.append(S.submit(86400, key=9))
            except tm.TMError as e:
                assert e.code == -4                  # TM_EAGAIN
                refused += 1
        for tk in tks:
            assert S.wait(tk)[0] == 0
    assert refused >= 1 and len(tks) >= 1
    with pytest.raises(tm.TMError):
        tm.Server(0)


def test_server_resident_graph_reuse(tm):
    g = graphgen.chung_lu_pareto(7, 3000, 80_000)
    case("server residency")
    with tm.Server(64 * GB) as S:
        rc, first, _ = S.wait(S.submit(3600, g.src, g.dst, g.t, n=g.n, key=42))
        assert rc == 0
        outs = [S.wait(S.submit(d, key=42)) for d in (3600, 600, 86400)]
        assert all(o[0] == 0 for o in outs)
        assert S.stats()["resident_graphs"] == 1
        with pytest.raises(tm.TMError) as ei:
            S.submit(10, key=999)                    # unknown key, no edges
        assert ei.value.code == -5
    np.testing.assert_array_equal(outs[0][1], first)
    for (rc, out, _), d in zip(outs, (3600, 600, 86400)):
        np.testing.assert_array_equal(out, oracle.count(g.src, g.dst, g.t, d, n=g.n))


def test_server_key_known_while_building(tm):
    """Edge-less requests for a key whose graph is still being built (taken
    from the queue, not yet resident) wait for it instead of failing."""
    g = graphgen.chung_lu_pareto(77, 50_000, 1_000_000)
    deltas = [60, 600, 3600, 86400]
    case("server key known while building, m=1e6")
    with tm.Server(64 * GB, max_inflight=4) as S:
        first = S.submit(3600, g.src, g.dst, g.t, n=g.n, key=5)
        rest = [S.submit(d, key=5) for d in deltas * 5]
        got = [S.wait(first)] + [S.wait(tk) for tk in rest]
    assert all(rc == 0 for rc, _, _ in got)
    with tm.build_graph(g.src, g.dst, g.t, n=g.n) as G:
        want = {d: G.count(d) for d in deltas}
    assert np.array_equal(got[0][1], want[3600])
    for (rc, out, _), d in zip(got[1:], deltas * 5):
        assert np.array_equal(out, want[d])
