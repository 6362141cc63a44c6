"""GPU parity at the full sizes of the batched and serving workloads.

Expected counts come from tests/golden/make_golden.py, which runs only the
CPU oracle (the paper's Algorithms 1 and 2) on the regenerated inputs; each
record carries the sha256 of its input arrays, and a member whose
regenerated input differs is reported, not silently compared.
"""
import json
import multiprocessing as mp
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
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


def _gen(item):
    g = graphgen.batch_graph(item)
    return g.src, g.dst, g.t, g.n, graphgen.edge_hash(g)


def _procs():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.mark.timeout(900)
def test_batch_sample_full_size(tm):
    """256 graphs of the 4,096-graph batch (the 20 largest, up to 2e6 edges,
    the 10 widest windows, up to delta 86,275, the 10 smallest, the rest
    drawn uniformly; 9.7e7 edges in all), built as one union graph from
    device pointers and counted with per-graph delta through the captured
    hipGraph, against the oracle's per-graph counts; then once more eagerly
    with every triangle candidate through the hub slices."""
    import torch
    rec = json.load(open(os.path.join(GOLDEN, "batch_counts.json")))
    spec = graphgen.batch_spec()
    mem = rec["members"]
    items = [spec[r["index"]] for r in mem]
    case(f"batch sample: generating {len(items)} graphs")
    with mp.get_context("fork").Pool(_procs()) as pool:
        graphs = pool.map(_gen, items, chunksize=4)
    for r, g in zip(mem, graphs):
        assert g[4] == r["edge_sha256"], f"graph {r['index']}: regenerated input differs"
    deltas = np.array([r["delta"] for r in mem], np.int64)
    off = np.zeros(len(graphs) + 1, np.uint64)
    off[1:] = np.cumsum([g[0].size for g in graphs])
    ncount = np.array([g[3] for g in graphs], np.uint32)
    dev = torch.device("cuda:0")
    src, dst, t = (torch.from_numpy(np.concatenate([g[k] for g in graphs])).to(dev) for k in range(3))
    del graphs
    case(f"batch sample: build {len(mem)} graphs, {int(off[-1])} edges")
    with tm.build_batch_arrays(src, dst, t, off, ncount) as B:
        case("batch sample: captured count")
        got = B.count_batch_raw(deltas)
        case("batch sample: eager count, hub_min=1")
        got_hub = B.count_batch_raw_ex(deltas, use_graph=False, hub_min=1)
    for i, r in enumerate(mem):
        want = np.array(r["raw"], dtype=np.uint64)
        np.testing.assert_array_equal(got[i], want, err_msg=f"graph {r['index']} delta={r['delta']}")
        np.testing.assert_array_equal(got_hub[i], want, err_msg=f"graph {r['index']} hub_min=1")
    del src, dst, t
    torch.cuda.empty_cache()


def _small_requests(seed, k):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        m = int(np.exp(rng.uniform(np.log(1e3), np.log(2e5))))
        g = graphgen.chung_lu_pareto(seed * 1000 + i, max(3, m // 20), m)
        out.append((g, int(np.exp(rng.uniform(np.log(60), np.log(86400))))))
    return out


@pytest.mark.timeout(900)
def test_server_full_size_requests(tm):
    """The server with the largest request size of the serving workload: a
    keyed 5e7-edge graph (graphgen.serve_max) at delta 60, 3,600 and 86,400,
    and the keyed 2e7-edge power-law graph, mixed with small anonymous
    requests that arrive while the large graphs build and count.  Every
    large result equals the oracle's stored counts, every small one the
    oracle run here."""
    rec_s = json.load(open(os.path.join(GOLDEN, "serve_counts.json")))
    rec_p = json.load(open(os.path.join(GOLDEN, "powerlaw_counts.json")))
    case("server full size: generating the 5e7-edge and 2e7-edge graphs")
    big = graphgen.serve_max()
    assert graphgen.edge_hash(big) == rec_s["edge_sha256"]
    pl = graphgen.powerlaw()
    assert graphgen.edge_hash(pl) == rec_p["edge_sha256"]
    small = _small_requests(7, 24)
    s_deltas = [int(k) for k in rec_s["counts"]]
    with tm.Server(200 * GB, max_inflight=8) as S:
        tickets = []
        case("server full size: submit")
        tickets.append(("big", s_deltas[0], S.submit(s_deltas[0], big.src, big.dst, big.t, n=big.n,
                                                     key=101)))
        for j, (g, d) in enumerate(small[:8]):
            tickets.append(("small", j, S.submit(d, g.src, g.dst, g.t, n=g.n)))
        tickets.append(("pl", 3600, S.submit(3600, pl.src, pl.dst, pl.t, n=pl.n, key=102)))
        for d in s_deltas[1:]:
            tickets.append(("big", d, S.submit(d, key=101)))
        for j, (g, d) in enumerate(small[8:], start=8):
            tickets.append(("small", j, S.submit(d, g.src, g.dst, g.t, n=g.n)))
        tickets.append(("big", s_deltas[-1], S.submit(s_deltas[-1], key=101)))
        results = []
        for kind, arg, tk in tickets:
            rc, out, times = S.wait(tk)
            assert rc == 0, (kind, arg, rc)
            results.append((kind, arg, out))
        st = S.stats()
    assert st["failed"] == 0
    for kind, arg, got in results:
        case(f"server full size: check {kind} {arg}")
        if kind == "big":
            want = np.array(rec_s["counts"][str(arg)]["grid"], dtype=np.uint64)
        elif kind == "pl":
            want = np.array(rec_p["counts"][str(arg)]["grid"], dtype=np.uint64)
        else:
            g, d = small[arg]
            want = oracle.count(g.src, g.dst, g.t, d, n=g.n)
        np.testing.assert_array_equal(got, want, err_msg=f"{kind} {arg}")
