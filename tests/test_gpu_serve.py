"""The served build: requests of different sizes and k overlap on the device, and
each request's tables are the same in the mix as built alone (bit for bit), and
the same as the oracle's."""

import numpy as np
import pytest

import oracle
from paper_1003_1940_amd import synth
from .gpu_util import FIELDS, gpu_graph, say

pytestmark = pytest.mark.gpu


def _requests(n, rate, pool_size, scale):
    from paper_1003_1940_amd.serve import Request, pin_read_set
    arrivals, which, ks, pool = synth.served_trace(n, rate=rate, pool_size=pool_size,
                                                   scale=scale)
    pinned = [pin_read_set(p.bases, p.offsets) for p in pool]
    reqs = [Request(i, pinned[w][0], pinned[w][1], int(k), float(a))
            for i, (a, w, k) in enumerate(zip(arrivals, which, ks))]
    return reqs, pool, which


def _tables(g):
    return g.to_numpy()


def _assert_same(a, b, label):
    for f in FIELDS:
        if a[f] is None or b[f] is None:
            continue
        assert np.array_equal(a[f], b[f]), f"{label}: column {f} differs"


@pytest.fixture(scope="module")
def served():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the MI355X")
    from paper_1003_1940_amd.serve import Server
    reqs, pool, which = _requests(40, rate=4000.0, pool_size=10, scale=0.02)
    say(f"[gpu-serve] {len(reqs)} requests, pool of {len(pool)} sets, "
        f"{sum(p.n_bases for p in pool)} bases")
    srv = Server(slots=6, keep_results=True, zkey=True)
    stats = srv.run(reqs)
    say(f"[gpu-serve] served: peak in flight {stats['peak_inflight']}")
    return reqs, pool, which, stats


def test_served_equals_alone(served):
    reqs, pool, which, stats = served
    assert stats["peak_inflight"] >= 2, "requests never overlapped on the device"
    alone = {}
    for r, w in zip(reqs, which):
        assert r.status == 0, f"request {r.rid}: status {r.status}"
        key = (int(w), r.k)
        if key not in alone:
            g, t = gpu_graph(pool[w].bases, pool[w].offsets, r.k)
            assert g.status == 0
            alone[key] = t
        _assert_same(_tables(r.graph), alone[key], f"request {r.rid} (set {w}, k={r.k})")


def test_served_equals_oracle(served):
    reqs, pool, which, _ = served
    seen = set()
    for r, w in zip(reqs, which):
        key = (int(w), r.k)
        if key in seen or len(seen) >= 6:
            continue
        seen.add(key)
        ref = oracle.build_graph(pool[w].bases, pool[w].offsets, r.k)
        got = _tables(r.graph)
        assert r.graph.n_nodes == len(ref.node_count) and r.graph.n_edges == len(ref.edge_mult)
        for f in FIELDS:
            assert np.array_equal(got[f], getattr(ref, f)), f"request {r.rid}: {f} vs oracle"


def test_fifo_and_tight_budget_agree(served):
    """One build at a time (first in, first out), and a memory budget that admits
    only the largest request alone, give the same tables."""
    from paper_1003_1940_amd.serve import Request, Server
    reqs, pool, which, _ = served
    fresh = [Request(r.rid, r.bases, r.offsets, r.k, r.arrival_s) for r in reqs[:16]]
    fifo = Server(slots=1, keep_results=True, zkey=True)
    st = fifo.run(fresh)
    assert st["peak_inflight"] == 1
    for a, b in zip(fresh, reqs[:16]):
        assert a.status == 0
        _assert_same(_tables(a.graph), _tables(b.graph), f"fifo request {a.rid}")
    tight = [Request(r.rid, r.bases, r.offsets, r.k, r.arrival_s) for r in reqs[:16]]
    from paper_1003_1940_amd.serve import request_bytes
    need = max(request_bytes(int(r.bases.numel()), int(r.offsets.numel()) - 1,
                             pool[w].kmer_count(r.k), r.k, True)
               for r, w in zip(tight, which[:16]))
    srv = Server(slots=6, hbm_budget=need, keep_results=True, zkey=True)
    srv.run(tight)
    for a, b in zip(tight, reqs[:16]):
        assert a.status == 0
        _assert_same(_tables(a.graph), _tables(b.graph), f"tight-budget request {a.rid}")


def test_request_over_budget_is_refused(served):
    from paper_1003_1940_amd.serve import Request, Server
    reqs, _, _, _ = served
    r = reqs[0]
    srv = Server(slots=2, hbm_budget=1024)
    with pytest.raises(ValueError):
        srv.run([Request(0, r.bases, r.offsets, r.k, 0.0)])
