"""Full-size checks at the benchmark configuration: the 2,000,000-read k = 31
workload, built exactly as bench.py builds it.  The oracle cannot hold the whole
graph, so (1) every output row is checked against the invariants that hold at
any size, and (2) sampled rows, and sampled keys that must be absent, are counted
by the oracle's probe scan over all reads."""

import numpy as np
import pytest

import oracle
from paper_1003_1940_amd import synth
from . import keys_np as K
from .gpu_util import gpu_graph, say
from .invariants import check_graph

pytestmark = pytest.mark.gpu


class _G:
    def __init__(self, d):
        self.__dict__.update(d)


@pytest.fixture(scope="module")
def repeats_full():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the MI355X")
    oracle.build(force=False)
    say("[gpu-fullsize] generating the 2,000,000-read k=31 workload")
    rs = synth.plain_repeats()
    say("[gpu-fullsize] building on the GPU")
    g, got = gpu_graph(rs.bases, rs.offsets, 31)
    assert g.status == 0
    yield rs, g, got
    del g
    import gc
    gc.collect()
    torch.cuda.empty_cache()  # later tests size their budgets from free HBM


def test_fullsize_invariants(repeats_full):
    rs, g, got = repeats_full
    say(f"[gpu-fullsize] invariants over {g.n_nodes} nodes, {g.n_edges} edges")
    check_graph(_G(got), 31, rs.bases, rs.offsets)


def test_fullsize_sampled_counts(repeats_full):
    rs, g, got = repeats_full
    rng = np.random.default_rng(2024)
    k = 31
    ni = np.sort(rng.choice(len(got["node_count"]), size=400, replace=False))
    ei = np.sort(rng.choice(len(got["edge_mult"]), size=400, replace=False))
    node_probes = [K.to_str(got["node_key"][i, 0], got["node_key"][i, 1], k) for i in ni]
    # keys absent from the table: random canonical k-mers that are not nodes
    absent = []
    nodes = got["node_key"][:, 0]
    while len(absent) < 40:
        lo = rng.integers(0, 1 << 62, dtype=np.uint64)
        clo, chi, _ = K.canonical(np.array([lo], np.uint64), np.array([0], np.uint64), k)
        i = np.searchsorted(nodes, clo[0])
        if i >= len(nodes) or nodes[i] != clo[0]:
            absent.append(K.to_str(clo[0], 0, k))
    edge_probes = [(K.to_str(got["edge_u"][i, 0], 0, k), K.to_str(got["edge_v"][i, 0], 0, k),
                    int(got["edge_orient"][i])) for i in ei]
    say("[gpu-fullsize] oracle probe scan over all reads")
    nc, ec = oracle.probe_counts(rs.bases, rs.offsets, k, node_probes + absent, edge_probes)
    assert np.array_equal(nc[:len(ni)], got["node_count"][ni]), "sampled node counts differ"
    assert (nc[len(ni):] == 0).all(), "a key absent from the node table occurs in the reads"
    assert np.array_equal(ec, got["edge_mult"][ei]), "sampled edge multiplicities differ"


def test_fullsize_adjacency(repeats_full):
    """STEP-4 lists of the full graph: totals, every edge end exactly once, and
    sampled entries sit in the bucket of their endpoint and side."""
    import torch
    from paper_1003_1940_amd import api
    rs, g, got = repeats_full
    say("[gpu-fullsize] adjacency lists")
    a = api.adjacency(g)
    n, m = g.n_nodes, g.n_edges
    off = a.offsets
    assert off.numel() == 2 * n + 1 and int(off[0]) == 0 and int(off[-1]) == 2 * m
    assert bool((off[1:] >= off[:-1]).all())
    ends = a.inc_edge.to(torch.int64) * 2 + a.inc_end.to(torch.int64)
    assert bool((torch.bincount(ends, minlength=2 * m) == 1).all())
    rng = np.random.default_rng(7)
    pos = torch.from_numpy(rng.choice(2 * m, 4000, replace=False)).cuda()
    bucket = torch.searchsorted(off, pos, right=True) - 1
    node, side = bucket // 2, bucket % 2
    e = a.inc_edge[pos].to(torch.int64)
    end = a.inc_end[pos].to(torch.int64)
    key = torch.where(end == 0, g.edge_u[e], g.edge_v[e])
    assert bool((key == g.node_kmer[node]).all()), "an entry is not at its endpoint's node"
    o = g.edge_orient[e].to(torch.int64)
    # the u end lies on side o1, the v end on side 1 - o2
    assert bool((torch.where(end == 0, o >> 1, 1 - (o & 1)) == side).all()), "wrong side"
