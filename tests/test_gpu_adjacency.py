"""STEP-4 adjacency lists on the GPU against the oracle's, element by element:
offsets, edge rows and ends, over special cases, random read sets, both key
widths and the workload recipes; and an endpoint missing from the node table is
reported on the device."""

import random

import numpy as np
import pytest

import oracle
from oracle.adjacency import graph_adjacency
from paper_1003_1940_amd import synth
from .gpu_util import gpu_graph, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the MI355X")
    oracle.build(force=False)


def compare_adjacency(bases, offsets, k, label):
    from paper_1003_1940_amd import api
    say(f"[gpu-adjacency] {label} k={k} reads={len(offsets) - 1}")
    g, _ = gpu_graph(bases, offsets, k)
    assert g.status == 0
    a = api.adjacency(g, edge_buckets=True)
    off, ie, ien = a.to_numpy()
    ref = oracle.build_graph(bases, offsets, k)
    roff, rie, rien = graph_adjacency(ref)
    assert np.array_equal(off, roff), f"{label}: offsets differ"
    assert np.array_equal(ie, rie), f"{label}: edge rows differ"
    assert np.array_equal(ien, rien), f"{label}: ends differ"
    # buckets of both ends of every edge: 2 * node row + side (u end on side o1,
    # v end on side 1 - o2)
    row = {(int(x), int(y)): i for i, (x, y) in enumerate(ref.node_key)}
    o = ref.edge_orient.astype(np.int64)
    want = np.array([[2 * row[(int(a0), int(a1))] + (oo >> 1),
                      2 * row[(int(b0), int(b1))] + 1 - (oo & 1)]
                     for (a0, a1), (b0, b1), oo in zip(ref.edge_u, ref.edge_v, o)],
                    np.uint32).reshape(-1)
    got = a.edge_bucket.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want), f"{label}: edge end buckets differ"


def _rs(reads):
    r = synth.from_strings(reads)
    return r.bases, r.offsets


SPECIAL = [(["AATGCATC"], 3), (["AAAA"], 3), (["ACAC", "TGTG"], 3), (["ACGT"], 3),
           (["AC", "ACG", "ACGTA", ""], 3), (["ATGG", "CCAT", "GGAC", "GGTC", "TGGA", "TGGT"], 3),
           (["ACGTACGT"], 1), (["AC" * 40], 1), (["GGGGG", "CCCCCC"], 3), (["ACG"], 5)]


def test_adjacency_special_cases():
    for i, (reads, k) in enumerate(SPECIAL):
        b, o = _rs(reads)
        compare_adjacency(b, o, k, f"special[{i}]")


def test_adjacency_random_sets():
    rnd = random.Random(8)
    for t in range(30):
        k = rnd.choice((1, 3, 5, 9, 15, 31, 33, 63))
        alpha = rnd.choice(("AC", "ACGT", "ACGT", "GT"))
        reads = ["".join(rnd.choice(alpha) for _ in range(rnd.randint(0, 3 * k + 40)))
                 for _ in range(rnd.randint(1, 40))]
        b, o = _rs(reads)
        compare_adjacency(b, o, k, f"random[{t}]")


@pytest.mark.parametrize("k", [21, 31, 33, 63])
def test_adjacency_workloads(k):
    rng = np.random.default_rng(500 + k)
    g = synth.random_genome(rng, 20_000)
    rs = synth.sample_reads(rng, g, 3000, 150, 0.01)
    compare_adjacency(rs.bases, rs.offsets, k, "k-sweep")


def test_adjacency_recipes():
    rs = synth.plain_small()
    compare_adjacency(rs.bases, rs.offsets, 31, "plain_small (10k reads)")
    rs = synth.plain_repeats(scale=0.005)
    compare_adjacency(rs.bases, rs.offsets, 31, "plain_repeats 0.5%")
    rs = synth.plain_large(scale=2.5e-4)
    compare_adjacency(rs.bases, rs.offsets, 63, "plain_large 0.025%")
    b, o = _rs(["A" * 100] * 50 + ["ACGT" * 30] * 40)
    compare_adjacency(b, o, 31, "homopolymers and palindromic repeats")


def test_adjacency_missing_endpoint_is_reported():
    import torch
    from paper_1003_1940_amd import api
    rs = synth.plain_small(scale=0.01)
    g, _ = gpu_graph(rs.bases, rs.offsets, 31)
    say("[gpu-adjacency] an edge endpoint removed from the node table")
    # drop the node that the first edge's u names: shift the later keys down
    nk = g.node_kmer[:g.n_nodes].clone()
    i = int(torch.nonzero(nk == g.edge_u[0])[0, 0])
    g.node_kmer[i:g.n_nodes - 1] = nk[i + 1:]
    g.n_nodes -= 1
    a = api.adjacency_async(g)
    assert api.read_result(a.result)[2] == 9  # DBG_E_ARG
