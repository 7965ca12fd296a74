"""Chain compaction (Sec. 7) on the GPU against the oracle, element by element:
every node's chain, rank and orientation, the chain table, the labels and the
kept edges, over special cases, random read sets (linear and circular sources),
both key widths, several min_nodes, and workload-shaped inputs; at the full
2,000,000-read k = 31 size, properties that hold at any size plus sampled
chains checked string by string."""

import random

import numpy as np
import pytest

import oracle
from oracle.compact import graph_compact, key_string, revcomp
from paper_1003_1940_amd import synth
from .gpu_util import gpu_graph, say
from . import test_compact_oracle as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the MI355X")
    oracle.build(force=False)


def _u32(t):
    return t.cpu().numpy().view(np.uint32).astype(np.int64)


def gpu_compact(bases, offsets, k, min_nodes):
    from paper_1003_1940_amd import api
    g, _ = gpu_graph(bases, offsets, k)
    assert g.status == 0
    adj = api.adjacency(g, edge_buckets=True)
    return g, api.compact(g, adj, min_nodes)


def compare_compact(bases, offsets, k, min_nodes, label):
    say(f"[gpu-compact] {label} k={k} min_nodes={min_nodes} reads={len(offsets) - 1}")
    _, c = gpu_compact(bases, offsets, k, min_nodes)
    ref = graph_compact(oracle.build_graph(bases, offsets, k), min_nodes)
    assert c.n_chains == len(ref.labels), f"{label}: chain count"
    assert np.array_equal(_u32(c.node_chain), ref.node_chain), f"{label}: node chains differ"
    assert np.array_equal(_u32(c.node_rank), ref.node_rank), f"{label}: node ranks differ"
    assert np.array_equal(c.node_orient.cpu().numpy(), ref.node_orient), f"{label}: orientations"
    assert np.array_equal(_u32(c.chain_head), ref.chain_head), f"{label}: chain heads differ"
    assert np.array_equal(_u32(c.chain_len), ref.chain_len), f"{label}: chain lengths differ"
    assert np.array_equal(c.chain_cyclic.cpu().numpy(), ref.chain_cyclic), f"{label}: cyclic"
    assert np.array_equal(c.label_offsets.cpu().numpy().view(np.uint64), ref.label_offsets), \
        f"{label}: label offsets differ"
    assert bytes(c.labels.cpu().numpy()).decode() == "".join(ref.labels), f"{label}: labels"
    assert np.array_equal(_u32(c.kept_row), ref.kept_row), f"{label}: kept rows differ"
    assert np.array_equal(_u32(c.kept_u), ref.kept_u), f"{label}: kept u chains differ"
    assert np.array_equal(_u32(c.kept_v), ref.kept_v), f"{label}: kept v chains differ"
    assert np.array_equal(c.kept_orient.cpu().numpy(), ref.kept_orient), f"{label}: kept sides"
    return c, ref


def _rs(reads):
    r = synth.from_strings(reads)
    return r.bases, r.offsets


def test_compact_golden_example():
    gd = T._golden()
    b, o = _rs(gd["read"])
    for mn in (2, 3):
        c, _ = compare_compact(b, o, 3, mn, "Sec. 5.1 example")
        assert [c.label(i) for i in range(c.n_chains)] == gd[f"min{mn}.labels"]


def test_compact_special_cases():
    for i, (reads, k) in enumerate(T.SPECIAL):
        b, o = _rs(reads)
        for mn in (1, 2, 3):
            compare_compact(b, o, k, mn, f"special[{i}]")


def test_compact_closed_forms():
    rnd = random.Random(11)
    for k, length in ((11, 400), (31, 3000), (63, 3000)):
        G = T._distinct_kmer_genome(rnd, length, k)
        rl = 3 * k
        reads = [G[i:i + rl] for i in range(0, length - rl + 1, k)] + [G[-rl:]]
        b, o = _rs(reads)
        c, _ = compare_compact(b, o, k, 3, f"linear genome {length}")
        assert c.n_chains == 1 and c.label(0) in (G, revcomp(G)) and c.n_kept == 0
        Gc = T._distinct_kmer_genome(rnd, length, k, circular=True)
        ext = Gc + Gc[:2 * k]
        reads = [ext[i:i + 2 * k] for i in range(0, length, k // 2 + 1)]
        b, o = _rs(reads)
        c, _ = compare_compact(b, o, k, 3, f"circular genome {length}")
        assert c.n_chains == 1 and c.n_cyclic == 1 and c.n_kept == 1


def test_compact_random_sets():
    rnd = random.Random(1003)
    for t in range(40):
        k = rnd.choice((1, 3, 5, 7, 9, 15, 31, 33, 63))
        reads = T._random_reads(rnd, k)
        b, o = _rs(reads)
        compare_compact(b, o, k, rnd.choice((0, 2, 3, 4)), f"random[{t}]")


@pytest.mark.parametrize("k", [21, 31, 33, 63])
def test_compact_workloads(k):
    rng = np.random.default_rng(900 + k)
    g = synth.random_genome(rng, 20_000)
    rs = synth.sample_reads(rng, g, 3000, 150, 0.01)
    compare_compact(rs.bases, rs.offsets, k, 3, "k-sweep")


def test_compact_repeats_recipe():
    rs = synth.plain_repeats(scale=0.005)
    compare_compact(rs.bases, rs.offsets, 31, 3, "plain_repeats 0.5%")


def test_compact_fullsize_properties():
    """The 2,000,000-read k = 31 workload: chains partition the nodes, ranks and
    lengths agree, merged + kept = edges, and sampled chains spell their nodes
    (string checks on the host)."""
    import torch
    from paper_1003_1940_amd import api
    say("[gpu-compact] full-size plain_repeats_k31")
    rs = synth.plain_repeats()
    g = api.build(rs.bases, rs.offsets, 31)
    assert g.status == 0
    adj = api.adjacency(g, edge_buckets=True)
    c = api.compact(g, adj, 3)
    n, m = g.n_nodes, g.n_edges
    say(f"[gpu-compact] {n} nodes -> {c.n_chains} chains, {c.n_kept} kept edges, "
        f"{c.n_cyclic} cycles")
    clen = c.chain_len.to(torch.int64)
    assert int(clen.sum()) == n
    assert bool(((clen == 1) | (clen >= 3)).all())
    assert m - c.n_kept == int((clen - 1).sum())
    assert c.label_len == c.n_chains * 30 + n
    nc = c.node_chain.to(torch.int64)
    assert bool((torch.bincount(nc, minlength=c.n_chains) == clen).all())
    assert bool((c.node_rank.to(torch.int64) < clen[nc]).all())
    heads = c.chain_head.to(torch.int64)
    assert bool((heads[1:] > heads[:-1]).all())
    assert bool((nc[heads] == torch.arange(c.n_chains, device=nc.device)).all())
    assert bool((c.node_rank[heads] == 0).all())
    # sampled chains: every node's k-mer, as the walk reads it, at its rank
    rng = np.random.default_rng(5)
    long_ids = torch.nonzero(clen >= 3).flatten().cpu().numpy()
    pick = rng.choice(long_ids, min(300, len(long_ids)), replace=False)
    keys = g.node_kmer.cpu().numpy().view(np.uint64)
    ncn = nc.cpu().numpy()
    rank = c.node_rank.cpu().numpy().view(np.uint32)
    ori = c.node_orient.cpu().numpy()
    members = {int(p): [] for p in pick}
    for v in np.nonzero(np.isin(ncn, pick))[0]:
        members[int(ncn[v])].append(v)
    off = c.label_offsets.cpu().numpy().view(np.uint64)
    for ci, vs in members.items():
        s = bytes(c.labels[int(off[ci]):int(off[ci + 1])].cpu().numpy()).decode()
        for v in vs:
            km = key_string(int(keys[v]), 0, 31)
            want = km if ori[v] == 0 else revcomp(km)
            r = int(rank[v])
            assert s[r:r + 31] == want, f"chain {ci} rank {r}"
