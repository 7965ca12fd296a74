"""The out-of-memory build by key-space slices on the GPU: prefix counts against
counts computed here from the read strings, and sliced builds (many slices,
uneven slices, a budget of exactly the largest prefix) equal, row for row, to
the one-shot build and to the oracle, for both key widths; a slice over its key
budget is reported on the device."""

import random

import numpy as np
import pytest

import oracle
from paper_1003_1940_amd import sliced, synth
from . import keys_np as K
from .gpu_util import gpu_graph, say

pytestmark = pytest.mark.gpu

COLS = ("node_key", "node_count", "edge_u", "edge_v", "edge_orient", "edge_mult")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the MI355X")
    oracle.build(force=False)


def prefix_ref(bases, offsets, length):
    """Counts of the top 12 bits of the canonical keys of every window."""
    off = np.asarray(offsets, np.uint64)
    n = int(off[-1])
    if n == 0:
        return np.zeros(sliced.PREFIX_BINS, np.uint64)
    codes = K.codes(np.asarray(bases[:n], np.uint8))
    starts, _ = K.window_starts(off, length)
    if len(starts) == 0:
        return np.zeros(sliced.PREFIX_BINS, np.uint64)
    lo, hi = K.window_keys(codes, starts, length)
    clo, chi, _ = K.canonical(lo, hi, length)
    bits = 2 * length
    p = []
    for a, b in zip(clo.tolist(), chi.tolist()):
        v = (b << 64) | a
        p.append(v >> (bits - 12) if bits >= 12 else v << (12 - bits))
    return np.bincount(np.array(p, np.int64), minlength=sliced.PREFIX_BINS).astype(np.uint64)


def _rs(reads):
    r = synth.from_strings(reads)
    return r.bases, r.offsets


def test_prefix_counts_match_the_strings():
    from paper_1003_1940_amd import api
    rnd = random.Random(61)
    cases = [(["AATGCATC"], 3), (["ACGTACGT", "TTTT", "G"], 1), (["AC" * 30], 5)]
    for _ in range(8):
        k = rnd.choice((3, 5, 11, 31, 33, 63))
        cases.append((["".join(rnd.choice("ACGT") for _ in range(rnd.randint(0, 3 * k + 40)))
                       for _ in range(rnd.randint(1, 30))], k))
    for reads, k in cases:
        b, o = _rs(reads)
        say(f"[gpu-sliced] prefix counts k={k} reads={len(reads)}")
        packed, offs, n_bases = api.upload(b, o)
        ec, nc = sliced.prefix_counts(packed, n_bases, offs, k,
                                      max(sliced.positions(o, k), 1))
        assert np.array_equal(ec, prefix_ref(b, o, k + 1)), f"edge prefixes k={k}"
        assert np.array_equal(nc, prefix_ref(b, o, k)), f"node prefixes k={k}"
    # long reads: keys shorter than the 12-bit prefix and than a 4-base digit
    rng = np.random.default_rng(64)
    g = synth.random_genome(rng, 5000)
    rs = synth.sample_reads(rng, g, 400, 150, 0.01)
    for k in (1, 3, 5, 7):
        say(f"[gpu-sliced] prefix counts k={k} long reads")
        packed, offs, n_bases = api.upload(rs.bases, rs.offsets)
        ec, nc = sliced.prefix_counts(packed, n_bases, offs, k, sliced.positions(rs.offsets, k))
        assert np.array_equal(ec, prefix_ref(rs.bases, rs.offsets, k + 1)), f"edges k={k}"
        assert np.array_equal(nc, prefix_ref(rs.bases, rs.offsets, k)), f"nodes k={k}"
    rs = synth.plain_small(scale=0.2)
    packed, offs, n_bases = api.upload(rs.bases, rs.offsets)
    ec, nc = sliced.prefix_counts(packed, n_bases, offs, 31,
                                  sliced.positions(rs.offsets, 31))
    assert np.array_equal(nc, prefix_ref(rs.bases, rs.offsets, 31))
    assert int(ec.sum()) == sliced.positions(rs.offsets, 32)


def compare_sliced(bases, offsets, k, label, n_slices=None, budget=None, with_oracle=True):
    say(f"[gpu-sliced] {label} k={k} slices={n_slices} budget={budget}")
    s = sliced.build_sliced(bases, offsets, k, budget=budget, n_slices=n_slices)
    _, one = gpu_graph(bases, offsets, k)
    for c in COLS:
        assert np.array_equal(s.tables[c], one[c]), f"{label}: {c} differs from the one-shot build"
    if with_oracle:
        ref = oracle.build_graph(bases, offsets, k)
        assert np.array_equal(s.tables["node_key"], ref.node_key), f"{label}: oracle nodes"
        assert np.array_equal(s.tables["edge_mult"], ref.edge_mult), f"{label}: oracle mult"
    return s


def test_sliced_random_sets():
    rnd = random.Random(62)
    for t in range(16):
        k = rnd.choice((1, 3, 5, 9, 31, 33, 63))
        reads = ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(0, 3 * k + 60)))
                 for _ in range(rnd.randint(1, 40))]
        b, o = _rs(reads)
        s = compare_sliced(b, o, k, f"random[{t}]", n_slices=rnd.choice((1, 2, 5, 40)))
        assert len(s.slices) >= 1


def test_sliced_budget_of_the_largest_prefix():
    """The smallest workable budget: many slices, each at most one prefix wide
    where the keys crowd."""
    from paper_1003_1940_amd import api
    rng = np.random.default_rng(63)
    g = synth.random_genome(rng, 4000)
    rs = synth.sample_reads(rng, g, 600, 100, 0.01)
    for k in (15, 31, 33):
        packed, offs, n_bases = api.upload(rs.bases, rs.offsets)
        ec, nc = sliced.prefix_counts(packed, n_bases, offs, k, sliced.positions(rs.offsets, k))
        budget = int(max(ec.max(), nc.max()))
        s = compare_sliced(rs.bases, rs.offsets, k, "largest prefix", budget=budget)
        assert len(s.slices) > 20
        assert max(max(r) for r in s.rows) <= budget


@pytest.mark.parametrize("k,n_slices", [(31, 8), (63, 5)])
def test_sliced_workloads(k, n_slices):
    rs = synth.plain_small(scale=0.5) if k == 31 else synth.plain_large(scale=0.001)
    s = compare_sliced(rs.bases, rs.offsets, k, "workload", n_slices=n_slices,
                       with_oracle=False)
    assert len(s.slices) >= n_slices


def test_slice_over_budget_is_reported():
    """A slice whose keys exceed max_keys stops with DBG_E_OVERFLOW on the device
    (its key buffers are never written past their end)."""
    import torch
    from paper_1003_1940_amd import api
    rs = synth.plain_small(scale=0.05)
    k = 31
    packed, offs, n_bases = api.upload(rs.bases, rs.offsets)
    n_pos = sliced.positions(rs.offsets, k)
    max_keys = n_pos // 4
    nbytes = int(api.load().dbg_slice_workspace_bytes(offs.numel() - 1, n_pos, max_keys, k))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = api.alloc_outputs(k, max_keys, max_keys, "cuda", False)
    res = torch.zeros(3, dtype=torch.int64, device="cuda")
    sliced.build_slice_async(packed, n_bases, offs, k, n_pos, max_keys, 0, sliced.PREFIX_BINS,
                             out, max_keys, max_keys, res, ws)
    _, _, status = api.read_result(res)
    assert status == 4, f"status {status}"
    # the same workspace then builds a slice that fits
    ec, nc = sliced.prefix_counts(packed, n_bases, offs, k, n_pos)
    plan = sliced.plan_slices(ec, nc, max_keys)
    lo, hi = plan[0]
    sliced.build_slice_async(packed, n_bases, offs, k, n_pos, max_keys, lo, hi, out, max_keys,
                             max_keys, res, ws)
    n_nodes, n_edges, status = api.read_result(res)
    assert status == 0 and n_nodes > 0 and n_edges > 0
