"""Pins of the STEP-4 adjacency oracle (CPU): the hand-derived lists of the Sec. 5.1
example read, structural invariants, a degree identity that ties the lists to the
node counts and the reads, and planted mistakes that each pin must catch."""

import inspect
import os
import random

import numpy as np
import pytest

import oracle
from oracle import adjacency as adj_mod
from paper_1003_1940_amd import synth
from . import keys_np as K

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "step4_adjacency_sides.txt")


def _golden():
    d = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        d[key] = vals
    return d


def _graph(reads, k):
    rs = synth.from_strings(reads)
    return rs, oracle.build_graph(rs.bases, rs.offsets, k)


def _node_index(g):
    return {(int(a), int(b)): i for i, (a, b) in enumerate(g.node_key)}


def _check_walk_sides(g, rs, offsets, inc_edge, inc_end):
    k = g.k
    if not rs.n_bases:
        return
    idx = _node_index(g)
    codes = K.codes(rs.bases[:rs.n_bases])
    off = rs.offsets.astype(np.int64)
    starts = np.concatenate([np.arange(off[i], off[i + 1] - k) for i in range(len(off) - 1)
                             if off[i + 1] - off[i] >= k + 1] or [np.zeros(0, np.int64)])
    if not len(starts):
        return
    xl, xh = K.window_keys(codes, starts, k)
    yl, yh = K.window_keys(codes, starts + 1, k)
    xcl, xch, xflip = K.canonical(xl, xh, k)
    ycl, ych, yflip = K.canonical(yl, yh, k)
    off = offsets.astype(np.int64)

    def bucket_ends(node, side):
        b = 2 * node + side
        return {(int(inc_edge[t]), int(inc_end[t])) for t in range(off[b], off[b + 1])}

    for t in range(len(starts)):
        a = idx[(int(xcl[t]), int(xch[t]))]
        b = idx[(int(ycl[t]), int(ych[t]))]
        out_side = 1 if xflip[t] else 0
        in_side = 0 if yflip[t] else 1
        ea = bucket_ends(a, out_side)
        eb = bucket_ends(b, in_side)
        # one edge row with one end in each bucket (two different ends of the row)
        ok = any((r, 1 - e) in eb for r, e in ea)
        assert ok, f"no edge joins node {a} side {out_side} to node {b} side {in_side}"


def check_adjacency(g, rs, offsets, inc_edge, inc_end):
    """Invariants of the (node, side) CSR of graph g built from reads rs."""
    n, m = len(g.node_count), len(g.edge_mult)
    k = g.k
    assert len(offsets) == 2 * n + 1 and offsets[0] == 0 and offsets[-1] == 2 * m
    assert (np.diff(offsets.astype(np.int64)) >= 0).all()
    assert len(inc_edge) == 2 * m and len(inc_end) == 2 * m
    # every edge row once per end
    seen = np.zeros((m, 2), np.int64)
    np.add.at(seen, (inc_edge.astype(np.int64), inc_end.astype(np.int64)), 1)
    assert (seen == 1).all()
    # entry (node i, side s): its end is at node i with orientation s
    bucket = np.repeat(np.arange(2 * n), np.diff(offsets.astype(np.int64)))
    node, side = bucket >> 1, bucket & 1
    j = inc_edge.astype(np.int64)
    ends = np.where(inc_end[:, None] == 0, g.edge_u[j], g.edge_v[j])
    assert (ends == g.node_key[node]).all()
    # sides from the reads themselves: for every (k+1)-mer window x.c of a read,
    # with y its last k bases, some edge has an end on the side of x's node that a
    # walk reading x in the read's direction leaves by (0 when x is canonical, 1
    # otherwise) and its other end on the side of y's node that the walk enters
    # by (1 when y is canonical, 0 otherwise)
    _check_walk_sides(g, rs, offsets, inc_edge, inc_end)
    # inside a bucket, (edge, end) strictly ascending
    key = j * 2 + inc_end
    same = bucket[1:] == bucket[:-1]
    assert (key[1:][same] > key[:-1][same]).all()
    # degree identity: multiplicity summed over a node's incidences equals twice
    # its count minus the reads that begin with it and the reads that end with it
    deg = np.zeros(n, np.int64)
    np.add.at(deg, node, g.edge_mult[j].astype(np.int64))
    codes = K.codes(rs.bases[:rs.n_bases]) if rs.n_bases else np.zeros(0, np.uint8)
    off = rs.offsets.astype(np.int64)
    ok_reads = np.nonzero(np.diff(off) >= k)[0]
    first = off[ok_reads]
    last = off[ok_reads + 1] - k
    endcount = np.zeros(n, np.int64)
    for starts in (first, last):
        lo, hi = K.window_keys(codes, starts, k)
        clo, chi, _ = K.canonical(lo, hi, k)
        idx = np.array([np.flatnonzero((g.node_key[:, 0] == a) & (g.node_key[:, 1] == b))[0]
                        for a, b in zip(clo, chi)], np.int64)
        np.add.at(endcount, idx, 1)
    assert (deg == 2 * g.node_count.astype(np.int64) - endcount).all()


def test_golden_sec5_example():
    gd = _golden()
    k = int(gd["k"][0])
    rs, g = _graph(gd["read"], k)
    off, e, end = adj_mod.graph_adjacency(g)
    assert off.tolist() == [int(x) for x in gd["offsets"]]
    assert [f"{a}:{b}" for a, b in zip(e.tolist(), end.tolist())] == gd["entries"]
    check_adjacency(g, rs, off, e, end)


SPECIAL = [(["AAAA"], 3), (["ACAC", "TGTG"], 3), (["ACGT"], 3), (["AC", "ACG", "ACGTA", ""], 3),
           (["ATGG", "CCAT", "GGAC", "GGTC", "TGGA", "TGGT"], 3), (["ACGTACGT"], 1),
           (["GGGGG", "CCCCCC"], 3)]


@pytest.mark.parametrize("idx", range(len(SPECIAL)))
def test_invariants_special(idx):
    reads, k = SPECIAL[idx]
    rs, g = _graph(reads, k)
    check_adjacency(g, rs, *adj_mod.graph_adjacency(g))


def test_invariants_random_and_workload():
    rnd = random.Random(4)
    for t in range(25):
        k = rnd.choice((1, 3, 5, 7, 15, 31, 33))
        alpha = rnd.choice(("AC", "ACGT", "ACGT"))
        reads = ["".join(rnd.choice(alpha) for _ in range(rnd.randint(0, 3 * k + 30)))
                 for _ in range(rnd.randint(1, 30))]
        rs, g = _graph(reads, k)
        check_adjacency(g, rs, *adj_mod.graph_adjacency(g))
    rs = synth.plain_small(scale=0.05)
    g = oracle.build_graph(rs.bases, rs.offsets, 31)
    check_adjacency(g, rs, *adj_mod.graph_adjacency(g))


MUTANTS = {
    "ends_swapped": ("recs.append((iu, o >> 1, j, 0))", "recs.append((iu, o >> 1, j, 1))"),
    "orientations_swapped": ("recs.append((iu, o >> 1, j, 0))", "recs.append((iu, o & 1, j, 0))"),
    "v_end_on_arrowhead_value": ("recs.append((iv, 1 - (o & 1), j, 1))",
                                 "recs.append((iv, o & 1, j, 1))"),
    "u_end_side_flipped": ("recs.append((iu, o >> 1, j, 0))", "recs.append((iu, 1 - (o >> 1), j, 0))"),
    "side_major_order": ("recs.sort()", "recs.sort(key=lambda r: (r[1], r[0], r[2], r[3]))"),
    "self_loop_once": ("recs.append((iv, 1 - (o & 1), j, 1))",
                       "recs.append((iv, 1 - (o & 1), j, 1)) if iv != iu else None"),
    "offsets_shifted": ("offsets[b + 1] = offsets[b] + counts[b]",
                        "offsets[b + 1] = offsets[b] + counts[b - 1] if b else 0"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name):
    old, new = MUTANTS[name]
    src = inspect.getsource(adj_mod.adjacency)
    assert old in src
    ns = {"np": np}
    exec(src.replace(old, new), ns)
    bad = ns["adjacency"]
    failures = 0
    cases = [(["AATGCATC"], 3), (["ACAC", "TGTG"], 3), (["AAAA", "GGGGG"], 3),
             (["ACGTTGCAAGT", "TTGCA"], 3)]
    for reads, k in cases:
        rs, g = _graph(reads, k)
        try:
            out = bad(g.node_key, g.edge_u, g.edge_v, g.edge_orient)
            check_adjacency(g, rs, *out)
            if reads == ["AATGCATC"]:
                gd = _golden()
                assert out[0].tolist() == [int(x) for x in gd["offsets"]]
                assert [f"{a}:{b}" for a, b in zip(out[1].tolist(), out[2].tolist())] == \
                    gd["entries"]
        except (AssertionError, IndexError, KeyError):
            failures += 1
    assert failures > 0, f"mutant {name} passed every pin"
