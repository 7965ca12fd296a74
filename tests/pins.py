"""Checks that pin the oracle to facts outside itself.

Each ``pin_*`` function raises AssertionError on a mismatch.  They take the path
of an oracle build (``None`` = the normal one) so the mutation test can run them
against deliberately broken copies of the oracle's source.
"""

import os
import random

import numpy as np

import oracle
from . import brute
from . import keys_np as K
from .invariants import check_graph

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_fixture(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


def _input(reads):
    bases = "".join(reads).encode()
    offsets = np.zeros(len(reads) + 1, np.uint64)
    np.cumsum([len(r) for r in reads], out=offsets[1:])
    return bases, offsets


def oracle_strings(reads, k, lib_path=None):
    """Oracle output on a list of string reads, as (node_rows, edge_rows) in the
    same shape as ``brute.brute_tables``."""
    bases, offsets = _input(reads)
    g = oracle.build_graph(bases, offsets, k, threads=2, strings=True, lib_path=lib_path)
    nodes = [(s, int(c)) for s, c in zip(g.node_str, g.node_count)]
    edges = [(u, v, o, z, int(m)) for (u, v, o, z), m in zip(g.edge_str, g.edge_mult)]
    return nodes, edges, g


def edge_spellings(edge_rows):
    """Every (k+1)-mer an edge stands for, read along either strand."""
    out = set()
    for u, v, o, _z, _m in edge_rows:
        s = brute.spell((u, v, o[0], o[1]))
        out.add(s)
        out.add(brute.rc(s))
    return out


# ---------------------------------------------------------------------------
# Values the paper prints.

def pin_reverse_complement(lib_path=None):
    for kmer, expected in read_fixture("sec2_reverse_complement.txt"):
        assert oracle.revcomp(kmer, lib_path=lib_path) == expected


def pin_fig2(lib_path=None):
    rows = {r[0]: r[1:] for r in read_fixture("fig2_example.txt") if r[0] in ("k", "reads", "source", "walk")}
    mols = [r[1:] for r in read_fixture("fig2_example.txt") if r[0] == "molecule"]
    edges = [r[1:] for r in read_fixture("fig2_example.txt") if r[0] == "edge"]
    k = int(rows["k"][0])
    reads = rows["reads"]
    nodes, erows, _ = oracle_strings(reads, k, lib_path)
    node_set = {n for n, _ in nodes}
    for pos, neg in mols:
        # the positive strand is the node key, and the negative one is its reverse complement
        assert pos in node_set and oracle.revcomp(pos, lib_path=lib_path) == neg
    spellings = edge_spellings(erows)
    for x, y, o in edges:
        sx = x if o[0] == "+" else brute.rc(x)
        sy = y if o[1] == "+" else brute.rc(y)
        assert sx + sy[-1] in spellings
    # The printed read GTTC occurs in neither strand of the source; reading it as
    # GGTC (which does) makes every step of the dashed walk an edge, and with the
    # read as printed exactly the step GACC is missing.
    walk = rows["walk"][0]
    steps = [walk[i:i + k + 1] for i in range(len(walk) - k)]
    assert [s for s in steps if s not in spellings] == ["GACC"]
    fixed = ["GGTC" if r == "GTTC" else r for r in reads]
    _, erows_fixed, _ = oracle_strings(fixed, k, lib_path)
    assert all(s in edge_spellings(erows_fixed) for s in steps)


def pin_spurious_edge(lib_path=None):
    fx = {r[0]: r[1:] for r in read_fixture("sec5_1_spurious_edge.txt")}
    k = int(fx["k"][0])
    nodes, erows, _ = oracle_strings(fx["reads"], k, lib_path)
    node_set = {n for n, _ in nodes}
    assert {brute.molecule(v) for v in fx["vertices"]} <= node_set
    pairs = {frozenset((u, v)) for u, v, *_ in erows}
    a, b = fx["no_edge"]
    assert frozenset((brute.molecule(a), brute.molecule(b))) not in pairs
    a, b = fx["edge_between"]
    assert frozenset((brute.molecule(a), brute.molecule(b))) in pairs


# ---------------------------------------------------------------------------
# Brute force from the definition.

def pin_exhaustive(ks=(1, 3, 5, 7), lib_path=None):
    """Every (k+1)-mer as a read of its own, all in one input: the oracle's records
    and multiplicities equal the definition's."""
    for k in ks:
        n = k + 1
        reads = ["".join("ACGT"[(v >> (2 * (n - 1 - i))) & 3] for i in range(n))
                 for v in range(4 ** n)]
        o_nodes, o_edges, _ = oracle_strings(reads, k, lib_path)
        b_nodes, b_edges = brute.brute_tables(reads, k)
        assert o_nodes == b_nodes, f"k={k}: nodes differ from the definition"
        assert o_edges == b_edges, f"k={k}: edges differ from the definition"
        # records and canonical (k+1)-mers are in one-to-one correspondence
        assert len(o_edges) == len({brute.molecule(r) for r in reads})


def pin_single_kmers(ks=(1, 3), lib_path=None):
    """Each (k+1)-mer alone: exactly one edge, whose spelling is that (k+1)-mer
    or its reverse complement."""
    for k in ks:
        n = k + 1
        for v in range(4 ** n):
            z = "".join("ACGT"[(v >> (2 * (n - 1 - i))) & 3] for i in range(n))
            _, erows, _ = oracle_strings([z], k, lib_path)
            assert len(erows) == 1 and erows[0][4] == 1
            assert brute.spell(tuple(erows[0][:2]) + tuple(erows[0][2])) in (z, brute.rc(z))


def pin_random_sets(n_sets=150, seed=7, lib_path=None):
    rnd = random.Random(seed)
    for t in range(n_sets):
        k = rnd.choice((1, 3, 5, 7))
        alpha = rnd.choice(("AC", "ACGT", "AT", "ACGT"))
        reads = ["".join(rnd.choice(alpha) for _ in range(rnd.randint(0, 3 * k + 2)))
                 for _ in range(rnd.randint(1, 6))]
        o_nodes, o_edges, g = oracle_strings(reads, k, lib_path)
        b_nodes, b_edges = brute.brute_tables(reads, k)
        assert o_nodes == b_nodes, f"set {t} k={k} {reads}: nodes"
        assert o_edges == b_edges, f"set {t} k={k} {reads}: edges"
        bases, offsets = _input(reads)
        check_graph(g, k, np.frombuffer(bases, np.uint8), offsets)


# ---------------------------------------------------------------------------
# Hand-derived special cases (each derivation is in the comment).

def pin_special_cases(lib_path=None):
    # AAAA, k=3: k-mers AAA, AAA -> node AAA count 2; one (k+1)-mer AAAA whose two
    # k-mers are both the positive strand of AAA -> (AAA, AAA, ++).
    # TTTT is the reverse complement of AAAA, so it must give the same record.
    for r in ("AAAA", "TTTT"):
        n, e, _ = oracle_strings([r], 3, lib_path)
        assert n == [("AAA", 2)] and e == [("AAA", "AAA", "++", "AAAA", 1)], r
    # GGGGG: GGG = negative strand of CCC, three times; two (k+1)-mers GGGG.
    n, e, _ = oracle_strings(["GGGGG"], 3, lib_path)
    assert n == [("CCC", 3)] and e == [("CCC", "CCC", "++", "CCCC", 2)]
    # ACAC and TGTG: ACA, CAC are both canonical; ACAC joins them on their
    # positive strands, while TGTG = TGT GTG = negative strands of ACA and CAC, so
    # the same pair of k-molecules carries two different edges.
    n, e, _ = oracle_strings(["ACAC", "TGTG"], 3, lib_path)
    assert n == [("ACA", 2), ("CAC", 2)]
    assert e == [("ACA", "CAC", "++", "ACAC", 1), ("ACA", "CAC", "--", "CACA", 1)]
    # ACGT is its own reverse complement: ACG (positive) then CGT (the negative
    # strand of ACG) -> a self-edge (ACG, ACG, +-).
    n, e, _ = oracle_strings(["ACGT"], 3, lib_path)
    assert n == [("ACG", 2)] and e == [("ACG", "ACG", "+-", "ACGT", 1)]
    # Reads shorter than k add nothing; a read of length exactly k adds a node and
    # no edge; the empty read adds nothing.
    n, e, _ = oracle_strings(["AC", "ACG", "ACGTA", ""], 3, lib_path)
    assert n == [("ACG", 3), ("GTA", 1)]
    assert e == [("ACG", "ACG", "+-", "ACGT", 1), ("ACG", "GTA", "-+", "CGTA", 1)]


# ---------------------------------------------------------------------------
# Sort + run-length reduce reduces to a library routine.

def pin_numpy_unique(rs, k, lib_path=None):
    """np.unique over canonical keys computed by numpy equals the oracle's node
    table, and its edge column z with multiplicities."""
    g = oracle.build_graph(rs.bases, rs.offsets, k, threads=0, lib_path=lib_path)
    lo, hi, cnt = K.unique_keys(rs.bases, rs.offsets, k)
    assert np.array_equal(g.node_key[:, 0], lo) and np.array_equal(g.node_key[:, 1], hi)
    assert np.array_equal(g.node_count, cnt.astype(np.uint64))
    lo, hi, cnt = K.unique_keys(rs.bases, rs.offsets, k + 1)
    assert np.array_equal(g.edge_z[:, 0], lo) and np.array_equal(g.edge_z[:, 1], hi)
    assert np.array_equal(g.edge_mult, cnt.astype(np.uint64))
    return g


ALL_PINS = (pin_reverse_complement, pin_fig2, pin_spurious_edge, pin_special_cases,
            pin_exhaustive, pin_random_sets)
