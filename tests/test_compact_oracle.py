"""Pins of the chain-compaction oracle (Sec. 7, CPU): the hand-derived result of the
Sec. 5.1 example read, closed forms (a linear genome compacts to one chain that
spells it, a circular genome to one broken cycle that spells its rotation from
the smallest k-mer), a brute force that finds unitigs from the read strings
alone, structural invariants (labels spell the chain's nodes, kept edges spell
their (k+1)-mers, every read stays a walk), and planted mistakes that each pin
must catch."""

import inspect
import os
import random

import numpy as np
import pytest

import oracle
from oracle import compact as cmod
from paper_1003_1940_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sec7_compaction_example.txt")
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def rc(s):
    return "".join(COMP[c] for c in reversed(s))


def canon(s):
    return min(s, rc(s))


def _graph(reads, k):
    rs = synth.from_strings(reads)
    return oracle.build_graph(rs.bases, rs.offsets, k)


def _golden():
    d = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        d[key] = vals
    return d


# ---------------------------------------------------------------- invariants

def _node_strings(g):
    return [cmod.key_string(a, b, g.k) for a, b in g.node_key]


def _edge_zmer(g, j, kmers, row):
    """(k+1)-mer of edge row j, spelled from its record."""
    o = int(g.edge_orient[j])
    u = row[(int(g.edge_u[j][0]), int(g.edge_u[j][1]))]
    v = row[(int(g.edge_v[j][0]), int(g.edge_v[j][1]))]
    x = kmers[u] if (o >> 1) == 0 else rc(kmers[u])
    y = kmers[v] if (o & 1) == 0 else rc(kmers[v])
    assert x[1:] == y[:-1]
    return x + y[-1]


def check_compacted(g, c, reads=None, min_nodes=3):
    k = g.k
    n, m = len(g.node_key), len(g.edge_orient)
    kmers = _node_strings(g)
    row = {(int(a), int(b)): i for i, (a, b) in enumerate(g.node_key)}
    nc = len(c.labels)
    # chains partition the nodes; ranks run 0 .. len - 1; heads ascend
    assert sorted(c.node_chain.tolist()) == sorted(
        sum([[i] * int(L) for i, L in enumerate(c.chain_len)], []))
    assert (np.diff(c.chain_head) > 0).all() if nc > 1 else True
    members = [[] for _ in range(nc)]
    for v in range(n):
        members[c.node_chain[v]].append((int(c.node_rank[v]), v, int(c.node_orient[v])))
    for ci in range(nc):
        mem = sorted(members[ci])
        assert [r for r, _, _ in mem] == list(range(len(mem)))
        assert mem[0][1] == c.chain_head[ci]
        L = len(mem)
        assert L == 1 or L >= min_nodes
        s = c.labels[ci]
        assert len(s) == k + L - 1
        # the label spells the chain's nodes in order
        for r, v, t in mem:
            assert s[r:r + k] == (kmers[v] if t == 0 else rc(kmers[v]))
        if L == 1:
            assert mem[0][2] == 0 and s == kmers[mem[0][1]]
        elif c.chain_cyclic[ci]:
            # a broken cycle starts at its smallest node, read forward, and its
            # last k-mer runs back into its first
            assert mem[0][1] == min(v for _, v, _ in mem) and mem[0][2] == 0
        else:
            assert s[:k] < rc(s)[:k]
    # every edge is merged (joins consecutive ranks of one chain) or kept
    merged = m - len(c.kept_row)
    assert merged == sum(int(L) - 1 for L in c.chain_len)
    assert (np.diff(c.kept_row) > 0).all() if len(c.kept_row) > 1 else True
    for j, cu, cv, o in zip(c.kept_row, c.kept_u, c.kept_v, c.kept_orient):
        su, sv = int(o) >> 1, 1 - (int(o) & 1)
        Su, Sv = c.labels[cu], c.labels[cv]
        x = Su[-k:] if su == 0 else rc(Su[:k])
        y = Sv[:k] if sv == 1 else rc(Sv[-k:])
        assert x[1:] == y[:-1], f"kept edge {j} does not join its chains' ends"
        assert canon(x + y[-1]) == canon(_edge_zmer(g, int(j), kmers, row)), \
            f"kept edge {j} spells another (k+1)-mer"
    # every read is still a walk: consecutive k-mers follow their chain's order
    # or cross a kept edge
    if reads:
        where = {}
        for ci in range(nc):
            for r, v, t in members[ci]:
                where[kmers[v]] = (ci, r, t)
        kept_set = set()
        for j in c.kept_row:
            kept_set.add(canon(_edge_zmer(g, int(j), kmers, row)))
        for read in reads:
            for i in range(len(read) - k):
                x, y = read[i:i + k], read[i + 1:i + k + 1]
                cx, cy = canon(x), canon(y)
                ax, ay = where[cx], where[cy]
                fx = 0 if x == cx else 1
                fy = 0 if y == cy else 1
                inside = (ax[0] == ay[0] and (
                    (fx == ax[2] and fy == ay[2] and ay[1] == ax[1] + 1) or
                    (fx != ax[2] and fy != ay[2] and ay[1] == ax[1] - 1)))
                assert inside or canon(x + y[-1]) in kept_set, \
                    f"read step {x}->{y} is neither inside a chain nor a kept edge"


# -------------------------------------------------------------- brute force

def brute_unitigs(reads, k):
    """Maximal non-branching walks from the read strings alone: oriented k-mers,
    successors and predecessors by one-base extension present as a (k+1)-mer of
    some read (either strand).  Returns the chain labels (linear chains: the
    smaller of the spelled string and its reverse complement; cycles: the walk
    from the smallest canonical k-mer, read forward)."""
    zset = set()
    nodes = set()
    for r in reads:
        for i in range(len(r) - k + 1):
            nodes.add(canon(r[i:i + k]))
        for i in range(len(r) - k):
            zset.add(canon(r[i:i + k + 1]))

    def succ(x):
        return [x[1:] + b for b in "ACGT" if canon(x + b) in zset]

    def pred(x):
        return [b + x[:-1] for b in "ACGT" if canon(b + x) in zset]

    def link(x):  # the unique successor joined to x, or None
        s = succ(x)
        if len(s) != 1:
            return None
        y = s[0]
        if canon(y) == canon(x) or len(pred(y)) != 1:
            return None
        return y

    def back(x):
        p = pred(x)
        if len(p) != 1:
            return None
        w = p[0]
        return w if link(w) == x else None

    labels, seen = [], set()
    for v in sorted(nodes):
        if v in seen:
            continue
        # walk back to the start of v's chain (or around a cycle)
        x, cyc = v, False
        while True:
            w = back(x)
            if w is None:
                break
            if canon(w) == v:
                cyc = True
                break
            x = w
        if cyc:
            walk = [v]
            while True:
                y = link(walk[-1])
                if canon(y) == v:
                    break
                walk.append(y)
            low = min(canon(w) for w in walk)
            # restart at the smallest node, read forward
            if low not in walk:
                walk = [rc(w) for w in reversed(walk)]
            i = walk.index(low)
            walk = walk[i:] + walk[:i]
        else:
            walk = [x]
            while link(walk[-1]) is not None:
                walk.append(link(walk[-1]))
        for w in walk:
            seen.add(canon(w))
        s = walk[0] + "".join(w[-1] for w in walk[1:])
        labels.append((s if cyc else min(s, rc(s)), len(walk), cyc))
    return labels


def _labels_under(brute, min_nodes):
    out = []
    for s, L, cyc in brute:
        if L >= min_nodes or L == 1:
            out.append(s)
        else:
            k = len(s) - L + 1
            out += [canon(s[i:i + k]) for i in range(L)]
    return sorted(out)


# --------------------------------------------------------------------- pins

def test_golden_sec5_example():
    gd = _golden()
    k = int(gd["k"][0])
    g = _graph(gd["read"], k)
    for mn in (2, 3):
        c = cmod.graph_compact(g, mn)
        p = f"min{mn}."
        assert c.node_chain.tolist() == [int(x) for x in gd[p + "node_chain"]]
        assert c.node_rank.tolist() == [int(x) for x in gd[p + "node_rank"]]
        assert c.node_orient.tolist() == [int(x) for x in gd[p + "node_orient"]]
        assert c.labels == gd[p + "labels"]
        kept = [f"{a}:{b}:{d}:{e}" for a, b, d, e in
                zip(c.kept_row, c.kept_u, c.kept_v, c.kept_orient)]
        assert kept == gd[p + "kept"]
        check_compacted(g, c, gd["read"], mn)


def _distinct_kmer_genome(rnd, length, k, circular=False):
    while True:
        G = "".join(rnd.choice("ACGT") for _ in range(length))
        ext = G + G[:k - 1] if circular else G
        ks = [canon(ext[i:i + k]) for i in range(len(ext) - k + 1)]
        if len(set(ks)) == len(ks):
            return G


@pytest.mark.parametrize("k,length", [(5, 60), (11, 400), (31, 2000), (33, 1500), (63, 3000)])
def test_linear_genome_closed_form(k, length):
    """Error-free reads tiling a genome whose canonical k-mers are distinct: the
    graph is one path and compacts to one chain spelling the genome or its
    reverse complement (the one with the smaller first k-mer); no edge is kept."""
    rnd = random.Random(k * 1000 + length)
    G = _distinct_kmer_genome(rnd, length, k)
    rl = 3 * k
    reads = [G[i:i + rl] for i in range(0, length - rl + 1, k)] + [G[-rl:]]
    g = _graph(reads, k)
    for mn in (2, 3):
        c = cmod.graph_compact(g, mn)
        want = G if G[:k] < rc(G)[:k] else rc(G)
        assert c.labels == [want]
        assert len(c.kept_row) == 0 and c.chain_cyclic.tolist() == [0]
        check_compacted(g, c, reads, mn)


@pytest.mark.parametrize("k,length", [(5, 40), (11, 300), (31, 1000), (63, 1200)])
def test_circular_genome_closed_form(k, length):
    """Reads tiling a circular genome with distinct canonical k-mers: one cycle,
    broken at its smallest node read forward; the label is the rotation from
    there (on the strand that holds that k-mer forward) plus k - 1 wrapped bases,
    and the closing edge is kept as a self-loop from the chain's end to its
    start.  Its record lists the smallest node (the chain's first) as u, whose end
    is the chain's entry side 1 (o1 = 1), and the last node as v, whose end is
    the chain's exit side 0 (o2 = 1 - 0): (0, 0, o1 1, o2 1)."""
    rnd = random.Random(7 * k + length)
    G = _distinct_kmer_genome(rnd, length, k, circular=True)
    rl = 2 * k
    ext = G + G[:rl]
    reads = [ext[i:i + rl] for i in range(0, length, k // 2 + 1)]
    g = _graph(reads, k)
    low = min(canon((G + G)[i:i + k]) for i in range(length))
    strand = G if low in G + G[:k - 1] else rc(G)
    i = (strand + strand[:k - 1]).index(low)
    rot = strand[i:] + strand[:i]
    want = rot + rot[:k - 1]
    for mn in (2, 3):
        c = cmod.graph_compact(g, mn)
        assert c.labels == [want]
        assert c.chain_cyclic.tolist() == [1]
        assert [(int(a), int(b), int(o)) for a, b, o in zip(c.kept_u, c.kept_v, c.kept_orient)] \
            == [(0, 0, 3)]
        check_compacted(g, c, reads, mn)


def _random_reads(rnd, k):
    alpha = rnd.choice(("AC", "ACGT", "ACGT", "ACG"))
    if rnd.random() < 0.3:
        # reads around a short circular sequence (cycles, sometimes with a
        # substitution that branches off them)
        C = "".join(rnd.choice(alpha) for _ in range(rnd.randint(3, 6 * k + 20)))
        ext = C * (2 + (3 * k + 10) // len(C))
        reads = []
        for _ in range(rnd.randint(2, 25)):
            L = rnd.randint(k, 3 * k + 10)
            i = rnd.randrange(len(C))
            r = ext[i:i + L]
            if rnd.random() < 0.15:
                j = rnd.randrange(L)
                r = r[:j] + rnd.choice("ACGT") + r[j + 1:]
            reads.append(r if rnd.random() < 0.5 else rc(r))
        return reads
    if rnd.random() < 0.5:
        G = "".join(rnd.choice(alpha) for _ in range(rnd.randint(k + 5, 8 * k + 60)))
        reads = []
        for _ in range(rnd.randint(1, 25)):
            L = rnd.randint(k, min(len(G), 3 * k + 10))
            i = rnd.randint(0, len(G) - L)
            r = G[i:i + L]
            if rnd.random() < 0.3:
                j = rnd.randrange(L)
                r = r[:j] + rnd.choice("ACGT") + r[j + 1:]
            reads.append(r if rnd.random() < 0.5 else rc(r))
        return reads
    return ["".join(rnd.choice(alpha) for _ in range(rnd.randint(0, 3 * k + 20)))
            for _ in range(rnd.randint(1, 20))]


def test_brute_force_random_sets():
    rnd = random.Random(1940)
    for t in range(160):
        k = rnd.choice((1, 3, 5, 7, 9, 15, 31, 33))
        reads = _random_reads(rnd, k)
        g = _graph(reads, k)
        brute = brute_unitigs(reads, k)
        for mn in (2, 3):
            c = cmod.graph_compact(g, mn)
            assert sorted(c.labels) == _labels_under(brute, mn), f"case {t} k={k} min={mn}"
            check_compacted(g, c, reads, mn)


SPECIAL = [(["AAAA"], 3), (["AAAAAAA"], 3), (["ACAC", "TGTG"], 3), (["ACGT"], 3),
           (["ACGTACGT"], 1), (["ACGTACGT"], 3), (["AC" * 20], 1), (["AC" * 20], 3),
           (["GGGGG", "CCCCCC"], 3), (["ATGG", "CCAT", "GGAC", "GGTC", "TGGA", "TGGT"], 3),
           (["AC", "ACG", "ACGTA", ""], 3), (["ACG"], 5), ([""], 3)]


@pytest.mark.parametrize("idx", range(len(SPECIAL)))
def test_special_cases(idx):
    reads, k = SPECIAL[idx]
    g = _graph(reads, k)
    brute = brute_unitigs(reads, k)
    for mn in (1, 2, 3, 4):
        c = cmod.graph_compact(g, mn)
        assert sorted(c.labels) == _labels_under(brute, max(mn, 1))
        check_compacted(g, c, reads, max(mn, 1))


def test_workload_invariants():
    rng = np.random.default_rng(77)
    G = synth.random_genome(rng, 3000)
    rs = synth.sample_reads(rng, G, 400, 60, 0.01)
    k = 15
    g = oracle.build_graph(rs.bases, rs.offsets, k)
    reads = [bytes(rs.bases[rs.offsets[i]:rs.offsets[i + 1]]).decode() for i in range(400)]
    c = cmod.graph_compact(g, 3)
    check_compacted(g, c, reads, 3)
    assert sorted(c.labels) == _labels_under(brute_unitigs(reads, k), 3)
    # most k-mers of a 60x error-free-ish genome sit in chains of three or more
    assert (c.chain_len >= 3).sum() > 0


# ---------------------------------------------------------- planted mistakes

MUTANTS = {
    "sides_as_arrowheads": ("ends.append(((u, o >> 1), (v, 1 - (o & 1))))",
                            "ends.append(((u, o >> 1), (v, o & 1)))"),
    "min_nodes_ignored": ("if len(walk) >= max(min_nodes, 1) or len(walk) == 1:",
                          "if True:"),
    "cycle_broken_at_largest": ("low = min(x for x, _ in cyc)", "low = max(x for x, _ in cyc)"),
    "larger_twin": ("choose = walk if first_kmer(walk) <= first_kmer(twin) else twin",
                    "choose = walk if first_kmer(walk) > first_kmer(twin) else twin"),
    "chain_side_without_orientation": ("cu = su ^ int(node_orient[u])", "cu = su"),
    "entering_flipped": ("return 0 if side == 1 else 1", "return 0 if side == 0 else 1"),
    "closing_edge_merged": ("for c in walk[:-1]:", "for c in walk:"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name):
    old, new = MUTANTS[name]
    src = inspect.getsource(cmod)
    assert old in src, name
    ns = {}
    exec(compile(src.replace(old, new), "mutant", "exec"), ns)
    bad = ns["compact"]
    rnd = random.Random(3)
    G = _distinct_kmer_genome(rnd, 120, 7)
    Gc = _distinct_kmer_genome(rnd, 80, 7, circular=True)
    cases = [(["AATGCATC"], 3, 2), (["AATGCATC"], 3, 3), ([G[i:i + 21] for i in range(0, 100, 5)], 7, 2),
             ([(Gc + Gc[:21])[i:i + 21] for i in range(0, 80, 4)], 7, 3), (["AAAAAAA", "ACGTT"], 3, 2)]
    for t in range(6):
        k = rnd.choice((3, 5, 7))
        cases.append((_random_reads(rnd, k), k, rnd.choice((2, 3))))
    failures = 0
    for reads, k, mn in cases:
        g = _graph(reads, k)
        try:
            c = bad(g.node_key, g.edge_u, g.edge_v, g.edge_orient, k, mn)
            check_compacted(g, c, reads, mn)
            assert sorted(c.labels) == _labels_under(brute_unitigs(reads, k), mn)
            if reads == ["AATGCATC"]:
                gd = _golden()
                assert c.labels == gd[f"min{mn}.labels"]
                kept = [f"{a}:{b}:{d}:{e}" for a, b, d, e in
                        zip(c.kept_row, c.kept_u, c.kept_v, c.kept_orient)]
                assert kept == gd[f"min{mn}.kept"]
        except (AssertionError, IndexError, KeyError, ValueError, RecursionError):
            failures += 1
    assert failures > 0, f"mutant {name} passed every pin"
