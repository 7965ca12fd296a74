"""Brute-force bi-directed de Bruijn graph, straight from the definition in Sec. 2.

Pure Python, for tiny inputs only.  It does not use the STEP-1 table at all: it
walks every string of S and of its reverse complements, joins every pair of
adjacent k-mers (x, y), and records the arrow heads by which strand of its
k-molecule each k-mer is.  A bi-directed edge read along the other strand,
(v, u, not o2, not o1), is the same edge, so each record is collapsed to one
representative of that pair (smaller k-molecule first; for a self-pair the smaller
orientation pair).  Every adjacency occurs once on each strand, so the counts over
S and its reverse complements are halved to give counts over the reads.
"""

from collections import Counter

_COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}
FLIP = {"+": "-", "-": "+"}


def rc(s: str) -> str:
    return "".join(_COMP[c] for c in reversed(s))


def molecule(x: str) -> str:
    """The positive strand (canonical k-mer) of x's k-molecule."""
    return min(x, rc(x))


def strand(x: str) -> str:
    return "+" if x == molecule(x) else "-"


def representative(rec):
    a, b, p, q = rec
    return min((a, b, p, q), (b, a, FLIP[q], FLIP[p]))


def spell(rec) -> str:
    """The (k+1)-mer an edge record stands for: the strand of u named by o1,
    followed by the last base of the strand of v named by o2."""
    u, v, o1, o2 = rec
    a = u if o1 == "+" else rc(u)
    b = v if o2 == "+" else rc(v)
    assert a[1:] == b[:-1], "edge endpoints do not overlap by k-1"
    return a + b[-1]


def brute_graph(reads, k):
    """Returns (nodes, edges): nodes {canonical k-mer: count}, edges
    {(u, v, o1, o2): multiplicity} with o in {'+', '-'}."""
    strings = list(reads) + [rc(r) for r in reads]
    node_occ = Counter()
    edge_occ = Counter()
    for z in strings:
        for j in range(len(z) - k + 1):
            node_occ[molecule(z[j:j + k])] += 1
        for j in range(len(z) - k):
            x, y = z[j:j + k], z[j + 1:j + k + 1]
            edge_occ[representative((molecule(x), molecule(y), strand(x), strand(y)))] += 1
    assert all(c % 2 == 0 for c in node_occ.values())
    assert all(c % 2 == 0 for c in edge_occ.values())
    return ({v: c // 2 for v, c in node_occ.items()},
            {e: c // 2 for e, c in edge_occ.items()})


def brute_tables(reads, k):
    """Brute-force result in the output order: nodes ascending, edges ascending by
    the canonical (k+1)-mer they spell.  Returns (node_rows, edge_rows) with
    node_rows [(kmer, count)] and edge_rows [(u, v, 'o1o2', zhat, mult)]."""
    nodes, edges = brute_graph(reads, k)
    node_rows = sorted(nodes.items())
    edge_rows = []
    for (u, v, o1, o2), m in edges.items():
        edge_rows.append((u, v, o1 + o2, molecule(spell((u, v, o1, o2))), m))
    edge_rows.sort(key=lambda r: r[3])
    return node_rows, edge_rows
