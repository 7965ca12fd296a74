"""TEST INFRASTRUCTURE ONLY -- the oracle of bi-directed chain compaction (Sec. 7):
the simplified bi-directed graph of a built graph.  Only tests, the smoke check
and the CPU baseline of the benchmark use it.

The steps follow Sec. 7.1 in order, on plain Python lists:

1. Candidate edges.  Sides are those of the STEP-4 lists (side 0 of a node is
   left, side 1 entered, by a walk reading its canonical k-mer forward; the u
   end of (u, v, o1, o2) lies on side o1, the v end on side 1 - o2).  The paper
   offers "one in- and one out-edge" as one possible criterion; it is read per
   edge end: an edge is a candidate when it is not a self-loop and each of its
   two ends is the only end on its side of its node.  Then every node has at most
   one candidate end per side, so the transformed graph below is a set of lists
   and cycles, and no walk through a merged node can be lost (nothing else
   touches the sides that the merge joins).  (Leaving self-loops out changes
   nothing: a self-loop whose two ends are alone on their sides is its node's
   only edge, a cycle of one node that merges nothing.)
2. ListRankingTransform (Lemma 1): every node v becomes v+ (read forward) and
   v- (read reverse-complemented).  Leaving v+ is leaving v by side 0, leaving
   v- by side 1; entering v+ is entering by side 1, entering v- by side 0.  A
   candidate edge joining (u, su) and (v, sv) gives the arc from the copy of u
   that leaves by su to the copy of v that enters by sv, and its twin, from the
   copy of v that leaves by sv to the copy of u that enters by su.
3. List ranking: each list is followed from its head (a copy with no incoming
   arc), numbering its members.  Copies on cycles are reached from no head;
   each cycle is broken on the fly at its smallest node: the list through v+ of
   the smallest node v starts at v+, its twin ends at v-.
4. Both a chain and its reverse complement come out of the ranking.  Each is
   canonicalised (the copy whose first k-mer is the smaller; for a broken
   cycle, the copy starting at v+) and duplicates are removed by sorting.
5. Chains of fewer than ``min_nodes`` nodes (the paper keeps three or more) are
   not compacted: their nodes stay single.

Result (the simplified graph): every node belongs to one chain (a single node
is a chain of one); chains are numbered in the order of their first node's row;
a node has a rank (position along its chain's canonical walk) and an orientation
(0 when the walk reads its canonical k-mer forward).  A chain's label is the
string its walk spells, k + len - 1 bases.  Every edge that is not merged into a
chain (candidate edges inside a kept chain, except the edge that closed a broken
cycle) is kept, in row order, with its ends moved to chain sides: an end on
side s of a node with orientation t lies on side s xor t of the chain, and the
kept edge is written (chain_u, chain_v, o1, o2) with o1 = side at u and
o2 = 1 - side at v, the convention of the input edges.

Plain Python; it shares nothing with the GPU library.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BASES = "ACGT"
_COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def key_string(lo: int, hi: int, k: int) -> str:
    """The k-mer of a key (two bits per base, first base most significant)."""
    v = (int(hi) << 64) | int(lo)
    return "".join(BASES[(v >> (2 * (k - 1 - i))) & 3] for i in range(k))


def revcomp(s: str) -> str:
    return "".join(_COMP[c] for c in reversed(s))


@dataclass
class Compacted:
    node_chain: np.ndarray    # per node: chain number
    node_rank: np.ndarray     # per node: position along the chain's walk
    node_orient: np.ndarray   # per node: 0 forward, 1 reverse complement
    chain_head: np.ndarray    # per chain: row of its first node
    chain_len: np.ndarray     # per chain: nodes
    chain_cyclic: np.ndarray  # per chain: 1 when it was a cycle broken open
    labels: list              # per chain: spelled string
    kept_row: np.ndarray      # kept edges: input edge row
    kept_u: np.ndarray        # kept edges: chain of the u end
    kept_v: np.ndarray        # kept edges: chain of the v end
    kept_orient: np.ndarray   # kept edges: (o1 << 1) | o2 on chain sides

    @property
    def label_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([len(s) for s in self.labels])]).astype(np.uint64)


def _ends(node_key, edge_u, edge_v, edge_orient):
    """Node rows and sides of both ends of every edge."""
    row = {(int(a), int(b)): i for i, (a, b) in enumerate(np.asarray(node_key))}
    ends = []
    for j in range(len(edge_orient)):
        o = int(edge_orient[j])
        u = row[(int(edge_u[j][0]), int(edge_u[j][1]))]
        v = row[(int(edge_v[j][0]), int(edge_v[j][1]))]
        ends.append(((u, o >> 1), (v, 1 - (o & 1))))
    return ends


def compact(node_key, edge_u, edge_v, edge_orient, k: int, min_nodes: int = 3) -> Compacted:
    n = len(node_key)
    m = len(edge_orient)
    kmers = [key_string(a, b, k) for a, b in np.asarray(node_key)]
    ends = _ends(node_key, edge_u, edge_v, edge_orient)

    # step 1: candidate edges
    per_side = {}
    for (a, b) in ends:
        for end in (a, b):
            per_side[end] = per_side.get(end, 0) + 1
    candidate = [a[0] != b[0] and per_side[a] == 1 and per_side[b] == 1 for a, b in ends]

    # step 2: ListRankingTransform; copy (v, t): t = 0 for v+, 1 for v-
    def leaving(side):     # copy that leaves its node by `side`
        return 0 if side == 0 else 1

    def entering(side):    # copy that enters its node by `side`
        return 0 if side == 1 else 1

    nxt, prv, arc_edge = {}, {}, {}
    for j, ((u, su), (v, sv)) in enumerate(ends):
        if not candidate[j]:
            continue
        for (x, sx), (y, sy) in (((u, su), (v, sv)), ((v, sv), (u, su))):
            a, b = (x, leaving(sx)), (y, entering(sy))
            assert a not in nxt and b not in prv, "not a list: a side has two candidate ends"
            nxt[a] = b
            prv[b] = a
            arc_edge[a] = j

    # step 3: list ranking from the heads; cycles broken at their smallest node
    lists = []
    placed = set()
    for v in range(n):
        for t in (0, 1):
            c = (v, t)
            if c in prv or c in placed:
                continue
            walk = [c]
            while walk[-1] in nxt:
                walk.append(nxt[walk[-1]])
            placed.update(walk)
            lists.append((walk, False))
    for v in range(n):
        if (v, 0) in placed:
            continue
        # v lies on a cycle; collect it and start at its smallest node, forward
        cyc = [(v, 0)]
        while nxt[cyc[-1]] != cyc[0]:
            cyc.append(nxt[cyc[-1]])
        low = min(x for x, _ in cyc)
        if (low, 0) not in cyc:  # this is the twin cycle: take the other one
            cyc = [(x, 1 - t) for x, t in reversed(cyc)]
        i = cyc.index((low, 0))
        walk = cyc[i:] + cyc[:i]
        twin = [(x, 1 - t) for x, t in reversed(walk)]
        placed.update(walk)
        placed.update(twin)
        lists.append((walk, True))
        lists.append((twin, True))

    # step 4: canonical copy of every chain, duplicates removed by sorting
    def first_kmer(walk):
        v, t = walk[0]
        return kmers[v] if t == 0 else revcomp(kmers[v])

    canon = []
    for walk, cyclic in lists:
        twin = [(x, 1 - t) for x, t in reversed(walk)]
        if cyclic:
            choose = walk if walk[0][1] == 0 and walk[0][0] == min(x for x, _ in walk) else twin
        else:
            choose = walk if first_kmer(walk) <= first_kmer(twin) else twin
        canon.append((tuple(choose), cyclic))
    canon = sorted(set(canon))

    # step 5: keep chains of min_nodes or more; the rest become single nodes
    chains = []
    for walk, cyclic in canon:
        if len(walk) >= max(min_nodes, 1) or len(walk) == 1:
            chains.append((list(walk), cyclic if len(walk) > 1 else False))
        else:
            for x, _ in walk:
                chains.append(([(x, 0)], False))
    chains.sort(key=lambda c: c[0][0][0])

    node_chain = np.zeros(n, np.int64)
    node_rank = np.zeros(n, np.int64)
    node_orient = np.zeros(n, np.uint8)
    labels = []
    for ci, (walk, _) in enumerate(chains):
        for r, (x, t) in enumerate(walk):
            node_chain[x], node_rank[x], node_orient[x] = ci, r, t
        s = first_kmer(walk)
        for x, t in walk[1:]:
            s += (kmers[x] if t == 0 else revcomp(kmers[x]))[-1]
        labels.append(s)

    # merged edges: the arc that joins rank r to rank r + 1 of a kept chain
    merged = set()
    for walk, _ in chains:
        for c in walk[:-1]:
            merged.add(arc_edge[c])
    kept = [j for j in range(m) if j not in merged]
    ku, kv, ko = [], [], []
    for j in kept:
        (u, su), (v, sv) = ends[j]
        cu = su ^ int(node_orient[u])
        cv = sv ^ int(node_orient[v])
        ku.append(node_chain[u])
        kv.append(node_chain[v])
        ko.append((cu << 1) | (1 - cv))
    return Compacted(node_chain, node_rank, node_orient,
                     np.array([w[0][0] for w, _ in chains], np.int64),
                     np.array([len(w) for w, _ in chains], np.int64),
                     np.array([1 if c else 0 for _, c in chains], np.uint8), labels,
                     np.array(kept, np.int64), np.array(ku, np.int64), np.array(kv, np.int64),
                     np.array(ko, np.uint8))


def graph_compact(g, min_nodes: int = 3) -> Compacted:
    """compact() of an OracleGraph."""
    return compact(g.node_key, g.edge_u, g.edge_v, g.edge_orient, g.k, min_nodes)
