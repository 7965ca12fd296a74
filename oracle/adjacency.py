"""TEST INFRASTRUCTURE ONLY -- the oracle of STEP-4 (Sec. 3): adjacency lists of the
bi-directed de Bruijn graph, from the node table and the edge list of the oracle.

Reading (the paper leaves the representation open): every distinct edge
(u, v, o1, o2) has two ends, one at u and one at v.  A node has two sides: side
0 is the end of its canonical k-mer that a walk reading the k-mer forward leaves
by (its suffix end), side 1 the end such a walk enters by (its prefix end).  The
STEP-1 record of a (k+1)-mer z = x.c with y = z[2..k+1] says how z passes the two
nodes: o1 = '+' when x is read forward, so the walk leaves u by side 0, and by
side 1 when o1 = '-'; o2 = '+' when y is read forward, so the walk enters v by
side 1, and by side 0 when o2 = '-'.  Hence the u end lies on side o1 and the v
end on side 1 - o2 ('+' = 0, '-' = 1).  The same sides result when the record
is written the other way round, (v, u, not o2, not o1), as the ELSE branches of
STEP-1 write it, so the side of an end does not depend on which endpoint the
record lists first.  A walk through a node uses one end on each side (the
walk rule of Sec. 2, read as the arrowheads' direction into or out of the node).
A self-loop gives its node two ends.  The adjacency lists are the ends grouped
by (node, side), nodes in node-table order and side 0 before side 1, and
ordered inside a group by edge row, u end first.  As a CSR: offsets[2 i + s] ..
offsets[2 i + s + 1] index the entries (edge row, end) of node i's side s; there
are 2 n_nodes + 1 offsets and 2 n_edges entries.

Written with plain Python lists and tuples (one sort); it shares nothing with the
GPU library.
"""

from __future__ import annotations

import numpy as np


def adjacency(node_key, edge_u, edge_v, edge_orient):
    """(offsets uint64[2 n + 1], inc_edge uint64[2 m], inc_end uint8[2 m]) of a
    graph given as (n, 2) node keys (sorted), (m, 2) endpoint keys and m
    orientation bytes ((o1 << 1) | o2)."""
    index = {(int(a), int(b)): i for i, (a, b) in enumerate(np.asarray(node_key))}
    n = len(index)
    recs = []
    for j in range(len(edge_orient)):
        o = int(edge_orient[j])
        iu = index[(int(edge_u[j][0]), int(edge_u[j][1]))]
        iv = index[(int(edge_v[j][0]), int(edge_v[j][1]))]
        recs.append((iu, o >> 1, j, 0))
        recs.append((iv, 1 - (o & 1), j, 1))
    recs.sort()
    counts = [0] * (2 * n)
    for node, side, _, _ in recs:
        counts[2 * node + side] += 1
    offsets = [0] * (2 * n + 1)
    for b in range(2 * n):
        offsets[b + 1] = offsets[b] + counts[b]
    return (np.array(offsets, np.uint64), np.array([r[2] for r in recs], np.uint64),
            np.array([r[3] for r in recs], np.uint8))


def graph_adjacency(g):
    """adjacency() of an OracleGraph."""
    return adjacency(g.node_key, g.edge_u, g.edge_v, g.edge_orient)
