"""TEST INFRASTRUCTURE ONLY -- the oracle of STEP-4 (Sec. 3): adjacency lists of the
bi-directed de Bruijn graph, from the node table and the edge list of the oracle.

Reading (the paper leaves the representation open): every distinct edge
(u, v, o1, o2) has two ends, the u end carrying arrowhead orientation o1 and the v
end carrying o2 ('+' = 0, '-' = 1).  Each end is an incidence of its node on the
side named by its orientation; a self-loop gives its node two incidences.  The
adjacency lists are the incidences grouped by (node, side), nodes in node-table
order and side '+' before '-', and ordered inside a group by edge row, u end
first.  As a CSR: offsets[2 i + s] .. offsets[2 i + s + 1] index the entries
(edge row, end) of node i's side s; there are 2 n_nodes + 1 offsets and
2 n_edges entries.

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
        recs.append((iv, o & 1, j, 1))
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
