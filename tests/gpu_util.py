"""Helpers for the GPU tests: run the library, compare with the oracle."""

import sys

import numpy as np

import oracle

FIELDS = ("node_key", "node_count", "edge_u", "edge_v", "edge_orient", "edge_mult", "edge_z")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_graph(bases, offsets, k, **kw):
    import paper_1003_1940_amd as dbg
    g = dbg.build(np.asarray(bases, np.uint8), np.asarray(offsets, np.uint64), k, **kw)
    return g, g.to_numpy()


def compare_with_oracle(bases, offsets, k, label="", threads=0):
    """Element-by-element equality of every output column with the oracle."""
    say(f"[gpu-parity] {label} k={k} reads={len(offsets) - 1} bases={int(offsets[-1])}")
    g, got = gpu_graph(bases, offsets, k)
    assert g.status == 0, f"{label}: device status {g.status}"
    ref = oracle.build_graph(bases, offsets, k, threads=threads)
    assert g.n_nodes == len(ref.node_count), f"{label}: n_nodes {g.n_nodes} != {len(ref.node_count)}"
    assert g.n_edges == len(ref.edge_mult), f"{label}: n_edges {g.n_edges} != {len(ref.edge_mult)}"
    for f in FIELDS:
        a, b = got[f], getattr(ref, f)
        if a is None:
            continue
        if not np.array_equal(np.asarray(a), np.asarray(b)):
            bad = np.nonzero(np.asarray(a).reshape(len(a), -1) != np.asarray(b).reshape(len(b), -1))[0]
            raise AssertionError(f"{label}: column {f} differs at rows {bad[:10]} "
                                 f"(gpu {a[bad[:3]]} vs oracle {b[bad[:3]]})")
    return g, got, ref
