"""Out-of-memory build by key-space slices (Sec. 6's out-of-core variant).

The paper sorts more keys than fit in memory as sorted runs and merges them R
ways.  Here the key space is cut instead: ``dbg_prefix_counts`` counts the
canonical (k+1)-mers and k-mers of every 12-bit key prefix on the device,
``plan_slices`` groups consecutive prefixes into slices whose keys fit a budget,
and ``dbg_build_slice`` builds the tables of one slice (re-reading the packed
reads, which take 2 bits per base).  Slices of increasing, disjoint prefix
ranges give increasing, disjoint parts of both sorted tables, so the host
concatenates them in order; nothing is merged.  Device memory holds the reads,
one slice's key buffers and one slice's output rows; the tables accumulate in
host memory.

Every step of the construction runs in the library's kernels; this module
plans the slices and moves the rows.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api

PREFIX_BITS = 12
PREFIX_BINS = 1 << PREFIX_BITS


def positions(offsets: np.ndarray, length: int) -> int:
    """Windows of `length` bases inside the reads (k-mer positions for
    length = k, (k+1)-mer positions for k + 1), from dbg_bounds."""
    off = np.asarray(offsets, np.uint64)
    if length % 2:
        return api.bounds(off, length)[0]
    return api.bounds(off, length - 1)[1]


def prefix_counts(packed, n_bases: int, offs, k: int, max_positions: int, stream=None):
    """(edge_counts, node_counts): uint64[4096] position counts of the canonical
    (k+1)-mer and k-mer prefixes (synchronises)."""
    dev = offs.device
    lib = api.load()
    n_reads = offs.numel() - 1
    nbytes = int(lib.dbg_prefix_workspace_bytes(n_reads, max_positions, k))
    if nbytes == 0:
        raise api.DbgError(2, "dbg_prefix_workspace_bytes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    counts = torch.empty(2 * PREFIX_BINS, dtype=torch.int64, device=dev)
    res = torch.zeros(3, dtype=torch.int64, device=dev)
    rc = lib.dbg_prefix_counts(api._ptr(packed), n_bases, api._ptr(offs), n_reads, k,
                               max_positions, api._ptr(counts[:PREFIX_BINS]),
                               api._ptr(counts[PREFIX_BINS:]), api._ptr(res), api._ptr(ws),
                               nbytes, api._stream(stream))
    if rc:
        raise api.DbgError(rc, "dbg_prefix_counts")
    _, _, st = api.read_result(res)
    if st:
        raise api.DbgError(st, "dbg_prefix_counts (device)")
    c = counts.cpu().numpy().view(np.uint64)
    return c[:PREFIX_BINS].copy(), c[PREFIX_BINS:].copy()


def plan_slices(edge_counts, node_counts, budget: int) -> list:
    """Consecutive prefix ranges [lo, hi) covering [0, 4096), each holding at
    most `budget` keys of either table (greedy, first fit).  A single prefix
    with more keys than the budget cannot be split: ValueError."""
    e = np.asarray(edge_counts, np.uint64).astype(np.int64)
    n = np.asarray(node_counts, np.uint64).astype(np.int64)
    if len(e) != PREFIX_BINS or len(n) != PREFIX_BINS:
        raise ValueError("prefix counts need 4096 bins")
    if budget < 1:
        raise ValueError("budget must be positive")
    big = np.nonzero((e > budget) | (n > budget))[0]
    if len(big):
        raise ValueError(f"prefix {int(big[0])} holds {int(max(e[big[0]], n[big[0]]))} keys, "
                         f"more than the budget of {budget}")
    out, lo, se, sn = [], 0, 0, 0
    for p in range(PREFIX_BINS):
        if se + e[p] > budget or sn + n[p] > budget:
            out.append((lo, p))
            lo, se, sn = p, 0, 0
        se += e[p]
        sn += n[p]
    out.append((lo, PREFIX_BINS))
    return out


@dataclass
class SlicedTables:
    """Host tables of a sliced build (keys as (n, 2) uint64 (lo, hi), the layout
    of ``Graph.to_numpy``) and how they were built."""
    k: int
    tables: dict
    slices: list                               # (lo, hi) prefix ranges
    rows: list = field(default_factory=list)   # (nodes, edges) per slice
    parts: list = field(default_factory=list)  # per slice: pinned host rows by column
    budget: int = 0
    workspace_bytes: int = 0
    seconds: dict = field(default_factory=dict)


def build_slice_async(packed, n_bases: int, offs, k: int, max_positions: int, max_keys: int,
                      lo: int, hi: int, out: dict, node_cap: int, edge_cap: int, result,
                      ws, stream=None):
    """Enqueue the build of one slice (no synchronisation)."""
    nodes, edges = api._structs(out, node_cap, edge_cap)
    rc = api.load().dbg_build_slice(api._ptr(packed), n_bases, api._ptr(offs), offs.numel() - 1,
                                    k, max_positions, max_keys, lo, hi, ctypes.byref(nodes),
                                    ctypes.byref(edges), api._ptr(result), api._ptr(ws),
                                    ws.numel(), api._stream(stream))
    if rc:
        raise api.DbgError(rc, "dbg_build_slice")


def _host_rows(out: dict, n_nodes: int, n_edges: int, stream) -> dict:
    """Pinned host copies of one slice's rows, enqueued on `stream`."""
    rows = {}
    for name, t in out.items():
        if t is None:
            rows[name] = None
            continue
        n = n_nodes if name.startswith("node") else n_edges
        h = torch.empty((n,) + tuple(t.shape[1:]), dtype=t.dtype, pin_memory=True)
        if n:
            with torch.cuda.stream(stream):
                h.copy_(t[:n], non_blocking=True)
        rows[name] = h
    return rows


def _numpy_tables(k: int, parts: list) -> dict:
    """Concatenate the slices' pinned rows into the layout of Graph.to_numpy."""
    def keys(name):
        a = np.concatenate([p[name].numpy() for p in parts]).view(np.uint64)
        if a.ndim == 1:
            a = np.stack([a, np.zeros_like(a)], axis=1)
        return a
    def counts(name):
        return np.concatenate([p[name].numpy() for p in parts]).view(np.uint32).astype(np.uint64)
    return dict(node_key=keys("node_kmer"), node_count=counts("node_count"),
                edge_u=keys("edge_u"), edge_v=keys("edge_v"),
                edge_orient=np.concatenate([p["edge_orient"].numpy() for p in parts]),
                edge_mult=counts("edge_mult"),
                edge_z=keys("edge_zkey") if parts[0]["edge_zkey"] is not None else None)


def build_sliced(bases: np.ndarray, offsets: np.ndarray, k: int, budget: int | None = None,
                 n_slices: int | None = None, zkey: bool = False, device="cuda",
                 concatenate: bool = True) -> SlicedTables:
    """Build the graph of (bases, offsets) slice by slice.  `budget` bounds the
    keys of either table in one slice (or `n_slices` sets it to the larger table's
    positions over n_slices); the tables come back on the host.  Two sets of
    device output rows alternate, so that the copy of one slice's rows to pinned
    host memory (on its own stream) runs while the next slice is built.  With
    ``concatenate`` the slices' rows are also joined into numpy tables in the
    layout of ``Graph.to_numpy``; otherwise they stay per slice in ``parts``."""
    import time
    t0 = time.perf_counter()
    offsets = np.asarray(offsets, np.uint64)
    n_pos = max(positions(offsets, k), 1)
    packed, offs, n_bases = api.upload(bases, offsets, device)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ec, nc = prefix_counts(packed, n_bases, offs, k, n_pos)
    t2 = time.perf_counter()
    if budget is None:
        most = max(int(ec.sum()), int(nc.sum()), 1)
        budget = max(-(-most // max(1, n_slices or 1)), int(ec.max()), int(nc.max()), 1)
    budget = int(budget)
    slices = plan_slices(ec, nc, budget)
    lib = api.load()
    nbytes = int(lib.dbg_slice_workspace_bytes(offs.numel() - 1, n_pos, budget, k))
    if nbytes == 0:
        raise api.DbgError(2, "dbg_slice_workspace_bytes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    outs = [api.alloc_outputs(k, budget, budget, device, zkey) for _ in range(2)]
    results = [torch.zeros(3, dtype=torch.int64, device=device) for _ in range(2)]
    res_host = [torch.zeros(3, dtype=torch.int64, pin_memory=True) for _ in range(2)]
    compute = torch.cuda.current_stream()
    copy = torch.cuda.Stream()
    built = [torch.cuda.Event() for _ in range(2)]
    copied = [None, None]
    parts, rows = [], []

    def enqueue(i):
        j = i % 2
        if copied[j] is not None:
            compute.wait_event(copied[j])  # the rows of slice i - 2 have left this set
        lo, hi = slices[i]
        build_slice_async(packed, n_bases, offs, k, n_pos, budget, lo, hi, outs[j], budget,
                          budget, results[j], ws, compute)
        with torch.cuda.stream(compute):
            res_host[j].copy_(results[j], non_blocking=True)
        built[j].record(compute)

    enqueue(0)
    for i in range(len(slices)):
        j = i % 2
        if i + 1 < len(slices):
            enqueue(i + 1)
        built[j].synchronize()  # slice i is done (slice i + 1 may be running)
        r = res_host[j].numpy().view(np.uint64)
        n_nodes, n_edges, status = int(r[0]), int(r[1]), int(r[2] & np.uint64(0xFFFFFFFF))
        if status:
            lo, hi = slices[i]
            raise api.DbgError(status, f"dbg_build_slice [{lo}, {hi}) (device)")
        copy.wait_event(built[j])
        parts.append(_host_rows(outs[j], n_nodes, n_edges, copy))
        ev = torch.cuda.Event()
        ev.record(copy)
        copied[j] = ev
        rows.append((n_nodes, n_edges))
    copy.synchronize()
    t3 = time.perf_counter()
    tables = _numpy_tables(k, parts) if concatenate else {}
    t4 = time.perf_counter()
    return SlicedTables(k, tables, slices, rows, parts, budget, nbytes,
                        {"upload": t1 - t0, "prefix_counts": t2 - t1, "slices": t3 - t2,
                         "concatenate": t4 - t3})
