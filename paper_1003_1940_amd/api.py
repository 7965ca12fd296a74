"""Python binding of ``libdbg.so``: argument marshalling only.

Every step of the construction runs in the library's HIP kernels; PyTorch only
provides device memory and streams.  There is no CPU fallback: if the library
is missing or no GPU is present these functions raise.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdbg.so")

DBG_OK, DBG_E_CAPACITY, DBG_E_SCRATCH = 0, 5, 11
_STATUS_NAMES = {0: "DBG_OK", 1: "DBG_E_NULL", 2: "DBG_E_K", 3: "DBG_E_OFFSETS",
                 4: "DBG_E_OVERFLOW", 5: "DBG_E_CAPACITY", 6: "DBG_E_WORKSPACE", 7: "DBG_E_HIP",
                 8: "DBG_E_BASE", 9: "DBG_E_ARG", 10: "DBG_E_INTERNAL", 11: "DBG_E_SCRATCH"}

# workspace held by the library for dbg_build_noalloc (DBG_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


class DbgError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {_STATUS_NAMES.get(code, code)} ({strerror(code)})")


class _Nodes(ctypes.Structure):
    _fields_ = [("kmer", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("capacity", ctypes.c_uint64)]


class _Edges(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("v", ctypes.c_void_p), ("orient", ctypes.c_void_p),
                ("mult", ctypes.c_void_p), ("zkey", ctypes.c_void_p),
                ("capacity", ctypes.c_uint64)]


class _Tuning(ctypes.Structure):
    _fields_ = [("node_path", ctypes.c_int), ("endpoint_ratio", ctypes.c_float),
                ("local_variant", ctypes.c_int), ("lds_digit_bias", ctypes.c_int),
                ("in_tile", ctypes.c_int), ("reserved", ctypes.c_int * 3)]


class _Chains(ctypes.Structure):
    _fields_ = [("node_chain", ctypes.c_void_p), ("node_rank", ctypes.c_void_p),
                ("node_orient", ctypes.c_void_p), ("chain_head", ctypes.c_void_p),
                ("chain_len", ctypes.c_void_p), ("chain_cyclic", ctypes.c_void_p),
                ("label_offsets", ctypes.c_void_p), ("labels", ctypes.c_void_p),
                ("label_capacity", ctypes.c_uint64), ("kept_row", ctypes.c_void_p),
                ("kept_u", ctypes.c_void_p), ("kept_v", ctypes.c_void_p),
                ("kept_orient", ctypes.c_void_p)]


TUNING_FIELDS = ("node_path", "endpoint_ratio", "local_variant", "lds_digit_bias", "in_tile")


NODES_AUTO, NODES_KMERS, NODES_ENDPOINTS = -1, 0, 1

_lib = None


def load():
    """Load libdbg.so (built by ``paper_1003_1940_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1003_1940_amd.hipbuild.build()")
        lib = ctypes.CDLL(LIB_PATH)
        u64, i32, vp, sz = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
        lib.dbg_workspace_bytes.restype = sz
        lib.dbg_workspace_bytes.argtypes = [u64, u64, u64, i32]
        lib.dbg_build.restype = i32
        lib.dbg_build.argtypes = [vp, u64, vp, u64, i32, u64, ctypes.POINTER(_Nodes),
                                  ctypes.POINTER(_Edges), vp, vp, sz, vp]
        lib.dbg_build_noalloc.restype = i32
        lib.dbg_build_noalloc.argtypes = [vp, u64, vp, u64, i32, u64, ctypes.POINTER(_Nodes),
                                          ctypes.POINTER(_Edges), vp, vp]
        lib.dbg_build_batched.restype = i32
        lib.dbg_build_batched.argtypes = [vp, u64, vp, u64, vp, u64, i32, u64,
                                          ctypes.POINTER(_Nodes), ctypes.POINTER(_Edges), vp, vp,
                                          vp, vp, sz, vp]
        lib.dbg_pack_ascii.restype = i32
        lib.dbg_pack_ascii.argtypes = [vp, u64, vp, vp, vp]
        lib.dbg_set_tuning.restype = i32
        lib.dbg_set_tuning.argtypes = [ctypes.POINTER(_Tuning)]
        lib.dbg_get_tuning.restype = i32
        lib.dbg_get_tuning.argtypes = [ctypes.POINTER(_Tuning)]
        lib.dbg_adjacency_workspace_bytes.restype = sz
        lib.dbg_adjacency_workspace_bytes.argtypes = [u64, u64, i32]
        lib.dbg_adjacency.restype = i32
        lib.dbg_adjacency.argtypes = [vp, u64, vp, vp, vp, u64, i32, vp, vp, vp, vp, vp, vp, sz,
                                      vp]
        lib.dbg_bounds.restype = i32
        lib.dbg_bounds.argtypes = [vp, u64, i32, vp, vp]
        lib.dbg_prefix_workspace_bytes.restype = sz
        lib.dbg_prefix_workspace_bytes.argtypes = [u64, u64, i32]
        lib.dbg_prefix_counts.restype = i32
        lib.dbg_prefix_counts.argtypes = [vp, u64, vp, u64, i32, u64, vp, vp, vp, vp, sz, vp]
        lib.dbg_slice_workspace_bytes.restype = sz
        lib.dbg_slice_workspace_bytes.argtypes = [u64, u64, u64, i32]
        lib.dbg_build_slice.restype = i32
        lib.dbg_build_slice.argtypes = [vp, u64, vp, u64, i32, u64, u64, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.POINTER(_Nodes),
                                        ctypes.POINTER(_Edges), vp, vp, sz, vp]
        lib.dbg_compact_workspace_bytes.restype = sz
        lib.dbg_compact_workspace_bytes.argtypes = [u64, u64]
        lib.dbg_compact.restype = i32
        lib.dbg_compact.argtypes = [vp, u64, u64, i32, vp, vp, vp, vp, ctypes.c_uint32,
                                    ctypes.POINTER(_Chains), vp, vp, sz, vp]
        lib.dbg_strerror.restype = ctypes.c_char_p
        lib.dbg_strerror.argtypes = [i32]
        _lib = lib
    return _lib


def get_tuning() -> dict:
    """The process-wide build tuning: node_path (NODES_AUTO, NODES_KMERS or
    NODES_ENDPOINTS), endpoint_ratio, local_variant (0, 1 or 2), lds_digit_bias
    and in_tile (0 or 1)."""
    t = _Tuning()
    rc = load().dbg_get_tuning(ctypes.byref(t))
    if rc:
        raise DbgError(rc, "dbg_get_tuning")
    return {"node_path": t.node_path, "endpoint_ratio": round(float(t.endpoint_ratio), 6),
            "local_variant": t.local_variant, "lds_digit_bias": t.lds_digit_bias,
            "in_tile": t.in_tile}


def set_tuning(node_path: int | None = None, endpoint_ratio: float | None = None,
               local_variant: int | None = None, lds_digit_bias: int | None = None,
               in_tile: int | None = None, defaults: bool = False) -> dict:
    """Change the process-wide tuning (unnamed fields keep their values;
    ``defaults=True`` first restores the library defaults).  Returns the new
    tuning.  Every setting gives identical tables."""
    lib = load()
    if defaults:
        rc = lib.dbg_set_tuning(None)
        if rc:
            raise DbgError(rc, "dbg_set_tuning")
    cur = get_tuning()
    new = dict(node_path=node_path, endpoint_ratio=endpoint_ratio, local_variant=local_variant,
               lds_digit_bias=lds_digit_bias, in_tile=in_tile)
    for f in TUNING_FIELDS:
        if new[f] is None:
            new[f] = cur[f]
    t = _Tuning(int(new["node_path"]), float(new["endpoint_ratio"]), int(new["local_variant"]),
                int(new["lds_digit_bias"]), int(new["in_tile"]))
    rc = lib.dbg_set_tuning(ctypes.byref(t))
    if rc:
        raise DbgError(rc, "dbg_set_tuning")
    return get_tuning()


def strerror(code: int) -> str:
    return load().dbg_strerror(code).decode()


def workspace_bytes(n_reads: int, n_sets: int, max_keys: int, k: int) -> int:
    return int(load().dbg_workspace_bytes(n_reads, n_sets, max_keys, k))


def key_words(k: int) -> int:
    """uint64 words per key: 1 for k <= 31, 2 for k >= 33."""
    return 1 if k <= 31 else 2


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_dev(t, name, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")


def pack(ascii_bases: torch.Tensor, stream=None):
    """ASCII bases (uint8 device tensor) -> 2-bit packed words (int64 device tensor
    holding the uint64 bit patterns) and a device result record whose status
    turns DBG_E_BASE on a byte outside ACGT/acgt."""
    _check_dev(ascii_bases, "ascii_bases", torch.uint8)
    n = ascii_bases.numel()
    packed = torch.empty(max(1, (n + 31) // 32), dtype=torch.int64, device=ascii_bases.device)
    res = torch.zeros(3, dtype=torch.int64, device=ascii_bases.device)
    rc = load().dbg_pack_ascii(_ptr(ascii_bases), n, _ptr(packed), _ptr(res), _stream(stream))
    if rc:
        raise DbgError(rc, "dbg_pack_ascii")
    return packed, res


@dataclass
class Graph:
    """Device-resident result.  Keys are int64 tensors holding uint64 bit
    patterns: shape (n,) for k <= 31, (n, 2) as (lo, hi) for k >= 33."""
    k: int
    node_kmer: torch.Tensor
    node_count: torch.Tensor
    edge_u: torch.Tensor
    edge_v: torch.Tensor
    edge_orient: torch.Tensor
    edge_mult: torch.Tensor
    edge_zkey: torch.Tensor | None
    n_nodes: int = 0
    n_edges: int = 0
    status: int = 0
    node_set_offsets: torch.Tensor | None = None
    edge_set_offsets: torch.Tensor | None = None
    extra: dict = field(default_factory=dict)

    def to_numpy(self):
        """Host copy with keys as (n, 2) uint64 (lo, hi) arrays."""
        def keys(t, n):
            a = t[:n].cpu().numpy().view(np.uint64)
            if a.ndim == 1:
                a = np.stack([a, np.zeros_like(a)], axis=1)
            return a
        nn_, ne = min(self.n_nodes, self.node_count.numel()), min(self.n_edges,
                                                                  self.edge_mult.numel())
        return dict(
            node_key=keys(self.node_kmer, nn_),
            node_count=self.node_count[:nn_].cpu().numpy().view(np.uint32).astype(np.uint64),
            edge_u=keys(self.edge_u, ne), edge_v=keys(self.edge_v, ne),
            edge_orient=self.edge_orient[:ne].cpu().numpy(),
            edge_mult=self.edge_mult[:ne].cpu().numpy().view(np.uint32).astype(np.uint64),
            edge_z=keys(self.edge_zkey, ne) if self.edge_zkey is not None else None)


class Workspace:
    """A reusable device workspace (a byte tensor) sized for a bound."""

    def __init__(self, n_reads: int, n_sets: int, max_keys: int, k: int, device="cuda"):
        self.nbytes = workspace_bytes(n_reads, n_sets, max_keys, k)
        if self.nbytes == 0:
            raise DbgError(2, "dbg_workspace_bytes")
        # 256-byte alignment: torch's caching allocator aligns blocks to 512 bytes
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        assert self.buf.data_ptr() % 256 == 0
        self.bound = (n_reads, n_sets, max_keys, k)


def alloc_outputs(k: int, node_cap: int, edge_cap: int, device="cuda", zkey: bool = True):
    w = key_words(k)
    shape = (lambda n: (n,)) if w == 1 else (lambda n: (n, 2))
    o = dict(
        node_kmer=torch.empty(shape(max(node_cap, 1)), dtype=torch.int64, device=device),
        node_count=torch.empty(max(node_cap, 1), dtype=torch.int32, device=device),
        edge_u=torch.empty(shape(max(edge_cap, 1)), dtype=torch.int64, device=device),
        edge_v=torch.empty(shape(max(edge_cap, 1)), dtype=torch.int64, device=device),
        edge_orient=torch.empty(max(edge_cap, 1), dtype=torch.uint8, device=device),
        edge_mult=torch.empty(max(edge_cap, 1), dtype=torch.int32, device=device),
        edge_zkey=torch.empty(shape(max(edge_cap, 1)), dtype=torch.int64, device=device)
        if zkey else None)
    return o


def _structs(out, node_cap, edge_cap):
    nodes = _Nodes(out["node_kmer"].data_ptr(), out["node_count"].data_ptr(), node_cap)
    edges = _Edges(out["edge_u"].data_ptr(), out["edge_v"].data_ptr(),
                   out["edge_orient"].data_ptr(), out["edge_mult"].data_ptr(),
                   out["edge_zkey"].data_ptr() if out["edge_zkey"] is not None else None, edge_cap)
    return nodes, edges


def build_async(packed, n_bases: int, offsets, k: int, max_keys: int, out: dict,
                node_cap: int, edge_cap: int, result, workspace: Workspace, stream=None,
                set_offsets=None, node_set_offsets=None, edge_set_offsets=None):
    """Enqueue one build (plain, or batched when ``set_offsets`` is given) on the
    stream without synchronising.  All tensors must be resident on the device."""
    _check_dev(packed, "packed", torch.int64)
    _check_dev(offsets, "offsets", torch.int64)
    _check_dev(result, "result", torch.int64)
    n_reads = offsets.numel() - 1
    nodes, edges = _structs(out, node_cap, edge_cap)
    lib = load()
    if set_offsets is None:
        rc = lib.dbg_build(_ptr(packed), n_bases, _ptr(offsets), n_reads, k, max_keys,
                           ctypes.byref(nodes), ctypes.byref(edges), _ptr(result),
                           _ptr(workspace.buf), workspace.nbytes, _stream(stream))
        where = "dbg_build"
    else:
        _check_dev(set_offsets, "set_offsets", torch.int64)
        rc = lib.dbg_build_batched(_ptr(packed), n_bases, _ptr(offsets), n_reads,
                                   _ptr(set_offsets), set_offsets.numel() - 1, k, max_keys,
                                   ctypes.byref(nodes), ctypes.byref(edges),
                                   _ptr(node_set_offsets), _ptr(edge_set_offsets), _ptr(result),
                                   _ptr(workspace.buf), workspace.nbytes, _stream(stream))
        where = "dbg_build_batched"
    if rc:
        raise DbgError(rc, where)


def build_noalloc_async(packed, n_bases: int, offsets, k: int, max_keys: int, out: dict,
                        node_cap: int, edge_cap: int, result, stream=None):
    """Enqueue one build through dbg_build_noalloc: no workspace argument, the
    library's static per-device scratch is used (builds needing more than
    NOALLOC_SCRATCH_BYTES raise DBG_E_SCRATCH; calls overlapping on one device
    race).  All tensors must be resident on the device."""
    _check_dev(packed, "packed", torch.int64)
    _check_dev(offsets, "offsets", torch.int64)
    _check_dev(result, "result", torch.int64)
    nodes, edges = _structs(out, node_cap, edge_cap)
    rc = load().dbg_build_noalloc(_ptr(packed), n_bases, _ptr(offsets), offsets.numel() - 1, k,
                                  max_keys, ctypes.byref(nodes), ctypes.byref(edges),
                                  _ptr(result), _stream(stream))
    if rc:
        raise DbgError(rc, "dbg_build_noalloc")


def bounds(offsets: np.ndarray, k: int) -> tuple:
    """(max_nodes, max_edges): the exact worst-case table sizes of reads given by
    host offsets (dbg_bounds)."""
    off = np.ascontiguousarray(offsets, np.uint64)
    if len(off) == 0:
        raise ValueError("offsets need at least one entry")
    mn, me = ctypes.c_uint64(0), ctypes.c_uint64(0)
    rc = load().dbg_bounds(off.ctypes.data, len(off) - 1, k, ctypes.byref(mn), ctypes.byref(me))
    if rc:
        raise DbgError(rc, "dbg_bounds")
    return int(mn.value), int(me.value)


def read_result(result) -> tuple:
    """(n_nodes, n_edges, status) from a device result record (synchronises)."""
    r = result.cpu().numpy().view(np.uint64)
    return int(r[0]), int(r[1]), int(r[2] & 0xFFFFFFFF)


FLAG_NODES_FROM_ENDPOINTS = 1


def read_flags(result) -> int:
    """DBG_FLAG_* bits of a device result record (synchronises)."""
    r = result.cpu().numpy().view(np.uint64)
    return int(r[2] >> np.uint64(32))


def upload(bases: np.ndarray, offsets: np.ndarray, device="cuda", stream=None):
    """ASCII reads (host) -> (packed words, device offsets, n_bases); packing runs
    on the device."""
    n_bases = int(offsets[-1])
    ascii_d = torch.from_numpy(np.ascontiguousarray(bases[:n_bases], np.uint8)).to(device)
    if ascii_d.numel() == 0:
        ascii_d = torch.zeros(1, dtype=torch.uint8, device=device)[:0]
    packed, res = pack(ascii_d, stream) if n_bases else (
        torch.zeros(1, dtype=torch.int64, device=device), None)
    offs = torch.from_numpy(np.ascontiguousarray(offsets, np.uint64).view(np.int64)).to(device)
    if res is not None:
        _, _, st = read_result(res)
        if st:
            raise DbgError(st, "dbg_pack_ascii")
    return packed, offs, n_bases


def build(bases: np.ndarray, offsets: np.ndarray, k: int, zkey: bool = True, device="cuda",
          node_cap: int | None = None, edge_cap: int | None = None,
          max_keys: int | None = None) -> Graph:
    """Convenience: upload host reads, build, synchronise, return the device graph
    sliced to its true sizes.  ``max_keys`` (at least the number of k-mer
    positions, the default) sizes the workspace."""
    offsets = np.asarray(offsets, np.uint64)
    n_k, _ = bounds(offsets, k)
    max_keys = n_k if max_keys is None else max(int(max_keys), n_k)
    packed, offs, n_bases = upload(bases, offsets, device)
    node_cap = n_k if node_cap is None else node_cap
    edge_cap = n_k if edge_cap is None else edge_cap
    out = alloc_outputs(k, node_cap, edge_cap, device, zkey)
    ws = Workspace(len(offsets) - 1, 1, max_keys, k, device)
    result = torch.zeros(3, dtype=torch.int64, device=device)
    build_async(packed, n_bases, offs, k, max_keys, out, node_cap, edge_cap, result, ws)
    n_nodes, n_edges, status = read_result(result)
    if status not in (DBG_OK, DBG_E_CAPACITY):
        raise DbgError(status, "dbg_build (device)")
    g = Graph(k, out["node_kmer"], out["node_count"], out["edge_u"], out["edge_v"],
              out["edge_orient"], out["edge_mult"], out["edge_zkey"], n_nodes, n_edges, status)
    g.extra["flags"] = read_flags(result)
    return g


def build_batched(bases: np.ndarray, offsets: np.ndarray, set_read_offsets: np.ndarray, k: int,
                  zkey: bool = True, device="cuda") -> Graph:
    """Convenience: several read sets (set s = reads [set_read_offsets[s],
    set_read_offsets[s+1])) built in one launch sequence; outputs concatenated
    per set with row offsets in node_set_offsets / edge_set_offsets."""
    offsets = np.asarray(offsets, np.uint64)
    sro = np.asarray(set_read_offsets, np.uint64)
    n_k, _ = bounds(offsets, k)
    packed, offs, n_bases = upload(bases, offsets, device)
    out = alloc_outputs(k, n_k, n_k, device, zkey)
    n_sets = len(sro) - 1
    ws = Workspace(len(offsets) - 1, n_sets, n_k, k, device)
    result = torch.zeros(3, dtype=torch.int64, device=device)
    sets_d = torch.from_numpy(sro.view(np.int64).copy()).to(device)
    nso = torch.zeros(n_sets + 1, dtype=torch.int64, device=device)
    eso = torch.zeros(n_sets + 1, dtype=torch.int64, device=device)
    build_async(packed, n_bases, offs, k, n_k, out, n_k, n_k, result, ws, set_offsets=sets_d,
                node_set_offsets=nso, edge_set_offsets=eso)
    n_nodes, n_edges, status = read_result(result)
    if status not in (DBG_OK, DBG_E_CAPACITY):
        raise DbgError(status, "dbg_build_batched (device)")
    return Graph(k, out["node_kmer"], out["node_count"], out["edge_u"], out["edge_v"],
                 out["edge_orient"], out["edge_mult"], out["edge_zkey"], n_nodes, n_edges, status,
                 node_set_offsets=nso, edge_set_offsets=eso)


class CapturedBuild:
    """A build (plain or batched) recorded once into a HIP graph and replayed.

    The library enqueues only kernels and never synchronises or reads device
    values on the host (grid sizes come from the bounds), so the whole launch
    sequence of one build can be captured on a stream.  The graph keeps the
    buffers it was captured with: to build other reads, copy them into
    ``packed`` / ``offsets`` (same number of bases and reads; for a batched build
    the same number of sets, new set offsets into ``set_offsets``) and replay.
    Outputs land in ``out`` and ``result`` as for ``build_async``."""

    def __init__(self, packed, n_bases: int, offsets, k: int, max_keys: int,
                 set_offsets=None, zkey: bool = True, device="cuda"):
        self.packed, self.offsets, self.set_offsets = packed, offsets, set_offsets
        self.n_bases, self.k, self.max_keys = n_bases, k, max_keys
        n_reads = offsets.numel() - 1
        n_sets = 1 if set_offsets is None else set_offsets.numel() - 1
        self.out = alloc_outputs(k, max_keys, max_keys, device, zkey)
        self.ws = Workspace(n_reads, n_sets, max_keys, k, device)
        self.result = torch.zeros(3, dtype=torch.int64, device=device)
        self.node_set_offsets = self.edge_set_offsets = None
        if set_offsets is not None:
            self.node_set_offsets = torch.zeros(n_sets + 1, dtype=torch.int64, device=device)
            self.edge_set_offsets = torch.zeros(n_sets + 1, dtype=torch.int64, device=device)
        self.graph = torch.cuda.CUDAGraph()
        self._enqueue()  # one eager build first: every kernel is loaded before capture
        torch.cuda.synchronize()
        with torch.cuda.graph(self.graph):
            self._enqueue()
        torch.cuda.synchronize()

    def _enqueue(self):
        build_async(self.packed, self.n_bases, self.offsets, self.k, self.max_keys, self.out,
                    self.max_keys, self.max_keys, self.result, self.ws,
                    set_offsets=self.set_offsets, node_set_offsets=self.node_set_offsets,
                    edge_set_offsets=self.edge_set_offsets)

    def replay(self):
        """Enqueue one replay on the current stream (no synchronisation)."""
        self.graph.replay()

    def graph_result(self) -> Graph:
        """The last replay's tables (synchronises)."""
        n_nodes, n_edges, status = read_result(self.result)
        o = self.out
        g = Graph(self.k, o["node_kmer"], o["node_count"], o["edge_u"], o["edge_v"],
                  o["edge_orient"], o["edge_mult"], o["edge_zkey"], n_nodes, n_edges, status,
                  node_set_offsets=self.node_set_offsets, edge_set_offsets=self.edge_set_offsets)
        g.extra["flags"] = read_flags(self.result)
        return g


@dataclass
class Adjacency:
    """STEP-4 adjacency lists as a CSR over buckets b = 2 * node + side (side 0:
    left by a walk reading the canonical k-mer forward, side 1: entered by it):
    entries offsets[b] .. offsets[b+1] of (edge row, end), end 0 = the u end.
    ``edge_bucket`` holds the buckets of both ends of every edge."""
    offsets: torch.Tensor    # int64, 2 n_nodes + 1
    inc_edge: torch.Tensor   # int32 holding uint32 edge rows, 2 n_edges
    inc_end: torch.Tensor    # uint8, 2 n_edges
    edge_bucket: torch.Tensor | None = None  # int32 holding uint32 buckets, 2 n_edges

    def to_numpy(self):
        return (self.offsets.cpu().numpy().view(np.uint64),
                self.inc_edge.cpu().numpy().view(np.uint32).astype(np.uint64),
                self.inc_end.cpu().numpy())


def adjacency_async(g: Graph, stream=None, result=None, workspace=None,
                    edge_buckets: bool = False) -> Adjacency:
    """Enqueue the adjacency lists of a built graph (its true row counts must be
    known on the host: ``g.n_nodes`` / ``g.n_edges``); ``edge_buckets`` also
    returns the bucket (2 * node + side) of every edge's ends."""
    n, m = int(g.n_nodes), int(g.n_edges)
    dev = g.node_kmer.device
    offsets = torch.empty(2 * n + 1, dtype=torch.int64, device=dev)
    inc_edge = torch.empty(max(1, 2 * m), dtype=torch.int32, device=dev)
    inc_end = torch.empty(max(1, 2 * m), dtype=torch.uint8, device=dev)
    enode = torch.empty(max(1, 2 * m), dtype=torch.int32, device=dev) if edge_buckets else None
    lib = load()
    nbytes = int(lib.dbg_adjacency_workspace_bytes(n, m, g.k))
    if nbytes == 0:
        raise DbgError(2, "dbg_adjacency_workspace_bytes")
    ws = workspace if workspace is not None else torch.empty(nbytes, dtype=torch.uint8,
                                                              device=dev)
    res = result if result is not None else torch.zeros(3, dtype=torch.int64, device=dev)
    rc = lib.dbg_adjacency(_ptr(g.node_kmer), n, _ptr(g.edge_u), _ptr(g.edge_v),
                           _ptr(g.edge_orient), m, g.k, _ptr(offsets), _ptr(inc_edge),
                           _ptr(inc_end), _ptr(enode) if enode is not None else None, _ptr(res),
                           _ptr(ws), ws.numel(), _stream(stream))
    if rc:
        raise DbgError(rc, "dbg_adjacency")
    a = Adjacency(offsets, inc_edge[:2 * m], inc_end[:2 * m],
                  enode[:2 * m] if enode is not None else None)
    a.result = res
    return a


def adjacency(g: Graph, edge_buckets: bool = False) -> Adjacency:
    """Adjacency lists of a built graph (synchronises; raises on a device error)."""
    a = adjacency_async(g, edge_buckets=edge_buckets)
    _, _, status = read_result(a.result)
    if status:
        raise DbgError(status, "dbg_adjacency (device)")
    return a


@dataclass
class Chains:
    """Simplified graph (Sec. 7 chain compaction) on the device; uint32 values
    are held in int32 tensors.  Chain c spells
    labels[label_offsets[c]:label_offsets[c + 1]] (ASCII)."""
    node_chain: torch.Tensor    # n_nodes
    node_rank: torch.Tensor     # n_nodes
    node_orient: torch.Tensor   # n_nodes, uint8
    chain_head: torch.Tensor    # n_chains
    chain_len: torch.Tensor     # n_chains
    chain_cyclic: torch.Tensor  # n_chains, uint8
    label_offsets: torch.Tensor  # n_chains + 1, int64
    labels: torch.Tensor        # label_len, uint8
    kept_row: torch.Tensor      # n_kept
    kept_u: torch.Tensor
    kept_v: torch.Tensor
    kept_orient: torch.Tensor   # uint8
    n_chains: int = -1
    n_kept: int = -1
    label_len: int = -1
    n_cyclic: int = -1
    result: torch.Tensor | None = None
    _full: dict = field(default_factory=dict)

    def finish(self):
        """Read the result record (synchronises) and trim the tables; raises on
        a device error."""
        r = self.result.cpu().numpy().view(np.uint64)
        status = int(r[4] & 0xFFFFFFFF)
        if status:
            raise DbgError(status, "dbg_compact (device)")
        self.n_chains, self.n_kept, self.label_len, self.n_cyclic = (int(x) for x in r[:4])
        f = self._full
        self.chain_head = f["chain_head"][:self.n_chains]
        self.chain_len = f["chain_len"][:self.n_chains]
        self.chain_cyclic = f["chain_cyclic"][:self.n_chains]
        self.label_offsets = f["label_offsets"][:self.n_chains + 1]
        self.labels = f["labels"][:self.label_len]
        self.kept_row = f["kept_row"][:self.n_kept]
        self.kept_u = f["kept_u"][:self.n_kept]
        self.kept_v = f["kept_v"][:self.n_kept]
        self.kept_orient = f["kept_orient"][:self.n_kept]
        return self

    def label(self, c: int) -> str:
        off = self.label_offsets
        return bytes(self.labels[int(off[c]):int(off[c + 1])].cpu().numpy()).decode()


def alloc_chains(n: int, m: int, k: int, device="cuda", label_capacity: int | None = None):
    """Output buffers of dbg_compact for a graph of n nodes and m edges."""
    i32, u8 = torch.int32, torch.uint8
    cap = n * k if label_capacity is None else int(label_capacity)
    z = lambda cnt, dt: torch.empty(max(1, cnt), dtype=dt, device=device)
    return {"node_chain": z(n, i32), "node_rank": z(n, i32), "node_orient": z(n, u8),
            "chain_head": z(n, i32), "chain_len": z(n, i32), "chain_cyclic": z(n, u8),
            "label_offsets": z(n + 1, torch.int64), "labels": z(cap, u8),
            "kept_row": z(m, i32), "kept_u": z(m, i32), "kept_v": z(m, i32),
            "kept_orient": z(m, u8)}


def compact_async(g: Graph, adj: Adjacency, min_nodes: int = 3, stream=None, out=None,
                  workspace=None, result=None, label_capacity: int | None = None) -> Chains:
    """Enqueue the chain compaction of a built graph from its adjacency lists
    (``adj`` must hold ``edge_bucket``: ``adjacency(g, edge_buckets=True)``)."""
    n, m = int(g.n_nodes), int(g.n_edges)
    if adj.edge_bucket is None and m:
        raise ValueError("the adjacency lists need edge_bucket (adjacency(g, edge_buckets=True))")
    dev = g.node_kmer.device
    out = out if out is not None else alloc_chains(n, m, g.k, dev, label_capacity)
    lib = load()
    nbytes = int(lib.dbg_compact_workspace_bytes(n, m))
    ws = workspace if workspace is not None else torch.empty(nbytes, dtype=torch.uint8,
                                                              device=dev)
    res = result if result is not None else torch.zeros(5, dtype=torch.int64, device=dev)
    st = _Chains(*[out[f].data_ptr() if f != "label_capacity" else out["labels"].numel()
                   for f, _ in _Chains._fields_])
    rc = lib.dbg_compact(_ptr(g.node_kmer), n, m, g.k, _ptr(adj.offsets),
                         _ptr(adj.inc_edge), _ptr(adj.inc_end),
                         _ptr(adj.edge_bucket) if adj.edge_bucket is not None else None,
                         int(min_nodes), ctypes.byref(st), _ptr(res), _ptr(ws), ws.numel(),
                         _stream(stream))
    if rc:
        raise DbgError(rc, "dbg_compact")
    c = Chains(out["node_chain"][:n], out["node_rank"][:n], out["node_orient"][:n],
               out["chain_head"], out["chain_len"], out["chain_cyclic"], out["label_offsets"],
               out["labels"], out["kept_row"], out["kept_u"], out["kept_v"], out["kept_orient"],
               result=res, _full=out)
    c.workspace = ws
    return c


def compact(g: Graph, adj: Adjacency | None = None, min_nodes: int = 3) -> Chains:
    """Chain compaction of a built graph (synchronises; raises on a device error)."""
    adj = adj if adj is not None else adjacency(g, edge_buckets=True)
    return compact_async(g, adj, min_nodes).finish()
