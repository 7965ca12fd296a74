"""TEST INFRASTRUCTURE ONLY -- the oracle.

A plain CPU construction of the bi-directed de Bruijn graph (nodes with counts,
canonical bi-directed edges with multiplicities), written from the definitions of
Sec. 2 and steps STEP-1 to STEP-3 of algorithm BiConstruct (Sec. 3) of Kundeti et
al.  The arithmetic lives in ``dbg_oracle.cpp`` (std::string k-mers, std::map
counts); this module compiles it with g++ and marshals arguments with ctypes.

Only ``tests/``, the smoke entry point and the CPU-baseline leg of ``bench.py``
may import this package.  It shares no code with the GPU library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dbg_oracle.cpp")
# DBG_ORACLE_LIB names another build of the same source to load instead (the
# sanitizer build, in the test that runs the pins under it)
_LIB = os.environ.get("DBG_ORACLE_LIB") or os.path.join(_HERE, "libdbg_oracle.so")
_LIB_ASAN = os.path.join(_HERE, "libdbg_oracle_asan.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle into ``oracle/libdbg_oracle.so`` (g++ -O2, C++17), or
    with ``sanitize`` into ``oracle/libdbg_oracle_asan.so`` with AddressSanitizer
    and UndefinedBehaviorSanitizer (any report aborts)."""
    out = _LIB_ASAN if sanitize else _LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        extra = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all"] if sanitize else ["-O2"])
        subprocess.run(["g++", *extra, "-std=c++17", "-fPIC", "-shared", "-pthread",
                        "-Wall", "-Wextra", "-o", tmp, _SRC], check=True)
        os.replace(tmp, out)
    return out


def _load(path: str | None = None):
    """Load the oracle library (default: the built one; ``path`` loads another
    build of the same source, e.g. a deliberately broken copy in a test)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    lib.oracle_build.restype = ctypes.c_void_p
    lib.oracle_build.argtypes = [ctypes.c_char_p, _u64p, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_int]
    for name in ("oracle_n_nodes", "oracle_n_edges"):
        getattr(lib, name).restype = ctypes.c_uint64
        getattr(lib, name).argtypes = [ctypes.c_void_p]
    lib.oracle_status.restype = ctypes.c_int
    lib.oracle_status.argtypes = [ctypes.c_void_p]
    lib.oracle_get_nodes.argtypes = [ctypes.c_void_p, _u64p, _u64p]
    lib.oracle_get_edges.argtypes = [ctypes.c_void_p, _u64p, _u64p, _u8p, _u64p, _u64p]
    lib.oracle_node_str.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_char_p]
    lib.oracle_edge_str.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_char_p,
                                    ctypes.c_char_p, ctypes.c_char_p]
    lib.oracle_free.argtypes = [ctypes.c_void_p]
    lib.oracle_revcomp.restype = ctypes.c_int
    lib.oracle_revcomp.argtypes = [ctypes.c_char_p, ctypes.c_uint64, ctypes.c_char_p]
    lib.oracle_probe.argtypes = [ctypes.c_char_p, _u64p, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_char_p, ctypes.c_uint64, _u64p,
                                 ctypes.c_char_p, ctypes.c_char_p, _u8p, ctypes.c_uint64,
                                 _u64p]
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_threads.argtypes = [ctypes.c_int]
    return lib


def _ptr(a: np.ndarray, typ):
    return a.ctypes.data_as(typ)


def _as_input(bases, offsets):
    b = np.ascontiguousarray(np.frombuffer(bytes(bases), dtype=np.uint8)
                             if isinstance(bases, (bytes, bytearray)) else bases, dtype=np.uint8)
    o = np.ascontiguousarray(offsets, dtype=np.uint64)
    return b, o


@dataclass
class OracleGraph:
    """Oracle output.  Keys are base-4 values (A0 C1 G2 T3, first base most
    significant) as (lo, hi) uint64 pairs, shape (n, 2)."""
    k: int
    node_key: np.ndarray     # (U_n, 2) uint64
    node_count: np.ndarray   # (U_n,) uint64
    edge_u: np.ndarray       # (U_e, 2) uint64
    edge_v: np.ndarray       # (U_e, 2) uint64
    edge_orient: np.ndarray  # (U_e,) uint8, (o1 << 1) | o2, '+' = 0
    edge_mult: np.ndarray    # (U_e,) uint64
    edge_z: np.ndarray       # (U_e, 2) uint64: canonical (k+1)-mer of the edge
    node_str: list | None = None
    edge_str: list | None = None  # (u, v, orient_string, z)


def build_graph(bases, offsets, k: int, threads: int = 0, strings: bool = False,
                lib_path: str | None = None) -> OracleGraph:
    """Run the oracle on reads ``bases[offsets[i]:offsets[i+1]]`` (ASCII ACGT)."""
    lib = _load(lib_path)
    b, o = _as_input(bases, offsets)
    n_reads = len(o) - 1
    h = lib.oracle_build(b.ctypes.data_as(ctypes.c_char_p), _ptr(o, _u64p), n_reads, k, threads)
    try:
        if lib.oracle_status(h) != 0:
            raise RuntimeError("oracle: two distinct edge records spell the same (k+1)-mer")
        nn, ne = lib.oracle_n_nodes(h), lib.oracle_n_edges(h)
        nk = np.zeros((nn, 2), np.uint64)
        nc = np.zeros(nn, np.uint64)
        lib.oracle_get_nodes(h, _ptr(nk, _u64p), _ptr(nc, _u64p))
        eu = np.zeros((ne, 2), np.uint64)
        ev = np.zeros((ne, 2), np.uint64)
        eo = np.zeros(ne, np.uint8)
        em = np.zeros(ne, np.uint64)
        ez = np.zeros((ne, 2), np.uint64)
        lib.oracle_get_edges(h, _ptr(eu, _u64p), _ptr(ev, _u64p), _ptr(eo, _u8p),
                             _ptr(em, _u64p), _ptr(ez, _u64p))
        g = OracleGraph(k, nk, nc, eu, ev, eo, em, ez)
        if strings:
            g.node_str, g.edge_str = [], []
            buf = ctypes.create_string_buffer(k + 2)
            for i in range(nn):
                lib.oracle_node_str(h, i, buf)
                g.node_str.append(buf.raw[:k].decode())
            ub, vb, zb = (ctypes.create_string_buffer(k + 2) for _ in range(3))
            for i in range(ne):
                lib.oracle_edge_str(h, i, ub, vb, zb)
                ori = "+-"[int(eo[i]) >> 1] + "+-"[int(eo[i]) & 1]
                g.edge_str.append((ub.raw[:k].decode(), vb.raw[:k].decode(), ori,
                                   zb.raw[:k + 1].decode()))
        return g
    finally:
        lib.oracle_free(h)


def revcomp(s: str, lib_path: str | None = None) -> str:
    lib = _load(lib_path)
    out = ctypes.create_string_buffer(len(s) + 1)
    if lib.oracle_revcomp(s.encode(), len(s), out) != 0:
        raise ValueError("not a DNA string over A, C, G, T")
    return out.raw[:len(s)].decode()


def probe_counts(bases, offsets, k: int, node_probes: list, edge_probes: list, threads: int = 0):
    """Count selected nodes and edges over all reads (see ``oracle_probe``).

    node_probes: list of k-character canonical strings.
    edge_probes: list of (u, v, orient) with u, v strings and orient = (o1 << 1) | o2.
    Returns (node_counts, edge_counts) as uint64 arrays.
    """
    lib = _load()
    b, o = _as_input(bases, offsets)
    n_reads = len(o) - 1
    npb = "".join(node_probes).encode()
    eu = "".join(e[0] for e in edge_probes).encode()
    ev = "".join(e[1] for e in edge_probes).encode()
    eo = np.array([e[2] for e in edge_probes], dtype=np.uint8)
    nc = np.zeros(len(node_probes), np.uint64)
    ec = np.zeros(len(edge_probes), np.uint64)
    lib.oracle_probe(b.ctypes.data_as(ctypes.c_char_p), _ptr(o, _u64p), n_reads, k, threads,
                     npb, len(node_probes), _ptr(nc, _u64p), eu, ev,
                     _ptr(eo if len(eo) else np.zeros(1, np.uint8), _u8p), len(edge_probes),
                     _ptr(ec, _u64p))
    return nc, ec


def host_threads(threads: int = 0) -> int:
    """Number of threads the oracle uses for ``threads`` (0 = every host core)."""
    return _load().oracle_threads(threads)
