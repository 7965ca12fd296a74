"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects bad arguments on the host before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dbg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dbg_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1003_1940_amd import api
    return api.load()


def test_header_declares_entry_points():
    assert declared_functions() == ["dbg_adjacency", "dbg_adjacency_workspace_bytes",
                                    "dbg_bounds", "dbg_build", "dbg_build_batched",
                                    "dbg_build_noalloc", "dbg_build_slice",
                                    "dbg_compact", "dbg_compact_workspace_bytes",
                                    "dbg_get_tuning", "dbg_pack_ascii", "dbg_prefix_counts",
                                    "dbg_prefix_workspace_bytes", "dbg_set_stage_events",
                                    "dbg_set_tuning", "dbg_slice_workspace_bytes",
                                    "dbg_strerror", "dbg_workspace_bytes"]


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror(lib):
    from paper_1003_1940_amd import api
    assert api.strerror(0) == "ok"
    assert "odd" in api.strerror(2)


def test_workspace_bytes(lib):
    from paper_1003_1940_amd import api
    assert api.workspace_bytes(10, 1, 1000, 31) > 0
    assert api.workspace_bytes(10, 1, 1000, 30) == 0   # even k
    assert api.workspace_bytes(10, 1, 1000, 65) == 0
    assert api.workspace_bytes(10, 0, 1000, 31) == 0   # no sets
    a = api.workspace_bytes(10, 1, 1000, 31)
    b = api.workspace_bytes(10, 1, 1000, 33)          # 128-bit keys
    assert b > a
    # 2M reads, 140M k-mer positions at k=31 fits in a few GB
    assert api.workspace_bytes(2_000_000, 1, 140_000_000, 31) < 4e9


def _call_build(lib, k=31, max_keys=100, ws_bytes=None, nodes_null=False, result_null=False,
                offsets_null=False):
    from paper_1003_1940_amd import api
    nodes = api._Nodes(0 if nodes_null else 16, 16, 10)
    edges = api._Edges(16, 16, 16, 16, None, 10)
    ws = ctypes.c_void_p(256)
    nbytes = api.workspace_bytes(1, 1, max_keys, 31) if ws_bytes is None else ws_bytes
    return lib.dbg_build(ctypes.c_void_p(16), 40, None if offsets_null else ctypes.c_void_p(16),
                         1, k, max_keys, ctypes.byref(nodes), ctypes.byref(edges),
                         None if result_null else ctypes.c_void_p(16), ws, nbytes, None)


def test_host_rejects_bad_arguments(lib):
    # Every case below is refused before any device work (dummy pointers are
    # never dereferenced).
    assert _call_build(lib, k=30) == 2         # DBG_E_K: even k
    assert _call_build(lib, k=0) == 2
    assert _call_build(lib, k=65) == 2
    assert _call_build(lib, nodes_null=True) == 1   # DBG_E_NULL
    assert _call_build(lib, result_null=True) == 1
    assert _call_build(lib, offsets_null=True) == 1
    assert _call_build(lib, max_keys=1 << 32) == 4  # DBG_E_OVERFLOW: counts are 32-bit
    assert _call_build(lib, ws_bytes=100) == 6      # DBG_E_WORKSPACE


def test_tuning_round_trip(lib):
    from paper_1003_1940_amd import api
    d = api.set_tuning(defaults=True)
    assert d == {"node_path": api.NODES_AUTO, "endpoint_ratio": pytest.approx(0.6),
                 "local_variant": 2, "lds_digit_bias": 0, "in_tile": 1}
    assert api.set_tuning(local_variant=1, lds_digit_bias=-2)["local_variant"] == 1
    assert api.set_tuning(in_tile=0)["in_tile"] == 0
    assert api.get_tuning()["lds_digit_bias"] == -2
    api.set_tuning(defaults=True)
    assert api.set_tuning(node_path=api.NODES_ENDPOINTS)["node_path"] == api.NODES_ENDPOINTS
    assert api.set_tuning(endpoint_ratio=0.25)["endpoint_ratio"] == pytest.approx(0.25)
    assert api.get_tuning()["node_path"] == api.NODES_ENDPOINTS  # unnamed field kept
    for bad in (dict(node_path=2), dict(node_path=-2), dict(endpoint_ratio=-0.1),
                dict(endpoint_ratio=3.0), dict(local_variant=3), dict(local_variant=-1),
                dict(lds_digit_bias=4), dict(lds_digit_bias=-4), dict(in_tile=2),
                dict(in_tile=-1)):
        with pytest.raises(api.DbgError):
            api.set_tuning(**bad)
    assert api.get_tuning()["endpoint_ratio"] == pytest.approx(0.25)  # refused: unchanged
    assert lib.dbg_get_tuning(None) == 1
    api.set_tuning(defaults=True)


def test_adjacency_host_checks(lib):
    v = ctypes.c_void_p(256)
    assert lib.dbg_adjacency_workspace_bytes(10, 20, 30) == 0        # even k
    assert lib.dbg_adjacency_workspace_bytes(10, 20, 31) > 0
    args = lambda **kw: dict(dict(nodes=v, n=10, u=v, vv=v, o=v, m=20, k=31, off=v, ie=v, ien=v,
                                  res=v, ws=v, wsb=1 << 30), **kw)
    def call(**kw):
        a = args(**kw)
        return lib.dbg_adjacency(a["nodes"], a["n"], a["u"], a["vv"], a["o"], a["m"], a["k"],
                                 a["off"], a["ie"], a["ien"], None, a["res"], a["ws"], a["wsb"],
                                 None)
    assert call(k=4) == 2                    # DBG_E_K
    assert call(off=None) == 1               # DBG_E_NULL
    assert call(u=None) == 1
    assert call(n=0) == 9                    # edges without nodes: DBG_E_ARG
    assert call(n=1 << 31) == 4              # DBG_E_OVERFLOW
    assert call(wsb=16) == 6                 # DBG_E_WORKSPACE
    assert call(ws=ctypes.c_void_p(257)) == 6


def test_compact_host_checks(lib):
    """dbg_compact's argument checks on the host (no device work is enqueued)."""
    from paper_1003_1940_amd import api
    assert lib.dbg_compact_workspace_bytes(10, 20) > 0
    assert lib.dbg_compact_workspace_bytes(0, 0) > 0
    v = 256
    full = api._Chains(*[v if f != "label_capacity" else 1000 for f, _ in api._Chains._fields_])
    no_labels = api._Chains(*[v if f not in ("labels", "label_capacity") else (0 if f == "labels"
                                                                               else 1000)
                              for f, _ in api._Chains._fields_])
    vp = ctypes.c_void_p(256)

    def call(n=10, m=20, k=31, out=full, ws=vp, wsb=1 << 30, enode=vp, res=vp):
        return lib.dbg_compact(vp, n, m, k, vp, vp, vp, enode, 3,
                               ctypes.byref(out) if out is not None else None, res, ws, wsb, None)
    assert call(k=4) == 2                     # DBG_E_K
    assert call(out=None) == 1                # DBG_E_NULL
    assert call(res=None) == 1
    assert call(out=no_labels) == 1           # labels needed with nodes
    assert call(enode=None) == 1              # edge_bucket needed with edges
    assert call(n=0) == 9                     # edges without nodes: DBG_E_ARG
    assert call(n=1 << 31) == 4               # DBG_E_OVERFLOW
    assert call(wsb=16) == 6                  # DBG_E_WORKSPACE
    assert call(ws=ctypes.c_void_p(257)) == 6


def test_slice_host_checks(lib):
    """dbg_build_slice / dbg_prefix_counts argument checks on the host."""
    from paper_1003_1940_amd import api
    v = ctypes.c_void_p(256)
    assert lib.dbg_slice_workspace_bytes(10, 1000, 100, 31) > 0
    assert lib.dbg_slice_workspace_bytes(10, 1000, 2000, 31) == 0   # max_keys > positions
    assert lib.dbg_slice_workspace_bytes(10, 1000, 100, 8) == 0     # even k
    # the slice workspace grows with its keys, not with the positions alone
    assert lib.dbg_slice_workspace_bytes(10, 10**8, 10**6, 31) < \
        lib.dbg_workspace_bytes(10, 1, 10**8, 31) / 4
    assert lib.dbg_prefix_workspace_bytes(10, 1000, 31) > 0
    nodes = api._Nodes(256, 256, 10)
    edges = api._Edges(256, 256, 256, 256, None, 10)

    def call(k=31, mp=1000, mk=100, lo=0, hi=4096, ws=v, wsb=1 << 30):
        return lib.dbg_build_slice(v, 100, v, 10, k, mp, mk, lo, hi, ctypes.byref(nodes),
                                   ctypes.byref(edges), v, ws, wsb, None)
    assert call(k=4) == 2                    # DBG_E_K
    assert call(mk=2000) == 9                # max_keys > max_positions: DBG_E_ARG
    assert call(lo=10, hi=5) == 9            # empty range reversed
    assert call(hi=4097) == 9                # past the last prefix
    assert call(mp=1 << 32) == 4             # DBG_E_OVERFLOW
    assert call(wsb=16) == 6                 # DBG_E_WORKSPACE
    assert call(ws=ctypes.c_void_p(257)) == 6

    def pc(k=31, mp=1000, ec=v, wsb=1 << 30):
        return lib.dbg_prefix_counts(v, 100, v, 10, k, mp, ec, v, v, v, wsb, None)
    assert pc(k=2) == 2
    assert pc(ec=None) == 1
    assert pc(mp=1 << 32) == 4
    assert pc(wsb=16) == 6


def test_bounds_on_the_host():
    """dbg_bounds: exact position counts from host offsets (no device work)."""
    from paper_1003_1940_amd import api
    off = np.array([0, 5, 5, 8, 40, 41], np.uint64)   # lengths 5, 0, 3, 32, 1
    for k in (1, 3, 5, 31):
        lens = np.diff(off.astype(np.int64))
        want = (int(np.maximum(lens - k + 1, 0).sum()), int(np.maximum(lens - k, 0).sum()))
        assert api.bounds(off, k) == want
    assert api.bounds(np.array([0], np.uint64), 3) == (0, 0)
    with pytest.raises(api.DbgError):
        api.bounds(off, 4)
    with pytest.raises(api.DbgError):
        api.bounds(np.array([1, 5], np.uint64), 3)
    with pytest.raises(api.DbgError):
        api.bounds(np.array([0, 5, 4], np.uint64), 3)
