"""dbg_build_noalloc (the build with the library's static per-device scratch)
against dbg_build (caller-provided workspace), through the C ABI: identical
tables, element by element, on two calls in a row, the second with a smaller
input (the scratch keeps the first call's contents); and a build larger than
the scratch is refused on the host with DBG_E_SCRATCH, enqueuing nothing."""

import numpy as np
import pytest

from paper_1003_1940_amd import api, synth
from .gpu_util import say

pytestmark = pytest.mark.gpu

FIELDS = ("node_key", "node_count", "edge_u", "edge_v", "edge_orient", "edge_mult", "edge_z")


def _run(rs, k, noalloc):
    import torch
    packed, offs, n_bases = api.upload(rs.bases, rs.offsets)
    n_k, _ = api.bounds(rs.offsets, k)
    out = api.alloc_outputs(k, n_k, n_k, "cuda", zkey=True)
    result = torch.zeros(3, dtype=torch.int64, device="cuda")
    if noalloc:
        api.build_noalloc_async(packed, n_bases, offs, k, n_k, out, n_k, n_k, result)
    else:
        ws = api.Workspace(rs.n_reads, 1, n_k, k)
        api.build_async(packed, n_bases, offs, k, n_k, out, n_k, n_k, result, ws)
    n_nodes, n_edges, status = api.read_result(result)
    g = api.Graph(k, out["node_kmer"], out["node_count"], out["edge_u"], out["edge_v"],
                  out["edge_orient"], out["edge_mult"], out["edge_zkey"], n_nodes, n_edges,
                  status)
    return g, g.to_numpy()


@pytest.mark.parametrize("k", [31, 63])
def test_noalloc_equals_build_twice(k):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the MI355X")
    first = synth.plain_small(scale=0.5)    # 5,000 reads
    second = synth.plain_small(scale=0.15)  # 1,500 reads, fewer than the first
    for label, rs in (("first", first), ("second, smaller", second)):
        say(f"[gpu-noalloc] k={k} {label} call: {rs.n_reads} reads")
        g_ref, ref = _run(rs, k, noalloc=False)
        g, got = _run(rs, k, noalloc=True)
        assert g_ref.status == 0 and g.status == 0, (g_ref.status, g.status)
        assert (g.n_nodes, g.n_edges) == (g_ref.n_nodes, g_ref.n_edges)
        for f in FIELDS:
            assert np.array_equal(got[f], ref[f]), f"{label} call, k={k}: column {f} differs"


def test_noalloc_refuses_builds_beyond_the_scratch():
    import torch
    say("[gpu-noalloc] oversize build refused on the host")
    rs = synth.plain_small(scale=0.01)
    packed, offs, n_bases = api.upload(rs.bases, rs.offsets)
    out = api.alloc_outputs(31, 16, 16, "cuda", zkey=False)
    result = torch.full((3,), 7, dtype=torch.int64, device="cuda")
    too_many = 200_000_000  # k-mer bound whose workspace exceeds the scratch
    assert api.workspace_bytes(rs.n_reads, 1, too_many, 31) > api.NOALLOC_SCRATCH_BYTES
    with pytest.raises(api.DbgError) as e:
        api.build_noalloc_async(packed, n_bases, offs, 31, too_many, out, 16, 16, result)
    assert e.value.code == api.DBG_E_SCRATCH
    torch.cuda.synchronize()
    assert bool((result == 7).all()), "a refused call wrote the result record"
