"""Full-size checks of the 40,000,000-read k = 63 build (3.52 G k-mer positions,
128-bit keys, more than 2^31 keys per table), built as bench.py builds it: output
capacity 0.55 x k-mer positions, no edge keys.  The oracle cannot build a graph
this size in a test's time, so every row is checked for properties that hold at
any size (order, totals, counts >= 1) on the device, and sampled rows for
canonical form, endpoint membership and the record <-> (k+1)-mer round trip."""

import gc
import os

import numpy as np
import pytest

from paper_1003_1940_amd import synth
from . import keys_np as K
from .gpu_util import say

pytestmark = pytest.mark.gpu

k = 63
CHUNK = 1 << 27  # rows per device-side check, to bound temporaries


def _unsigned(t):
    """int64 bit patterns reordered so that signed order is unsigned order."""
    import torch
    return t ^ torch.tensor(-(1 << 63), dtype=torch.int64, device=t.device)


def _ascending128(lo, hi):
    """Strict ascending order of (hi, lo) 128-bit keys held as int64 pairs
    (columns of one tensor), checked in chunks."""
    n = lo.numel()
    for a in range(0, max(n - 1, 0), CHUNK):
        b = min(n, a + CHUNK + 1)
        ulo, uhi = _unsigned(lo[a:b]), _unsigned(hi[a:b])
        ok = (uhi[1:] > uhi[:-1]) | ((uhi[1:] == uhi[:-1]) & (ulo[1:] > ulo[:-1]))
        if not bool(ok.all()):
            return False
    return True


def _chunked_sum(t):
    import torch
    s = 0
    for a in range(0, t.numel(), CHUNK):
        s += int((t[a:a + CHUNK].to(torch.int64) & 0xFFFFFFFF).sum().item())
    return s


def _find128(klo, khi, qlo, qhi):
    """Indices of query keys in sorted device keys (-1 where absent): a
    vectorised binary search on the device that gathers only the probed rows."""
    import torch
    n = klo.numel()
    qul, quh = _unsigned(qlo), _unsigned(qhi)
    lo = torch.zeros_like(qlo)
    hi = torch.full_like(qlo, n)
    while bool((lo < hi).any()):
        mid = (lo + hi) // 2
        midc = mid.clamp(max=n - 1)
        mh, ml = _unsigned(khi[midc]), _unsigned(klo[midc])
        below = (mh < quh) | ((mh == quh) & (ml < qul))
        active = lo < hi
        lo = torch.where(active & below, mid + 1, lo)
        hi = torch.where(active & ~below, mid, hi)
    idx = lo.clamp(max=n - 1)
    hit = (lo < n) & (_unsigned(khi[idx]) == quh) & (_unsigned(klo[idx]) == qul)
    return torch.where(hit, lo, torch.full_like(lo, -1))


@pytest.fixture(scope="module")
def large_full():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the MI355X")
    from paper_1003_1940_amd import api
    say("[gpu-fullsize-k63] generating 40,000,000 reads (forked workers draw them)")
    rs = synth.plain_large(workers=max(1, min(16, os.cpu_count() or 1)))
    n_k, n_e = rs.kmer_count(k), rs.kmer_count(k + 1)
    cap = int(n_k * 0.55)
    say(f"[gpu-fullsize-k63] building: {n_k} k-mers, output capacity {cap}")
    g = api.build(rs.bases, rs.offsets, k, zkey=False, node_cap=cap, edge_cap=cap)
    del rs
    gc.collect()
    yield g, n_k, n_e
    del g
    gc.collect()
    torch.cuda.empty_cache()  # later tests size their budgets from free HBM


def test_k63_fullsize_status_and_totals(large_full):
    g, n_k, n_e = large_full
    assert g.status == 0, f"device status {g.status}"
    assert 0 < g.n_nodes <= g.node_count.numel() and 0 < g.n_edges <= g.edge_mult.numel()
    say(f"[gpu-fullsize-k63] {g.n_nodes} nodes, {g.n_edges} edges")
    cnt, mult = g.node_count[:g.n_nodes], g.edge_mult[:g.n_edges]
    assert _chunked_sum(cnt) == n_k, "node counts do not add up to the k-mer positions"
    assert _chunked_sum(mult) == n_e, "edge multiplicities do not add up to the (k+1)-mers"
    assert not bool((cnt == 0).any()) and not bool((mult == 0).any())


def test_k63_fullsize_node_order(large_full):
    g, _, _ = large_full
    keys = g.node_kmer[:g.n_nodes]
    assert _ascending128(keys[:, 0], keys[:, 1]), "node keys are not strictly ascending"


def test_k63_fullsize_sampled_rows(large_full):
    import torch
    g, _, _ = large_full
    rng = np.random.default_rng(63)
    ni = torch.from_numpy(np.sort(rng.choice(g.n_nodes, 2000, replace=False))).cuda()
    nk = g.node_kmer[ni].cpu().numpy().view(np.uint64)
    lo, hi = nk[:, 0].copy(), nk[:, 1].copy()
    rlo, rhi = K.revcomp(lo, hi, k)
    assert K.less(lo, hi, rlo, rhi).all(), "a node key is not strictly canonical (odd k)"
    # consecutive sampled edges: records round-trip through their (k+1)-mer and
    # come in ascending order of it
    start = int(rng.integers(0, g.n_edges - 2001))
    sl = slice(start, start + 2000)
    u = g.edge_u[sl].cpu().numpy().view(np.uint64)
    v = g.edge_v[sl].cpu().numpy().view(np.uint64)
    o = g.edge_orient[sl].cpu().numpy()
    o1, o2 = (o >> 1) & 1, o & 1
    zlo, zhi, _ = K.spell(u[:, 0].copy(), u[:, 1].copy(), v[:, 0].copy(), v[:, 1].copy(), o1, o2, k)
    zlo, zhi, _ = K.canonical(zlo, zhi, k + 1)
    assert K.less(zlo[:-1], zhi[:-1], zlo[1:], zhi[1:]).all(), "edges not in (k+1)-mer order"
    rec = K.record_of(zlo, zhi, k)
    assert np.array_equal(rec[0], u[:, 0]) and np.array_equal(rec[1], u[:, 1])
    assert np.array_equal(rec[2], v[:, 0]) and np.array_equal(rec[3], v[:, 1])
    assert np.array_equal(rec[4], o1) and np.array_equal(rec[5], o2)
    assert not K.less(v[:, 0], v[:, 1], u[:, 0], u[:, 1]).any(), "an edge has u > v"
    # both endpoints of sampled edges are nodes
    keys = g.node_kmer[:g.n_nodes]
    ei = torch.from_numpy(rng.choice(g.n_edges, 2000, replace=False)).cuda()
    for col in (g.edge_u, g.edge_v):
        q = col[ei]
        found = _find128(keys[:, 0], keys[:, 1], q[:, 0].contiguous(), q[:, 1].contiguous())
        assert bool((found >= 0).all()), "an edge endpoint is not a node"
