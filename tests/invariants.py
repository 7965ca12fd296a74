"""Well-formedness checks that any correct graph output satisfies, whoever built
it.  Each check states the fact it tests; all are vectorised with numpy.

Arrays: node_key (U_n, 2) uint64 as (lo, hi); node_count (U_n,); edge_u, edge_v,
edge_z (U_e, 2); edge_orient (U_e,) uint8 = (o1 << 1) | o2 with '+' = 0;
edge_mult (U_e,).
"""

import numpy as np

from . import keys_np as K


def _lohi(a):
    a = np.asarray(a, np.uint64)
    if a.ndim == 1:
        return a, np.zeros_like(a)
    return a[:, 0], a[:, 1]


def strictly_ascending(lo, hi) -> bool:
    if len(lo) < 2:
        return True
    return bool(K.less(lo[:-1], hi[:-1], lo[1:], hi[1:]).all())


def check_graph(g, k: int, bases=None, offsets=None):
    """Runs every invariant; raises AssertionError naming the first that fails.
    ``g`` has the attributes listed in the module docstring."""
    nlo, nhi = _lohi(g.node_key)
    ulo, uhi = _lohi(g.edge_u)
    vlo, vhi = _lohi(g.edge_v)
    zlo, zhi = _lohi(g.edge_z)
    o = np.asarray(g.edge_orient, np.uint8)
    o1, o2 = (o >> 1) & 1, o & 1
    count = np.asarray(g.node_count, np.uint64)
    mult = np.asarray(g.edge_mult, np.uint64)

    # I1: nodes strictly ascending by key; edges strictly ascending by z.
    assert strictly_ascending(nlo, nhi), "I1: node keys not strictly ascending"
    assert strictly_ascending(zlo, zhi), "I1: edge z not strictly ascending"

    # I2: with k odd no k-mer equals its reverse complement, so every node is the
    # strictly smaller strand of its k-molecule.
    rlo, rhi = K.revcomp(nlo, nhi, k)
    assert K.less(nlo, nhi, rlo, rhi).all(), "I2: a node key is not strictly canonical"

    # I3: twin invariant.  The record spells z (its endpoints overlap by k - 1);
    # z is canonical; the record of z and of its reverse complement are both this
    # record.
    szlo, szhi, (alo, ahi, blo, bhi) = K.spell(ulo, uhi, vlo, vhi, o1, o2, k)
    a_suf_lo, a_suf_hi = K.mask128(alo, ahi, 2 * (k - 1))
    b_pre_lo, b_pre_hi = K.shr128(blo, bhi, 2)
    assert ((a_suf_lo == b_pre_lo) & (a_suf_hi == b_pre_hi)).all(), \
        "I3: edge endpoints do not overlap by k-1"
    czlo, czhi, _ = K.canonical(szlo, szhi, k + 1)
    assert ((czlo == zlo) & (czhi == zhi)).all(), "I3: z is not the canonical spelling"
    for tlo, thi in ((zlo, zhi), K.revcomp(zlo, zhi, k + 1)):
        r = K.record_of(tlo, thi, k)
        same = ((r[0] == ulo) & (r[1] == uhi) & (r[2] == vlo) & (r[3] == vhi) &
                (r[4] == o1) & (r[5] == o2))
        assert same.all(), "I3: a (k+1)-mer and its twin do not map to the stored record"

    # I7: every count and multiplicity is at least 1.
    assert (count >= 1).all(), "I7: zero node count"
    assert (mult >= 1).all(), "I7: zero edge multiplicity"

    # I6: every edge endpoint is a node.
    if len(ulo):
        for elo, ehi in ((ulo, uhi), (vlo, vhi)):
            idx = _find(nlo, nhi, elo, ehi)
            assert (idx >= 0).all(), "I6: edge endpoint missing from the node table"

    if bases is None:
        return
    off = np.asarray(offsets, np.int64)
    lens = np.diff(off)
    # I4: totals.  sum of multiplicities = number of (k+1)-mer positions,
    # sum of counts = number of k-mer positions.
    assert int(mult.sum()) == int(np.maximum(lens - k, 0).sum()), "I4: sum of multiplicities"
    assert int(count.sum()) == int(np.maximum(lens - k + 1, 0).sum()), "I4: sum of counts"

    # I5: degree identity.  Every k-mer occurrence has an edge to its successor and
    # from its predecessor in the read, except the read's first and last k-mer, so
    # per node: sum of incident multiplicities (a self-loop counts twice)
    # = 2 count - first - last.
    deg = np.zeros(len(nlo), np.int64)
    if len(ulo):
        np.add.at(deg, _find(nlo, nhi, ulo, uhi), mult.astype(np.int64))
        np.add.at(deg, _find(nlo, nhi, vlo, vhi), mult.astype(np.int64))
    c = K.codes(bases)
    has = lens >= k
    ends = np.zeros(len(nlo), np.int64)
    for starts in (off[:-1][has], (off[1:] - k)[has]):
        lo, hi = K.window_keys(c, starts, k)
        clo, chi, _ = K.canonical(lo, hi, k)
        np.add.at(ends, _find(nlo, nhi, clo, chi), 1)
    assert (deg == 2 * count.astype(np.int64) - ends).all(), "I5: degree identity"


def _find(nlo, nhi, qlo, qhi):
    """Index of each query key in the sorted key table, -1 if absent."""
    if len(nlo) == 0:
        return np.full(len(qlo), -1, np.int64)
    dt = np.dtype([("hi", "<u8"), ("lo", "<u8")])
    table = np.empty(len(nlo), dt)
    table["hi"], table["lo"] = nhi, nlo
    q = np.empty(len(qlo), dt)
    q["hi"], q["lo"] = qhi, qlo
    idx = np.minimum(np.searchsorted(table, q), len(nlo) - 1)
    ok = (nlo[idx] == qlo) & (nhi[idx] == qhi)
    return np.where(ok, idx, -1)
