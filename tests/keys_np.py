"""Vectorised k-mer keys in numpy, for checks on large outputs.

A key is the base-4 value of a string (A0 C1 G2 T3, first base most significant),
held as two uint64 arrays (lo, hi).  Written for the tests only; it shares nothing
with the oracle (which works on strings) or with the GPU library.
"""

import numpy as np

U64 = np.uint64
_CODE = np.full(256, 255, np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _CODE[_c] = _i


def codes(bases: np.ndarray) -> np.ndarray:
    c = _CODE[np.asarray(bases, np.uint8)]
    if (c == 255).any():
        raise ValueError("non-ACGT byte in input")
    return c


def window_starts(offsets: np.ndarray, length: int):
    """Stream positions of every window of ``length`` bases that lies inside one
    read, in read order, and the read index of each."""
    off = np.asarray(offsets, np.int64)
    lens = np.diff(off)
    cnt = np.maximum(lens - length + 1, 0)
    read = np.repeat(np.arange(len(lens)), cnt)
    first = np.repeat(off[:-1], cnt)
    idx_in_read = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    return first + idx_in_read, read


def window_keys(code_arr: np.ndarray, starts: np.ndarray, length: int):
    lo = np.zeros(len(starts), U64)
    hi = np.zeros(len(starts), U64)
    for t in range(length):
        c = code_arr[starts + t].astype(U64)
        hi = (hi << U64(2)) | (lo >> U64(62))
        lo = (lo << U64(2)) | c
    return lo, hi


def _rev_groups(x):
    x = ((x >> U64(2)) & U64(0x3333333333333333)) | ((x & U64(0x3333333333333333)) << U64(2))
    x = ((x >> U64(4)) & U64(0x0F0F0F0F0F0F0F0F)) | ((x & U64(0x0F0F0F0F0F0F0F0F)) << U64(4))
    return x.byteswap()


def shr128(lo, hi, s: int):
    if s == 0:
        return lo.copy(), hi.copy()
    if s >= 64:
        return hi >> U64(s - 64), np.zeros_like(hi)
    return (lo >> U64(s)) | (hi << U64(64 - s)), hi >> U64(s)


def shl128(lo, hi, s: int):
    if s == 0:
        return lo.copy(), hi.copy()
    if s >= 64:
        return np.zeros_like(lo), lo << U64(s - 64)
    return lo << U64(s), (hi << U64(s)) | (lo >> U64(64 - s))


def mask128(lo, hi, bits: int):
    if bits >= 128:
        return lo, hi
    if bits >= 64:
        return lo, hi & U64((1 << (bits - 64)) - 1)
    return lo & U64((1 << bits) - 1), np.zeros_like(hi)


def revcomp(lo, hi, length: int):
    """Reverse complement of keys of ``length`` bases."""
    nlo, nhi = _rev_groups(~hi), _rev_groups(~lo)  # 128-bit complement, groups reversed
    return shr128(nlo, nhi, 128 - 2 * length)


def less(alo, ahi, blo, bhi):
    return (ahi < bhi) | ((ahi == bhi) & (alo < blo))


def canonical(lo, hi, length: int):
    rlo, rhi = revcomp(lo, hi, length)
    take_rc = less(rlo, rhi, lo, hi)
    return np.where(take_rc, rlo, lo), np.where(take_rc, rhi, hi), take_rc


def record_of(zlo, zhi, k: int):
    """Edge record (u, v, o1, o2) of (k+1)-mers z, from the canonical forms of
    x = z[1..k] and y = z[2..k+1]: if x^ < y^ it is (x^, y^, s_x, s_y), if
    x^ > y^ it is (y^, x^, not s_y, not s_x), and for x^ = y^ the smaller of the two
    orientation pairs.  Strand s is 0 for the canonical strand, 1 otherwise."""
    xlo, xhi = shr128(zlo, zhi, 2)
    ylo, yhi = mask128(zlo, zhi, 2 * k)
    cxlo, cxhi, sx = canonical(xlo, xhi, k)
    cylo, cyhi, sy = canonical(ylo, yhi, k)
    sx = sx.astype(np.uint8)
    sy = sy.astype(np.uint8)
    x_first = less(cxlo, cxhi, cylo, cyhi)
    y_first = less(cylo, cyhi, cxlo, cxhi)
    tie = ~x_first & ~y_first
    ulo = np.where(y_first, cylo, cxlo)
    uhi = np.where(y_first, cyhi, cxhi)
    vlo = np.where(y_first, cxlo, cylo)
    vhi = np.where(y_first, cxhi, cyhi)
    o1 = np.where(y_first, 1 - sy, sx).astype(np.uint8)
    o2 = np.where(y_first, 1 - sx, sy).astype(np.uint8)
    # tie: the pair and its reversal (1 - o2, 1 - o1) name one edge; keep the smaller
    a1, a2 = 1 - o2, 1 - o1
    swap = tie & ((a1 < o1) | ((a1 == o1) & (a2 < o2)))
    o1 = np.where(swap, a1, o1).astype(np.uint8)
    o2 = np.where(swap, a2, o2).astype(np.uint8)
    return ulo, uhi, vlo, vhi, o1, o2


def spell(ulo, uhi, vlo, vhi, o1, o2, k: int):
    """The (k+1)-mer an edge record stands for: strand o1 of u, then the last base
    of strand o2 of v."""
    rulo, ruhi = revcomp(ulo, uhi, k)
    rvlo, rvhi = revcomp(vlo, vhi, k)
    alo = np.where(o1 == 1, rulo, ulo)
    ahi = np.where(o1 == 1, ruhi, uhi)
    blo = np.where(o2 == 1, rvlo, vlo)
    bhi = np.where(o2 == 1, rvhi, vhi)
    zlo, zhi = shl128(alo, ahi, 2)
    return zlo | (blo & U64(3)), zhi, (alo, ahi, blo, bhi)


def to_str(lo, hi, length: int) -> str:
    v = (int(hi) << 64) | int(lo)
    return "".join("ACGT"[(v >> (2 * (length - 1 - i))) & 3] for i in range(length))


def from_str(s: str):
    v = 0
    for ch in s:
        v = v * 4 + "ACGT".index(ch)
    return v & ((1 << 64) - 1), v >> 64


def unique_keys(bases, offsets, length: int):
    """np.unique over the canonical keys of every ``length``-window of the reads:
    returns (lo, hi, counts) in ascending key order."""
    c = codes(bases)
    starts, _ = window_starts(offsets, length)
    lo, hi = window_keys(c, starts, length)
    clo, chi, _ = canonical(lo, hi, length)
    if length <= 32:
        u, cnt = np.unique(clo, return_counts=True)
        return u, np.zeros_like(u), cnt
    both = np.stack([chi, clo], axis=1)
    u, cnt = np.unique(both, axis=0, return_counts=True)
    return u[:, 1].copy(), u[:, 0].copy(), cnt
