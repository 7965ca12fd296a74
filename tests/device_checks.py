"""Checks of large device-resident outputs with plain torch tensor arithmetic.

Test infrastructure only: it shares nothing with the HIP library or the oracle.
A key is the base-4 value of a string (A0 C1 G2 T3, first base most significant)
held as two int64 tensors (lo, hi) carrying the uint64 bit patterns, exactly like
``keys_np`` does with numpy arrays; ``tests/test_device_checks.py`` compares the
two on the CPU.  Everything here works on any device; the full-size tests run it
on the GPU in chunks.
"""

import torch

SIGN = -(1 << 63)  # the int64 bit pattern of 2^63: xor maps unsigned order to signed
M2 = 0x3333333333333333
M4 = 0x0F0F0F0F0F0F0F0F
M8 = 0x00FF00FF00FF00FF
M16 = 0x0000FFFF0000FFFF
M32 = 0xFFFFFFFF


def srl(x, s: int):
    """Logical right shift of int64 bit patterns by 0 <= s <= 64."""
    if s == 0:
        return x
    if s >= 64:
        return torch.zeros_like(x)
    return (x >> s) & ((1 << (64 - s)) - 1)


def u32(x):
    """uint32 values held in int32 tensors, widened to int64."""
    return x.to(torch.int64) & M32


def less(alo, ahi, blo, bhi):
    """Unsigned 128-bit a < b."""
    ah, bh = ahi ^ SIGN, bhi ^ SIGN
    return (ah < bh) | ((ah == bh) & ((alo ^ SIGN) < (blo ^ SIGN)))


def shr128(lo, hi, s: int):
    if s == 0:
        return lo, hi
    if s >= 128:
        return torch.zeros_like(lo), torch.zeros_like(hi)
    if s >= 64:
        return srl(hi, s - 64), torch.zeros_like(hi)
    return srl(lo, s) | (hi << (64 - s)), srl(hi, s)


def shl128(lo, hi, s: int):
    if s == 0:
        return lo, hi
    if s >= 64:
        return torch.zeros_like(lo), lo << (s - 64)
    return lo << s, (hi << s) | srl(lo, 64 - s)


def mask128(lo, hi, bits: int):
    if bits >= 128:
        return lo, hi
    if bits == 64:
        return lo, torch.zeros_like(hi)
    if bits > 64:
        return lo, hi & ((1 << (bits - 64)) - 1)
    return lo & ((1 << bits) - 1), torch.zeros_like(hi)


def _rev_groups(x):
    """The 32 two-bit groups of each 64-bit word in reverse order."""
    x = ((x >> 2) & M2) | ((x & M2) << 2)
    x = ((x >> 4) & M4) | ((x & M4) << 4)
    x = ((x >> 8) & M8) | ((x & M8) << 8)
    x = ((x >> 16) & M16) | ((x & M16) << 16)
    return srl(x, 32) | (x << 32)


def revcomp(lo, hi, length: int):
    """Reverse complement of keys of ``length`` bases (Sec. 2): complemented
    bases (bitwise not of each 2-bit code) in reverse order."""
    nlo, nhi = _rev_groups(~hi), _rev_groups(~lo)
    return shr128(nlo, nhi, 128 - 2 * length)


def canonical(lo, hi, length: int):
    """The smaller of each key and its reverse complement, and whether that is
    the reverse complement."""
    rlo, rhi = revcomp(lo, hi, length)
    t = less(rlo, rhi, lo, hi)
    return torch.where(t, rlo, lo), torch.where(t, rhi, hi), t


def spell(ulo, uhi, vlo, vhi, o1, o2, k: int):
    """The (k+1)-mer an edge record stands for: strand o1 of u followed by the
    last base of strand o2 of v."""
    rulo, ruhi = revcomp(ulo, uhi, k)
    rvlo, rvhi = revcomp(vlo, vhi, k)
    f1, f2 = o1 == 1, o2 == 1
    alo, ahi = torch.where(f1, rulo, ulo), torch.where(f1, ruhi, uhi)
    blo = torch.where(f2, rvlo, vlo)
    zlo, zhi = shl128(alo, ahi, 2)
    return zlo | (blo & 3), zhi


def record_of(zlo, zhi, k: int):
    """Edge record (u, v, o1, o2) of (k+1)-mers z from the canonical forms of
    x = z[1..k] and y = z[2..k+1]: (x^, y^, s_x, s_y) when x^ < y^, (y^, x^,
    not s_y, not s_x) when x^ > y^, and for x^ = y^ the smaller orientation
    pair of the two."""
    xlo, xhi = shr128(zlo, zhi, 2)
    ylo, yhi = mask128(zlo, zhi, 2 * k)
    cxlo, cxhi, sx = canonical(xlo, xhi, k)
    cylo, cyhi, sy = canonical(ylo, yhi, k)
    sx, sy = sx.to(torch.int64), sy.to(torch.int64)
    y_first = less(cylo, cyhi, cxlo, cxhi)
    tie = ~less(cxlo, cxhi, cylo, cyhi) & ~y_first
    ulo, uhi = torch.where(y_first, cylo, cxlo), torch.where(y_first, cyhi, cxhi)
    vlo, vhi = torch.where(y_first, cxlo, cylo), torch.where(y_first, cxhi, cyhi)
    o1 = torch.where(y_first, 1 - sy, sx)
    o2 = torch.where(y_first, 1 - sx, sy)
    a1, a2 = 1 - o2, 1 - o1
    swap = tie & ((a1 < o1) | ((a1 == o1) & (a2 < o2)))
    return (ulo, uhi, vlo, vhi, torch.where(swap, a1, o1), torch.where(swap, a2, o2))


def mix(lo, hi, seed: int):
    """A 64-bit hash of each key (multiply / xor-shift rounds); any fixed
    function of the key serves the bucketed checks below."""
    h = lo * 0x5851F42D4C957F2D + hi * 0x14057B7EF767814F + seed
    h = h ^ srl(h, 31)
    h = h * 0x3C79AC492BA7B653
    return h ^ srl(h, 29)


class BucketSums:
    """Integer sums of per-key contributions gathered into 2^bits buckets by a
    hash of the key, twice: plainly and weighted by a second hash.  If every
    key's contributions sum to zero, so does every bucket; a key whose
    contributions do not cancel leaves its bucket non-zero unless another such
    key in the same bucket cancels it in both sums (the weighted sums wrap
    modulo 2^64, which keeps the exact zero of a balanced key)."""

    def __init__(self, device, bits: int = 24, seed: int = 0x2545F4914F6CDD1D):
        self.bits, self.seed = bits, seed
        self.plain = torch.zeros(1 << bits, dtype=torch.int64, device=device)
        self.weighted = torch.zeros(1 << bits, dtype=torch.int64, device=device)

    def add(self, lo, hi, val):
        h = mix(lo, hi, self.seed)
        b = srl(h, 64 - self.bits)
        self.plain.index_add_(0, b, val)
        self.weighted.index_add_(0, b, val * (h | 1))

    def nonzero(self) -> int:
        return int(((self.plain != 0) | (self.weighted != 0)).sum().item())


_CODE = None


def codes_of(ascii_u8):
    """A/C/G/T bytes -> 0..3 (other bytes -> 255)."""
    global _CODE
    if _CODE is None or _CODE.device != ascii_u8.device:
        t = torch.full((256,), 255, dtype=torch.uint8)
        for i, c in enumerate(b"ACGT"):
            t[c] = i
        _CODE = t.to(ascii_u8.device)
    return _CODE[ascii_u8.to(torch.int64)]


def window_keys(codes, starts, length: int):
    """Keys of the windows codes[s : s + length] for every start s."""
    lo = torch.zeros(starts.numel(), dtype=torch.int64, device=codes.device)
    hi = torch.zeros_like(lo)
    for t in range(length):
        c = codes[starts + t].to(torch.int64)
        hi = (hi << 2) | srl(lo, 62)
        lo = (lo << 2) | c
    return lo, hi
