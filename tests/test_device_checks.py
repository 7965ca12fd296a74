"""The torch key helpers used by the full-size GPU checks, run on the CPU against
the numpy ones (keys_np) and against facts that hold for any graph."""

import numpy as np
import pytest
import torch

from . import device_checks as D
from . import keys_np as K


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.uint64).view(np.int64))


def _n(t):
    return t.numpy().view(np.uint64)


def _rand_keys(rng, n, length):
    lo = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=n, dtype=np.uint64)
    hi = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=n, dtype=np.uint64)
    return K.mask128(lo, hi, 2 * length)


@pytest.mark.parametrize("length", [1, 2, 17, 31, 32, 33, 48, 63, 64])
def test_revcomp_canonical_match_numpy(length):
    rng = np.random.default_rng(length)
    lo, hi = _rand_keys(rng, 5000, length)
    rl, rh = K.revcomp(lo, hi, length)
    tl, th = D.revcomp(_t(lo), _t(hi), length)
    assert np.array_equal(_n(tl), rl) and np.array_equal(_n(th), rh)
    cl, ch, f = K.canonical(lo, hi, length)
    dl, dh, g = D.canonical(_t(lo), _t(hi), length)
    assert np.array_equal(_n(dl), cl) and np.array_equal(_n(dh), ch)
    assert np.array_equal(g.numpy(), f)


@pytest.mark.parametrize("k", [1, 3, 31, 33, 63])
def test_record_and_spell_match_numpy(k):
    rng = np.random.default_rng(100 + k)
    zlo, zhi = _rand_keys(rng, 5000, k + 1)
    # include homopolymers and palindromes of length k + 1
    for s in ("A" * (k + 1), "T" * (k + 1), "C" * (k + 1), "AT" * ((k + 1) // 2)):
        a, b = K.from_str(s)
        zlo = np.append(zlo, np.uint64(a))
        zhi = np.append(zhi, np.uint64(b))
    want = K.record_of(zlo, zhi, k)
    got = D.record_of(_t(zlo), _t(zhi), k)
    for w, g in zip(want, got):
        assert np.array_equal(np.asarray(w).astype(np.uint64), g.numpy().astype(np.int64).view(np.uint64))
    sl, sh, _ = K.spell(*want, k)
    tl, th = D.spell(*got, k)
    assert np.array_equal(_n(tl), sl) and np.array_equal(_n(th), sh)


def test_less_is_unsigned_128():
    vals = [0, 1, (1 << 63) - 1, 1 << 63, (1 << 64) - 1]
    pairs = [(a, b) for a in vals for b in vals]
    alo = np.array([a for a, _ in pairs], np.uint64)
    blo = np.array([b for _, b in pairs], np.uint64)
    for ahi_v, bhi_v in ((0, 0), (1 << 63, 5), (5, 1 << 63)):
        ahi = np.full(len(pairs), ahi_v, np.uint64)
        bhi = np.full(len(pairs), bhi_v, np.uint64)
        want = K.less(alo, ahi, blo, bhi)
        got = D.less(_t(alo), _t(ahi), _t(blo), _t(bhi)).numpy()
        assert np.array_equal(want, got)


def test_window_keys_match_numpy():
    rng = np.random.default_rng(4)
    bases = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, 3000)]
    starts = np.arange(0, 3000 - 63, 7)
    lo, hi = K.window_keys(K.codes(bases), starts, 63)
    c = D.codes_of(torch.from_numpy(bases.copy()))
    tl, th = D.window_keys(c, torch.from_numpy(starts), 63)
    assert np.array_equal(_n(tl), lo) and np.array_equal(_n(th), hi)


def test_bucket_sums_balanced_and_unbalanced():
    rng = np.random.default_rng(8)
    lo, hi = _rand_keys(rng, 20000, 63)
    tl, th = _t(lo), _t(hi)
    vals = torch.from_numpy(rng.integers(1, 100, 20000))
    b = D.BucketSums("cpu", bits=10)
    b.add(tl, th, vals)
    perm = torch.from_numpy(rng.permutation(20000))
    b.add(tl[perm], th[perm], -vals[perm])
    assert b.nonzero() == 0
    # one contribution moved from one key to another: both buckets light up
    b.add(tl[:1], th[:1], torch.tensor([3]))
    b.add(tl[1:2], th[1:2], torch.tensor([-3]))
    assert b.nonzero() >= 1
