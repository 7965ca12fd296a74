"""Host logic of the sliced build: the slice planner (consecutive prefix ranges
that cover the key space and respect the key budget)."""

import numpy as np
import pytest

from paper_1003_1940_amd import sliced


def _check(plan, e, n, budget):
    assert plan[0][0] == 0 and plan[-1][1] == sliced.PREFIX_BINS
    for (a, b), (c, d) in zip(plan, plan[1:]):
        assert b == c and a < b
    for lo, hi in plan:
        assert int(e[lo:hi].sum()) <= budget and int(n[lo:hi].sum()) <= budget


def test_plan_covers_and_respects_budget():
    rng = np.random.default_rng(3)
    for t in range(50):
        e = rng.integers(0, 50, sliced.PREFIX_BINS).astype(np.uint64)
        n = rng.integers(0, 50, sliced.PREFIX_BINS).astype(np.uint64)
        # skew: canonical keys crowd the small prefixes
        e[:64] *= np.uint64(20)
        n[:64] *= np.uint64(20)
        budget = int(max(e.max(), n.max())) + int(rng.integers(0, 5000))
        plan = sliced.plan_slices(e, n, budget)
        _check(plan, e, n, budget)
        # greedy: no two neighbouring slices would fit together
        for (a, b), (_, d) in zip(plan, plan[1:]):
            assert int(e[a:d].sum()) > budget or int(n[a:d].sum()) > budget


def test_plan_single_slice_and_empty():
    z = np.zeros(sliced.PREFIX_BINS, np.uint64)
    assert sliced.plan_slices(z, z, 1) == [(0, sliced.PREFIX_BINS)]
    e = z.copy()
    e[7] = 5
    assert sliced.plan_slices(e, z, 5) == [(0, sliced.PREFIX_BINS)]


def test_plan_refuses_unsplittable_prefix():
    z = np.zeros(sliced.PREFIX_BINS, np.uint64)
    n = z.copy()
    n[100] = 11
    with pytest.raises(ValueError):
        sliced.plan_slices(z, n, 10)
    with pytest.raises(ValueError):
        sliced.plan_slices(z, z, 0)
    with pytest.raises(ValueError):
        sliced.plan_slices(z[:10], z, 5)
