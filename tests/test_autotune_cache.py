"""The autotuner's host side: candidate settings, input classes and the JSON
cache (no GPU needed; the library's tuning calls are host-only)."""

import pytest

from paper_1003_1940_amd import api, autotune


def test_candidates_cover_every_knob():
    c = autotune.candidates()
    assert len(c) == 18
    assert {x["node_path"] for x in c} == {api.NODES_KMERS, api.NODES_ENDPOINTS}
    assert {x["local_variant"] for x in c} == {0, 1, 2}
    assert {x["lds_digit_bias"] for x in c} == {-1, 0, 1}
    assert {x["in_tile"] for x in c} == {1}
    c2 = autotune.candidates(in_tiles=(1, 0))
    assert len(c2) == 36 and {x["in_tile"] for x in c2} == {0, 1}


def test_input_class():
    assert autotune.input_class(140_000_000, 200_000_000, 31) == "u64/n2^27"
    assert autotune.input_class(1, 1, 63) == "u128/n2^0"
    assert autotune.input_class(0, 0, 31) == "u64/n2^0"
    assert autotune.input_class(140_000_000, 200_000_000, 31, genome_hint=5_000_000) == \
        "u64/n2^27/cov2^5"


def test_cache_round_trip_and_apply(tmp_path):
    path = str(tmp_path / "tune.json")
    cache = autotune.TuneCache(path)
    best = dict(autotune.DEFAULT, node_path=api.NODES_ENDPOINTS, local_variant=1,
                lds_digit_bias=-1)
    r = autotune.TuneResult(best, [(best, 1.5, True)], 2.0,
                            autotune.input_class(1000, 2000, 31))
    cache.record(r)
    cache.save()
    again = autotune.TuneCache(path)
    assert again.lookup(1000, 2000, 31) == best
    assert again.lookup(1000, 2000, 33) is None          # other key width
    assert again.lookup(100_000, 2000, 31) is None       # other size class
    try:
        assert again.apply(1000, 2000, 31) == best
        assert again.apply(10 ** 6, 2000, 31) == autotune.DEFAULT  # untuned class
    finally:
        api.set_tuning(defaults=True)
