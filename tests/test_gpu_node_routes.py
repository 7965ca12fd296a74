"""The node table's two routes (STEP-3 of Sec. 3): enumerating every k-mer, and
summing the weighted endpoints of the distinct edges plus the read ends.  Each
route is forced in turn and compared with the oracle element by element; the
result flag shows which route ran."""

import random

import numpy as np
import pytest

import oracle
from paper_1003_1940_amd import synth
from .gpu_util import FIELDS, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the MI355X")
    oracle.build(force=False)
    from paper_1003_1940_amd import api
    yield
    api.set_tuning(defaults=True)


def _rs(reads):
    r = synth.from_strings(reads)
    return r.bases, r.offsets


def endpoint_route_fits(n_k, u_e, n_reads, k, max_keys):
    """Whether the endpoint records fit the workspace key buffers (the library's
    own rule, restated): keys below the weight offset, weights inside the buffer."""
    w = 8 if k <= 31 else 16
    kb = (max_keys + 2) * w
    off = (kb // (w + 4) * w) & ~15
    r = 2 * u_e + 2 * n_reads
    return u_e > 0 and n_k < 2 ** 31 and r * w <= off and off + 4 * r <= kb


def check_route(bases, offsets, k, route, label, max_keys_factor=4):
    from paper_1003_1940_amd import api
    api.set_tuning(node_path=route)
    lens = np.diff(np.asarray(offsets, np.int64))
    n_k = int(np.maximum(lens - k + 1, 0).sum()) if len(lens) else 0
    max_keys = max_keys_factor * n_k + 64
    say(f"[gpu-routes] {label} k={k} route={route} reads={len(lens)}")
    g = api.build(np.asarray(bases, np.uint8), np.asarray(offsets, np.uint64), k,
                  max_keys=max_keys)
    assert g.status == 0, f"{label}: status {g.status}"
    ref = oracle.build_graph(bases, offsets, k)
    assert g.n_nodes == len(ref.node_count) and g.n_edges == len(ref.edge_mult), label
    got = g.to_numpy()
    for f in FIELDS:
        if got[f] is None:
            continue
        assert np.array_equal(got[f], getattr(ref, f)), f"{label}: column {f} differs"
    took = bool(g.extra["flags"] & api.FLAG_NODES_FROM_ENDPOINTS)
    if route == api.NODES_KMERS:
        assert not took, label
    elif route == api.NODES_ENDPOINTS:
        assert took == endpoint_route_fits(n_k, len(ref.edge_mult), len(lens), k, max_keys), label
    return took


SPECIAL = [
    (["AAAA"], 3), (["TTTT"], 3), (["GGGGG"], 3), (["ACAC", "TGTG"], 3), (["ACGT"], 3),
    (["AC", "ACG", "ACGTA", ""], 3), (["AATGCATC"], 3),
    (["ATGG", "CCAT", "GGAC", "GTTC", "TGGA", "TGGT"], 3),
    (["A"], 1), (["ACGTACGT"], 1), (["AC" * 40], 1), ([""], 5), (["ACG"], 5),
    (["ACG", "ACG", "TTTT", "A"], 3), (["ACGTAC"] * 50 + ["GT"] * 7, 5),
]


@pytest.mark.parametrize("route", [0, 1])
def test_routes_special_cases(route):
    for i, (reads, k) in enumerate(SPECIAL):
        b, o = _rs(reads)
        check_route(b, o, k, route, f"special[{i}]")


@pytest.mark.parametrize("route", [0, 1])
def test_routes_random_sets(route):
    rnd = random.Random(23)
    took = 0
    for t in range(50):
        k = rnd.choice((1, 3, 5, 7, 15, 31, 33, 63))
        alpha = rnd.choice(("AC", "ACGT", "ACGT", "GT"))
        reads = ["".join(rnd.choice(alpha) for _ in range(rnd.randint(0, 3 * k + 40)))
                 for _ in range(rnd.randint(1, 40))]
        b, o = _rs(reads)
        took += check_route(b, o, k, route, f"random[{t}]")
    if route == 1:
        assert took >= 40


@pytest.mark.parametrize("k", [3, 21, 31, 33, 63])
def test_endpoint_route_k_sweep(k):
    rng = np.random.default_rng(300 + k)
    g = synth.random_genome(rng, 20_000)
    rs = synth.sample_reads(rng, g, 3000, 150, 0.01)
    assert check_route(rs.bases, rs.offsets, k, 1, "k-sweep")


def test_endpoint_route_repeats_and_identical_reads():
    rs = synth.plain_repeats(scale=0.005)
    assert check_route(rs.bases, rs.offsets, 31, 1, "plain_repeats 0.5%")
    # one read 3,000 times: the read-end records of one key outgrow a bucket, so
    # the weighted sum runs over an oversized bucket whose digits are exhausted
    rng = np.random.default_rng(5)
    read = "".join("ACGT"[c] for c in rng.integers(0, 4, 100))
    b, o = _rs([read] * 3000)
    assert check_route(b, o, 31, 1, "identical reads k=31")
    assert check_route(b, o, 63, 1, "identical reads k=63")
    b, o = _rs(["A" * 100] * 500 + ["T" * 100] * 500)
    assert check_route(b, o, 31, 1, "homopolymer k=31")
    b, o = _rs(["C" * 40] * 2000)
    assert check_route(b, o, 1, 1, "homopolymer k=1")


def test_endpoint_route_ragged_and_short_reads():
    rng = np.random.default_rng(9)
    reads = ["".join("ACGT"[c] for c in rng.integers(0, 4, L)) for L in range(0, 200)]
    b, o = _rs(reads)
    for k in (3, 31, 33, 63):
        assert check_route(b, o, k, 1, "ragged 0..199")


def _high_coverage():
    # 20x coverage of a 20,000-base genome with 0.1% errors: about 0.25 endpoint
    # records per k-mer
    rng = np.random.default_rng(77)
    g = synth.random_genome(rng, 20_000)
    return synth.sample_reads(rng, g, 4000, 100, 0.001)


def test_auto_route_picks_by_ratio():
    """AUTO takes the endpoint route when the records are few against the k-mers
    (high coverage) and enumerates otherwise; both give the oracle's tables."""
    from paper_1003_1940_amd import api
    rs = _high_coverage()
    api.set_tuning(node_path=api.NODES_AUTO, endpoint_ratio=0.6)
    assert check_route(rs.bases, rs.offsets, 31, -1, "auto, high coverage", max_keys_factor=1)
    api.set_tuning(endpoint_ratio=0.0)
    assert not check_route(rs.bases, rs.offsets, 31, -1, "auto, ratio 0", max_keys_factor=1)
    rs = synth.plain_repeats(scale=0.005)   # 0.2x coverage: nearly every edge distinct
    api.set_tuning(endpoint_ratio=0.6)
    assert not check_route(rs.bases, rs.offsets, 31, -1, "auto, low coverage",
                           max_keys_factor=1)
    api.set_tuning(defaults=True)


def test_batched_builds_enumerate():
    """Multi-set builds always enumerate (the endpoint route is single-set)."""
    from paper_1003_1940_amd import api
    api.set_tuning(node_path=api.NODES_ENDPOINTS)
    sets = synth.batched_sets(n_sets=4, scale=0.002)
    bases = np.concatenate([s.bases for s in sets])
    lens = np.concatenate([np.diff(s.offsets.astype(np.int64)) for s in sets])
    offsets = np.zeros(len(lens) + 1, np.uint64)
    np.cumsum(lens, out=offsets[1:])
    sro = np.zeros(len(sets) + 1, np.uint64)
    np.cumsum([s.n_reads for s in sets], out=sro[1:])
    say("[gpu-routes] batched with the endpoint route requested")
    g = api.build_batched(bases, offsets, sro, 31)
    assert g.status == 0
    allg = g.to_numpy()
    nso = g.node_set_offsets.cpu().numpy()
    for i, s in enumerate(sets):
        ref = oracle.build_graph(s.bases, s.offsets, 31)
        sl = slice(int(nso[i]), int(nso[i + 1]))
        assert np.array_equal(allg["node_key"][sl], ref.node_key)
        assert np.array_equal(allg["node_count"][sl], ref.node_count)
    api.set_tuning(defaults=True)
