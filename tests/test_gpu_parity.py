"""The HIP path against the oracle, element by element (exact integer equality).

Every case prints a line naming it before it touches the GPU."""

import random

import numpy as np
import pytest

import oracle
from paper_1003_1940_amd import synth
from .gpu_util import compare_with_oracle, gpu_graph, say
from .invariants import check_graph

pytestmark = pytest.mark.gpu


def _rs(reads):
    r = synth.from_strings(reads)
    return r.bases, r.offsets


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the MI355X")
    oracle.build(force=False)


SPECIAL = [
    (["AAAA"], 3), (["TTTT"], 3), (["GGGGG"], 3), (["ACAC", "TGTG"], 3), (["ACGT"], 3),
    (["AC", "ACG", "ACGTA", ""], 3), (["AATGCATC"], 3),
    (["ATGG", "CCAT", "GGAC", "GTTC", "TGGA", "TGGT"], 3),
    (["A"], 1), (["ACGTACGT"], 1), (["AC" * 40], 1), ([""], 5), (["ACG"], 5),
]


@pytest.mark.parametrize("idx", range(len(SPECIAL)))
def test_special_cases(idx):
    reads, k = SPECIAL[idx]
    b, o = _rs(reads)
    compare_with_oracle(b, o, k, label=f"special[{idx}]")


def test_random_small_sets():
    rnd = random.Random(11)
    for t in range(60):
        k = rnd.choice((1, 3, 5, 7, 9, 15, 31, 33, 63))
        alpha = rnd.choice(("AC", "ACGT", "ACGT", "GT"))
        reads = ["".join(rnd.choice(alpha) for _ in range(rnd.randint(0, 3 * k + 40)))
                 for _ in range(rnd.randint(1, 40))]
        b, o = _rs(reads)
        compare_with_oracle(b, o, k, label=f"random[{t}]")


@pytest.mark.parametrize("k", [1, 3, 5, 7, 15, 21, 31, 33, 47, 61, 63])
def test_k_sweep(k):
    rng = np.random.default_rng(100 + k)
    g = synth.random_genome(rng, 20_000)
    rs = synth.sample_reads(rng, g, 3000, 150, 0.01)
    compare_with_oracle(rs.bases, rs.offsets, k, label="k-sweep")


@pytest.mark.parametrize("in_tile", [1, 0])
@pytest.mark.parametrize("k", [33, 63])
def test_in_tile_level(k, in_tile):
    """128-bit keys: buckets of the in-tile level are split within their tiles
    and sorted as digit ranges.  Beside reads of a random genome, 4,000 copies of
    one read give in-tile buckets with digit cells too large for one batch
    (gathered, then split further down to uniform buckets), and 3,100 copies of a
    poly-A read a bucket too large for the in-tile level (scattered as before,
    at the same level).  Both settings of the knob give the oracle's tables."""
    from paper_1003_1940_amd import api
    rnd = random.Random(900 + k)
    genome = "".join(rnd.choice("ACGT") for _ in range(50_000))
    comp = str.maketrans("ACGT", "TGCA")
    reads = []
    for _ in range(3000):
        st = rnd.randrange(0, len(genome) - 150)
        r = genome[st:st + 150]
        reads.append(r.translate(comp)[::-1] if rnd.random() < 0.5 else r)
    reads += [genome[1000:1150]] * 4000 + ["A" * 150] * 3100
    rnd.shuffle(reads)
    b, o = _rs(reads)
    api.set_tuning(in_tile=in_tile)
    try:
        compare_with_oracle(b, o, k, label=f"in-tile level (in_tile={in_tile})")
    finally:
        api.set_tuning(defaults=True)


def test_plain_small_full():
    rs = synth.plain_small()
    _, got, ref = compare_with_oracle(rs.bases, rs.offsets, 31, label="plain_small (10k reads)")
    check_graph(ref, 31, rs.bases, rs.offsets)


def test_plain_repeats_subsample():
    rs = synth.plain_repeats(scale=0.005)  # 10,000 reads of the 2,000,000-read workload
    compare_with_oracle(rs.bases, rs.offsets, 31, label="plain_repeats 0.5%")


def test_plain_large_scaled():
    rs = synth.plain_large(scale=2.5e-4)  # 10,000 reads over a 25,000-base genome, k=63
    compare_with_oracle(rs.bases, rs.offsets, 63, label="plain_large 0.025%")


def test_identical_reads_oversized_buckets():
    # 3,000 copies of one read: every key occurs 3,000 times, so buckets exceed
    # the LDS capacity and go through the deeper partition levels.
    rng = np.random.default_rng(5)
    read = "".join("ACGT"[c] for c in rng.integers(0, 4, 100))
    b, o = _rs([read] * 3000)
    compare_with_oracle(b, o, 31, label="identical reads k=31")
    compare_with_oracle(b, o, 63, label="identical reads k=63")


def test_homopolymers_single_key():
    # one key repeated ~70,000 times: digits run out, the bucket is copied as is
    b, o = _rs(["A" * 100] * 500 + ["T" * 100] * 500)
    compare_with_oracle(b, o, 31, label="homopolymer k=31")
    compare_with_oracle(b, o, 33, label="homopolymer k=33")
    b, o = _rs(["C" * 40] * 2000)
    compare_with_oracle(b, o, 1, label="homopolymer k=1")


def test_every_start_offset_and_ragged_lengths():
    rng = np.random.default_rng(9)
    reads = []
    for L in range(0, 200):
        reads.append("".join("ACGT"[c] for c in rng.integers(0, 4, L)))
    b, o = _rs(reads)
    for k in (3, 31, 33, 63):
        compare_with_oracle(b, o, k, label="ragged 0..199")


def test_tiles_beyond_lds_staging():
    """Enumeration tiles that span more reads (1,024) or more bases (about 32,000)
    than a tile stages in LDS take the global-memory path; the same reads built
    with a few keys per read, and with keyless reads between keyed ones."""
    rng = np.random.default_rng(12)

    def rand(n):
        return "".join("ACGT"[c] for c in rng.integers(0, 4, n))

    for k in (31, 33):
        # one (k+1)-mer per read: a 4,096-key edge tile spans 4,096 reads
        reads = [rand(k + 1) for _ in range(9000)]
        b, o = _rs(reads)
        compare_with_oracle(b, o, k, label=f"reads of k+1 bases, k={k}")
        # five keys per keyed read, 40 keyless reads of k-1 bases after each: a
        # tile spans about 40,000 reads and more than 1M bases
        reads = []
        for _ in range(1500):
            reads.append(rand(k + 5))
            reads.extend(rand(k - 1) for _ in range(40))
        b, o = _rs(reads)
        compare_with_oracle(b, o, k, label=f"keyless reads between keyed ones, k={k}")


def test_no_keys_and_empty():
    b, o = _rs(["ACG", "AC", ""])
    compare_with_oracle(b, o, 31, label="all reads shorter than k")
    b, o = _rs([""])
    compare_with_oracle(b, o, 3, label="one empty read")


def test_determinism():
    rs = synth.plain_small(scale=0.5)
    _, a = gpu_graph(rs.bases, rs.offsets, 31)
    _, b = gpu_graph(rs.bases, rs.offsets, 31)
    for f in a:
        assert np.array_equal(a[f], b[f]), f


def test_batched_equals_plain():
    import paper_1003_1940_amd as dbg
    sets = synth.batched_sets(n_sets=12, scale=0.004)
    sets.insert(3, synth.from_strings([]))          # an empty set
    sets.insert(7, synth.from_strings(["ACG"]))     # a set with no edges
    bases = np.concatenate([s.bases for s in sets])
    lens = np.concatenate([np.diff(s.offsets.astype(np.int64)) for s in sets])
    offsets = np.zeros(len(lens) + 1, np.uint64)
    np.cumsum(lens, out=offsets[1:])
    sro = np.zeros(len(sets) + 1, np.uint64)
    np.cumsum([s.n_reads for s in sets], out=sro[1:])
    for k in (31, 63):
        say(f"[gpu-parity] batched {len(sets)} sets k={k}")
        g = dbg.api.build_batched(bases, offsets, sro, k)
        assert g.status == 0
        allg = g.to_numpy()
        nso = g.node_set_offsets.cpu().numpy()
        eso = g.edge_set_offsets.cpu().numpy()
        assert nso[-1] == g.n_nodes and eso[-1] == g.n_edges
        for i, s in enumerate(sets):
            ref = oracle.build_graph(s.bases, s.offsets, k)
            sl_n = slice(int(nso[i]), int(nso[i + 1]))
            sl_e = slice(int(eso[i]), int(eso[i + 1]))
            assert np.array_equal(allg["node_key"][sl_n], ref.node_key), f"set {i} nodes"
            assert np.array_equal(allg["node_count"][sl_n], ref.node_count), f"set {i} counts"
            for f in ("edge_u", "edge_v", "edge_orient", "edge_mult", "edge_z"):
                assert np.array_equal(allg[f][sl_e], getattr(ref, f)), f"set {i} {f}"


def test_device_status_bad_offsets():
    import torch
    from paper_1003_1940_amd import api
    b, o = _rs(["ACGTACGT", "ACGTAC"])
    packed, offs, n = api.upload(b, o)
    bad = torch.tensor([0, 9, 6], dtype=torch.int64, device="cuda")  # not monotone
    out = api.alloc_outputs(3, 16, 16)
    ws = api.Workspace(2, 1, 16, 3)
    res = torch.zeros(3, dtype=torch.int64, device="cuda")
    say("[gpu-parity] device-side offsets check")
    api.build_async(packed, n, bad, 3, 16, out, 16, 16, res, ws)
    assert api.read_result(res)[2] == 3  # DBG_E_OFFSETS


def test_capacity_short_reports_true_counts():
    from paper_1003_1940_amd import api
    rs = synth.plain_small(scale=0.05)
    ref = oracle.build_graph(rs.bases, rs.offsets, 31)
    say("[gpu-parity] capacity below the distinct count")
    g = api.build(rs.bases, rs.offsets, 31, node_cap=100, edge_cap=50)
    assert g.status == api.DBG_E_CAPACITY
    assert g.n_nodes == len(ref.node_count) and g.n_edges == len(ref.edge_mult)
    got = g.to_numpy()
    assert np.array_equal(got["node_key"][:100], ref.node_key[:100])
    assert np.array_equal(got["node_count"][:100], ref.node_count[:100])
    assert np.array_equal(got["edge_z"][:50], ref.edge_z[:50])
    assert np.array_equal(got["edge_mult"][:50], ref.edge_mult[:50])


def test_pack_rejects_non_acgt():
    import torch
    from paper_1003_1940_amd import api
    say("[gpu-parity] packer rejects N")
    a = torch.tensor(list(b"ACGTNACGT"), dtype=torch.uint8, device="cuda")
    _, res = api.pack(a)
    assert api.read_result(res)[2] == 8


@pytest.mark.parametrize("k,read_len,n_reads", [(31, 100, 20000), (63, 150, 12000)])
def test_shared_prefix_deep_levels(k, read_len, n_reads):
    """Reads that all begin with one 20-base head.  The k-mers that start inside
    the head share up to 40 leading bits, so thousands of distinct keys stay in
    one bucket through the first partition levels and split only at level 4 or 5
    into many LDS batches: the deep levels run on buckets of distinct keys, not
    only on repeats of one key.  A quarter of the reads repeat earlier ones and
    30% are reverse-complemented (their last k-mers canonicalise into the same
    buckets), so the buckets also hold duplicates of both strands."""
    rng = np.random.default_rng(2000 + k)
    head = np.concatenate([[0, 1], rng.integers(0, 4, 18)])  # "AC..." keeps it canonical
    n_unique = n_reads * 3 // 4
    codes = rng.integers(0, 4, size=(n_unique, read_len)).astype(np.uint8)
    codes[:, :20] = head
    codes = np.concatenate([codes, codes[rng.integers(0, n_unique, n_reads - n_unique)]])
    flip = rng.random(n_reads) < 0.3
    codes[flip] = 3 - codes[flip, ::-1]
    bases = np.frombuffer(b"ACGT", np.uint8)[codes].reshape(-1).copy()
    offsets = np.arange(n_reads + 1, dtype=np.uint64) * np.uint64(read_len)
    compare_with_oracle(bases, offsets, k, label=f"shared 20-base head, {n_reads} reads")
