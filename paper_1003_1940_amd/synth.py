"""Seeded synthetic read sets (the workloads), shared by the library's benchmark and
the tests.

This module only draws random DNA: genomes, read positions, strands and
substitution errors.  It holds none of the graph-construction arithmetic.  Reads are
returned as one ASCII byte array (``b"ACGT"`` letters) plus ``uint64`` offsets
(read i is ``bases[offsets[i]:offsets[i+1]]``), the format both the GPU library's
packer and the CPU oracle consume.

Recipe (every workload): a genome of i.i.d. bases with the given base
probabilities; read starts uniform on ``[0, G - L]``; each read reverse-complemented
with probability 0.5; then each base independently substituted with probability
``err`` by one of the three other bases, uniformly.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ALPHABET = np.frombuffer(b"ACGT", dtype=np.uint8)
SEED_BASE = 1003_1940 * 10


@dataclass
class ReadSet:
    bases: np.ndarray     # uint8 ASCII, concatenated reads
    offsets: np.ndarray   # uint64, n_reads + 1
    params: dict = field(default_factory=dict)

    @property
    def n_reads(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_bases(self) -> int:
        return int(self.offsets[-1])

    def kmer_count(self, k: int) -> int:
        """Number of read positions holding a k-mer: sum over reads of max(0, L - k + 1)."""
        lens = np.diff(self.offsets.astype(np.int64))
        return int(np.maximum(lens - k + 1, 0).sum())

    def subset(self, idx) -> "ReadSet":
        """Reads ``idx`` (an index array) as a new read set."""
        idx = np.asarray(idx, dtype=np.int64)
        lens = np.diff(self.offsets.astype(np.int64))[idx]
        offs = np.zeros(len(idx) + 1, np.uint64)
        np.cumsum(lens, out=offs[1:])
        parts = [self.bases[int(self.offsets[i]):int(self.offsets[i + 1])] for i in idx]
        bases = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
        return ReadSet(bases, offs, dict(self.params, subset=len(idx)))


def random_genome(rng: np.random.Generator, size: int, gc: float = 0.5) -> np.ndarray:
    """i.i.d. base codes 0..3 (A, C, G, T) with P(C) = P(G) = gc / 2."""
    if gc == 0.5:
        return rng.integers(0, 4, size=size, dtype=np.uint8)
    # C or G with probability gc, then which of the pair with probability 1/2
    strong = rng.random(size) < gc
    pick = rng.integers(0, 2, size=size, dtype=np.uint8)
    return np.where(strong, 1 + pick, 3 * pick).astype(np.uint8)


def insert_repeats(rng: np.random.Generator, genome: np.ndarray, copies: int, length: int) -> None:
    """Write one random element of ``length`` bases over the genome at ``copies``
    non-overlapping uniform positions (the genome keeps its size)."""
    element = rng.integers(0, 4, size=length, dtype=np.uint8)
    slots = len(genome) // length
    for s in np.sort(rng.choice(slots, size=copies, replace=False)):
        genome[s * length:(s + 1) * length] = element


def sample_reads(rng: np.random.Generator, genome: np.ndarray, n_reads: int, read_len,
                 err: float, p_rc: float = 0.5, chunk: int = 1 << 16) -> ReadSet:
    """Reads of length ``read_len`` (an int, or an array of per-read lengths)."""
    lens = (np.full(n_reads, int(read_len), np.int64) if np.isscalar(read_len)
            else np.asarray(read_len, np.int64))
    offsets = np.zeros(n_reads + 1, np.uint64)
    np.cumsum(lens, out=offsets[1:])
    out = np.empty(int(offsets[-1]), np.uint8)
    G = len(genome)
    for c0 in range(0, n_reads, chunk):
        c1 = min(n_reads, c0 + chunk)
        for L in np.unique(lens[c0:c1]):
            sel = np.nonzero(lens[c0:c1] == L)[0] + c0
            starts = rng.integers(0, G - L + 1, size=len(sel))
            codes = genome[starts[:, None] + np.arange(L)[None, :]]
            flip = rng.random(len(sel)) < p_rc
            codes[flip] = 3 - codes[flip, ::-1]
            if err > 0:
                flat = codes.reshape(-1)
                hit = bernoulli_positions(rng, flat.size, err)
                flat[hit] = (flat[hit] + rng.integers(1, 4, size=hit.size, dtype=np.uint8)) & 3
            letters = ALPHABET[codes]
            if len(sel) == c1 - c0:
                # every read of the chunk has this length: its rows are one slice
                out[int(offsets[c0]):int(offsets[c1])] = letters.reshape(-1)
            else:
                rows = offsets[sel].astype(np.int64)
                out[rows[:, None] + np.arange(L)[None, :]] = letters
    return ReadSet(out, offsets)


def bernoulli_positions(rng: np.random.Generator, n: int, p: float) -> np.ndarray:
    """Indices in [0, n) each chosen independently with probability p, in increasing
    order.  The gaps between successive chosen indices of a Bernoulli(p) sequence are
    i.i.d. geometric(p), so the positions are the running sums of geometric draws."""
    if n == 0 or p <= 0:
        return np.zeros(0, np.int64)
    parts, pos = [], -1
    want = int(n * p + 6 * math.sqrt(n * p) + 16)
    while pos < n:
        gaps = rng.geometric(p, size=want)
        at = pos + np.cumsum(gaps)
        parts.append(at)
        pos = int(at[-1])
    at = np.concatenate(parts)
    return at[at < n]


def from_strings(reads) -> ReadSet:
    """A read set from a list of Python strings (upper-case ACGT)."""
    enc = [r.encode() for r in reads]
    offsets = np.zeros(len(enc) + 1, np.uint64)
    np.cumsum([len(e) for e in enc], out=offsets[1:])
    bases = np.frombuffer(b"".join(enc), dtype=np.uint8).copy()
    return ReadSet(bases, offsets)


# ---------------------------------------------------------------------------
# The benchmark workloads.

def plain_small(scale: float = 1.0) -> ReadSet:
    """Plain build, k = 31: 100,000-base uniform genome; 10,000 reads of length 100,
    strand p = 0.5, 1% substitution errors."""
    rng = np.random.default_rng(SEED_BASE + 0)
    g = random_genome(rng, 100_000)
    n = max(1, int(10_000 * scale))
    rs = sample_reads(rng, g, n, 100, 0.01)
    rs.params = dict(workload="plain_small_k31", genome=100_000, reads=n, read_len=100,
                     err=0.01, seed=SEED_BASE + 0)
    return rs


def plain_repeats(scale: float = 1.0) -> ReadSet:
    """Plain build, k = 31: 5,000,000-base uniform genome carrying 200 exact copies
    of one random 1,000-base element; 2,000,000 reads of length 100 (40x), strand
    p = 0.5, 0.5% substitution errors.  ``scale`` shrinks the read count only."""
    rng = np.random.default_rng(SEED_BASE + 1)
    g = random_genome(rng, 5_000_000)
    insert_repeats(rng, g, 200, 1000)
    n = max(1, int(2_000_000 * scale))
    rs = sample_reads(rng, g, n, 100, 0.005)
    rs.params = dict(workload="plain_repeats_k31", genome=5_000_000, repeats="200x1000",
                     reads=n, read_len=100, err=0.005, seed=SEED_BASE + 1)
    return rs


READ_CHUNK = 1 << 20  # reads drawn per independent seed in the chunked sampler

_shared = {}


def _fill_chunk(ci):
    """Worker: reads of chunk ci into the shared output (forked processes)."""
    sh = _shared
    r0 = ci * READ_CHUNK
    r1 = min(sh["n"], r0 + READ_CHUNK)
    rs = sample_reads(np.random.default_rng(sh["seeds"][ci]), sh["genome"], r1 - r0, sh["L"],
                      sh["err"])
    sh["out"][r0 * sh["L"]:r1 * sh["L"]] = rs.bases
    return ci


def sample_reads_chunked(seed: int, genome: np.ndarray, n_reads: int, read_len: int,
                         err: float, workers: int = 1) -> ReadSet:
    """Fixed-length reads drawn in chunks of READ_CHUNK reads, chunk i from its own
    seed (SeedSequence(seed).spawn), so the result does not depend on
    ``workers``; with workers > 1 the chunks are drawn by forked processes into
    one shared buffer (fork before the process touches a GPU)."""
    import mmap
    L = int(read_len)
    n_chunks = (n_reads + READ_CHUNK - 1) // READ_CHUNK
    seeds = np.random.SeedSequence(seed).spawn(n_chunks)
    buf = mmap.mmap(-1, max(1, n_reads * L))
    out = np.frombuffer(buf, dtype=np.uint8, count=n_reads * L)
    _shared.update(n=n_reads, L=L, err=err, genome=genome, seeds=seeds, out=out)
    try:
        _map(_fill_chunk, list(range(n_chunks)), workers)
        bases = out.copy()
    finally:
        _shared.clear()
        del out
        buf.close()
    offsets = np.arange(n_reads + 1, dtype=np.uint64) * np.uint64(L)
    return ReadSet(bases, offsets)


def plain_large(scale: float = 1.0, workers: int = 1) -> ReadSet:
    """Plain build, k = 63: 100,000,000-base genome with GC content 0.41;
    40,000,000 reads of length 150 (60x), strand p = 0.5, 1% errors.  ``scale``
    shrinks the genome and the read count together (coverage stays 60x).  Reads
    are drawn in chunks of independent seeds (``workers`` processes may draw
    them; the reads are the same for any count)."""
    rng = np.random.default_rng(SEED_BASE + 2)
    G = max(1000, int(100_000_000 * scale))
    g = random_genome(rng, G, gc=0.41)
    n = max(1, int(40_000_000 * scale))
    rs = sample_reads_chunked(SEED_BASE + 20, g, n, 150, 0.01, workers)
    rs.params = dict(workload="plain_large_k63", genome=G, reads=n, read_len=150, err=0.01,
                     gc=0.41, seed=SEED_BASE + 2)
    return rs


def _map(fn, args, workers: int):
    """fn over args in order; with workers > 1 in forked processes (each item
    draws from its own seed, so the result does not depend on the split).  Fork
    before the process touches a GPU."""
    if workers <= 1 or len(args) <= 1:
        return [fn(a) for a in args]
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    ctx = multiprocessing.get_context("fork")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        return list(ex.map(fn, args, chunksize=1))


def _batched_set(arg):
    child, scale = arg
    rng = np.random.default_rng(child)
    G = int(round(math.exp(rng.uniform(math.log(2e4), math.log(2e6)))))
    cov = rng.uniform(10, 50)
    g = random_genome(rng, G)
    n = max(1, int(round(G * cov / 100 * scale)))
    rs = sample_reads(rng, g, n, 100, 0.01)
    rs.params = dict(genome=G, coverage=cov, reads=n)
    return rs


def batched_sets(n_sets: int = 256, scale: float = 1.0, workers: int = 1) -> list:
    """Batched build, k = 31: independent read sets, each from its own genome of
    size log-uniform in [20,000, 2,000,000]; reads of length 100 at coverage
    uniform in [10x, 50x], strand p = 0.5, 1% errors."""
    root = np.random.SeedSequence(SEED_BASE + 3)
    return _map(_batched_set, [(c, scale) for c in root.spawn(n_sets)], workers)


def _pool_set(arg):
    child, scale = arg
    prng = np.random.default_rng(child)
    G = int(round(math.exp(prng.uniform(math.log(1e4), math.log(5e6)) + math.log(scale))))
    G = max(G, 1000)
    L = int(prng.choice([100, 150]))
    n = max(1, int(round(G * 30 / L)))
    rs = sample_reads(prng, random_genome(prng, G), n, L, 0.01)
    rs.params = dict(genome=G, read_len=L, reads=n)
    return rs


def served_trace(n_requests: int, rate: float = 200.0, pool_size: int = 256,
                 scale: float = 1.0, workers: int = 1):
    """Served build: Poisson arrivals (mean ``rate`` per second) of requests whose
    read sets come from a pool of ``pool_size`` sets: genome size log-uniform in
    [10,000, 5,000,000] (times ``scale``), read length 100 or 150, coverage 30x,
    1% errors, k drawn from {31, 63}.  Returns (arrival_times_s, pool_index,
    k_per_request, pool)."""
    rng = np.random.default_rng(SEED_BASE + 4)
    children = np.random.SeedSequence(SEED_BASE + 40).spawn(pool_size)
    pool = _map(_pool_set, [(c, scale) for c in children], workers)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps)
    which = rng.integers(0, pool_size, size=n_requests)
    ks = rng.choice([31, 63], size=n_requests)
    return arrivals, which, ks, pool
