"""Autotuner of the build's run-time knobs.

Every knob of ``dbg_tuning_t`` leaves the tables unchanged and moves only the
time: the node-table route (k-mers or edge endpoints), the in-tile partition
level for 128-bit keys (on or off), the workgroup shape of the
LDS bucket sort (512 threads with the largest batch; 256 threads with half the
batch and two workgroups per CU; or the largest batch with 768 threads for
64-bit keys, 1,024 for 128-bit keys) and the bias of the first partition's digit
width inside a batch.  ``tune`` builds one input under every candidate setting,
checks that all of them produce bit-identical tables, times each, and returns
the fastest.  ``TuneCache`` keeps the choices in a JSON file keyed by an input
class (key width, and the k-mer count and coverage rounded to powers of two) so
that later builds of similar inputs can ``apply`` them without tuning again.
"""

from __future__ import annotations

import itertools
import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import api

DEFAULT = {"node_path": api.NODES_AUTO, "endpoint_ratio": 0.6, "local_variant": 2,
           "lds_digit_bias": 0, "in_tile": 1}


def candidates(node_paths=(api.NODES_KMERS, api.NODES_ENDPOINTS), local_variants=(0, 1, 2),
               biases=(-1, 0, 1), in_tiles=(1,)) -> list:
    """Every combination of the given values (18 by default; ``tune`` adds
    in_tile 0 for 128-bit keys, where the in-tile level exists: 36)."""
    return [dict(DEFAULT, node_path=n, local_variant=v, lds_digit_bias=b, in_tile=t)
            for n, v, b, t in itertools.product(node_paths, local_variants, biases, in_tiles)]


def input_class(n_kmers: int, n_bases: int, k: int, genome_hint: int | None = None) -> str:
    """Cache key: key width, log2 of the k-mer positions, and (when the caller
    knows it) log2 of the coverage."""
    w = "u64" if k <= 31 else "u128"
    s = f"{w}/n2^{int(math.log2(max(n_kmers, 1)))}"
    if genome_hint:
        s += f"/cov2^{int(round(math.log2(max(n_bases / genome_hint, 1e-9))))}"
    return s


@dataclass
class TuneResult:
    best: dict
    timings_ms: list            # (setting, median ms, took endpoint route)
    default_ms: float | None
    input_class: str
    extra: dict = field(default_factory=dict)

    @property
    def best_ms(self) -> float:
        return min(t for _, t, _ in self.timings_ms)


def _snapshot(out, n_nodes, n_edges):
    keep = {}
    for name, t in out.items():
        if t is None:
            continue
        n = n_nodes if name.startswith("node") else n_edges
        keep[name] = t[:n].clone()
    return keep


def _same(a: dict, b: dict) -> bool:
    import torch
    return a.keys() == b.keys() and all(torch.equal(a[n], b[n]) for n in a)


def tune(bases: np.ndarray, offsets: np.ndarray, k: int, settings: list | None = None,
         reps: int = 3, genome_hint: int | None = None, device="cuda") -> TuneResult:
    """Time one build of (bases, offsets) under each setting (median of ``reps``
    after one warm-up build) and return the fastest.  Raises if any setting's
    tables differ from the first setting's.  The process-wide tuning is restored
    afterwards."""
    import torch
    if settings is None:
        settings = candidates(in_tiles=(1, 0) if k > 31 else (1,))
    offsets = np.asarray(offsets, np.uint64)
    n_k, _ = api.bounds(offsets, k)
    packed, offs, n_bases = api.upload(bases, offsets, device)
    out = api.alloc_outputs(k, n_k, n_k, device, zkey=True)
    ws = api.Workspace(len(offsets) - 1, 1, n_k, k, device)
    result = torch.zeros(3, dtype=torch.int64, device=device)
    stream = torch.cuda.current_stream()
    saved = api.get_tuning()
    timings, ref = [], None

    def run_once():
        api.build_async(packed, n_bases, offs, k, n_k, out, n_k, n_k, result, ws, stream)

    try:
        for st in [DEFAULT] + list(settings):
            api.set_tuning(**st)
            run_once()
            torch.cuda.synchronize()
            n_nodes, n_edges, status = api.read_result(result)
            if status != 0:
                raise api.DbgError(status, f"tuning build {st}")
            snap = _snapshot(out, n_nodes, n_edges)
            if ref is None:
                ref = snap
            elif not _same(ref, snap):
                raise AssertionError(f"setting {st} changed the tables")
            took = bool(api.read_flags(result) & api.FLAG_NODES_FROM_ENDPOINTS)
            ts = []
            for _ in range(reps):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                run_once()
                b.record(stream)
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b))
            timings.append((dict(st), float(np.median(ts)), took))
    finally:
        api.set_tuning(**saved)
    default_ms = timings[0][1]
    cands = timings[1:] if len(timings) > 1 else timings
    best = min(cands, key=lambda x: x[1])[0]
    return TuneResult(best, cands, default_ms, input_class(n_k, n_bases, k, genome_hint),
                      extra={"n_kmers": n_k, "n_bases": n_bases})


class TuneCache:
    """Choices per input class, kept in a JSON file."""

    def __init__(self, path: str):
        self.path = path
        self.entries = {}
        if os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
            self.entries = {k: v for k, v in data.get("entries", {}).items()}

    def record(self, r: TuneResult):
        self.entries[r.input_class] = {"setting": r.best, "best_ms": r.best_ms,
                                       "default_ms": r.default_ms}

    def lookup(self, n_kmers: int, n_bases: int, k: int, genome_hint: int | None = None):
        e = self.entries.get(input_class(n_kmers, n_bases, k, genome_hint))
        return None if e is None else dict(e["setting"])

    def save(self):
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"entries": self.entries}, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def apply(self, n_kmers: int, n_bases: int, k: int, genome_hint: int | None = None) -> dict:
        """Set the process-wide tuning for an input of this class (the library's
        defaults when the class was never tuned); returns what was set."""
        st = self.lookup(n_kmers, n_bases, k, genome_hint) or dict(DEFAULT)
        return api.set_tuning(**st)
