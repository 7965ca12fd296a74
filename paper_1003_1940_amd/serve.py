"""Served graph construction: a request loop with continuous batching.

Requests (a read set and a k) arrive over time.  The server keeps up to ``slots``
builds in flight, each on its own HIP stream, and admits the oldest waiting
request as soon as a slot is free and the device memory that the request needs
(its reads, workspace and output tables, all computed from the read lengths
before launch) fits in what the in-flight builds leave of the HBM budget.  Builds
of different sizes and k therefore overlap on the device: a small request that
arrives behind a large one starts while the large one is still running, instead
of waiting for it as in a first-in first-out queue of single builds.

Every admitted request gets device-resident buffers of its own for its whole
life: its reads are copied from pinned host memory on its stream and packed there
(``dbg_pack_ascii``), then built (``dbg_build``); a timing event recorded after
the build marks completion.  Results stay on the device until the caller drops
them (``keep_results``).  The computation is the plain build's, launch for
launch, so a request's tables do not depend on what else is in flight.

Latency is measured from the request's arrival to its completion event on the
device clock, both against one reference event recorded when the loop starts.
"""

from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api


@dataclass
class Request:
    rid: int
    bases: torch.Tensor        # pinned uint8 ASCII reads
    offsets: torch.Tensor      # pinned int64 read offsets (n_reads + 1)
    k: int
    arrival_s: float           # seconds after the loop starts
    n_kmers: int = 0
    need_bytes: int = 0
    admit_s: float = -1.0      # host time of admission
    done_s: float = -1.0       # device time of completion
    slot: int = -1
    graph: api.Graph | None = None
    status: int = -1
    _bufs: dict = field(default_factory=dict, repr=False)
    _done: torch.cuda.Event | None = field(default=None, repr=False)

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def pin_read_set(bases: np.ndarray, offsets: np.ndarray):
    """Copy a host read set into pinned (page-locked) host tensors."""
    b = torch.empty(max(1, len(bases)), dtype=torch.uint8, pin_memory=True)
    b[:len(bases)].copy_(torch.from_numpy(np.ascontiguousarray(bases, np.uint8)))
    o = torch.empty(len(offsets), dtype=torch.int64, pin_memory=True)
    o.copy_(torch.from_numpy(np.ascontiguousarray(offsets, np.uint64).view(np.int64)))
    return b[:len(bases)], o


def request_bytes(n_bases: int, n_reads: int, n_kmers: int, k: int, zkey: bool) -> int:
    """Device bytes one build holds while in flight: ASCII staging, packed reads,
    offsets, workspace, output tables at the worst-case capacity (one row per
    k-mer position), result record; each rounded up to the allocator's 512-byte
    blocks."""
    def r(x):
        return (int(x) + 511) // 512 * 512
    w = 8 * api.key_words(k)
    cap = max(n_kmers, 1)
    out = r(cap * w) + r(cap * 4) + 2 * r(cap * w) + r(cap) + r(cap * 4)
    if zkey:
        out += r(cap * w)
    return (r(max(n_bases, 1)) + r(max(1, (n_bases + 31) // 32) * 8) + r((n_reads + 1) * 8)
            + r(api.workspace_bytes(n_reads, 1, n_kmers, k)) + out + 2 * r(24))


class Server:
    """Continuous-batching request loop over ``dbg_build`` on one GPU.

    ``slots`` streams bound the builds in flight; ``hbm_budget`` (bytes) bounds
    the device memory they hold together (default: 80% of the free HBM when the
    server is created).  ``slots=1`` gives the first-in first-out server that
    runs one build at a time."""

    def __init__(self, slots: int = 8, hbm_budget: int | None = None, device: int = 0,
                 keep_results: bool = False, zkey: bool = False, poll_s: float = 50e-6):
        if not torch.cuda.is_available():
            raise RuntimeError("the served build needs a GPU")
        api.load()
        self.dev = torch.device("cuda", device)
        self.slots = slots
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(slots)]
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            hbm_budget = int(free * 0.8)
        self.budget = int(hbm_budget)
        self.keep_results = keep_results
        self.zkey = zkey
        self.poll_s = poll_s

    def _launch(self, req: Request, slot: int):
        s = self.streams[slot]
        n_bases = int(req.bases.numel())
        n_reads = int(req.offsets.numel()) - 1
        with torch.cuda.stream(s):
            ascii_d = req.bases.to(self.dev, non_blocking=True)
            offs = req.offsets.to(self.dev, non_blocking=True)
            if n_bases:
                packed, pres = api.pack(ascii_d, s)
            else:
                packed = torch.zeros(1, dtype=torch.int64, device=self.dev)
                pres = torch.zeros(3, dtype=torch.int64, device=self.dev)
            ws = api.Workspace(n_reads, 1, req.n_kmers, req.k, self.dev)
            out = api.alloc_outputs(req.k, req.n_kmers, req.n_kmers, self.dev, self.zkey)
            result = torch.zeros(3, dtype=torch.int64, device=self.dev)
            api.build_async(packed, n_bases, offs, req.k, req.n_kmers, out, req.n_kmers,
                            req.n_kmers, result, ws, s)
            done = torch.cuda.Event(enable_timing=True)
            done.record(s)
        req._bufs = dict(ascii=ascii_d, offs=offs, packed=packed, pres=pres, ws=ws, out=out,
                         result=result)
        req._done = done
        req.slot = slot

    def _retire(self, req: Request, t0: torch.cuda.Event):
        req.done_s = t0.elapsed_time(req._done) / 1e3
        b = req._bufs
        n_nodes, n_edges, status = api.read_result(b["result"])
        _, _, pst = api.read_result(b["pres"])
        req.status = pst if pst else status
        if self.keep_results:
            o = b["out"]
            req.graph = api.Graph(req.k, o["node_kmer"], o["node_count"], o["edge_u"],
                                  o["edge_v"], o["edge_orient"], o["edge_mult"], o["edge_zkey"],
                                  n_nodes, n_edges, req.status)
        req._bufs = {}
        req._done = None

    def run(self, requests: list) -> dict:
        """Serve ``requests`` (sorted by arrival) in real time; returns statistics.
        Each request's ``done_s``, ``status`` (and ``graph`` with keep_results)
        are filled in."""
        for r in requests:
            lens = np.diff(r.offsets.numpy())
            r.n_kmers = int(np.maximum(lens - r.k + 1, 0).sum()) if len(lens) else 0
            r.need_bytes = request_bytes(int(r.bases.numel()), len(lens), r.n_kmers, r.k,
                                         self.zkey)
            if r.need_bytes > self.budget:
                raise ValueError(f"request {r.rid} needs {r.need_bytes} bytes, more than the "
                                 f"HBM budget {self.budget}")
        pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        waiting: deque = deque()
        inflight: dict = {}
        free_slots = list(range(self.slots))[::-1]
        used = 0
        peak_inflight = 0
        busy_integral = 0.0
        t0 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(self.dev)
        t0.record(torch.cuda.current_stream(self.dev))
        torch.cuda.synchronize(self.dev)
        host0 = time.perf_counter()
        last = 0.0
        while pending or waiting or inflight:
            now = time.perf_counter() - host0
            busy_integral += len(inflight) * (now - last)
            last = now
            while pending and pending[0].arrival_s <= now:
                waiting.append(pending.popleft())
            progressed = False
            for slot, req in list(inflight.items()):
                if req._done.query():
                    self._retire(req, t0)
                    used -= req.need_bytes
                    del inflight[slot]
                    free_slots.append(slot)
                    progressed = True
            while waiting and free_slots and used + waiting[0].need_bytes <= self.budget:
                req = waiting.popleft()
                slot = free_slots.pop()
                req.admit_s = time.perf_counter() - host0
                self._launch(req, slot)
                inflight[slot] = req
                used += req.need_bytes
                progressed = True
            peak_inflight = max(peak_inflight, len(inflight))
            if not progressed:
                if not inflight and not waiting and pending:
                    time.sleep(max(0.0, min(pending[0].arrival_s - now, 1e-3)))
                else:
                    time.sleep(self.poll_s)
        span = max(r.done_s for r in requests) - min(r.arrival_s for r in requests) \
            if requests else 0.0
        return dict(makespan_s=span, peak_inflight=peak_inflight,
                    mean_inflight=busy_integral / max(last, 1e-9))


def summarize(requests: list, skip: int = 0) -> dict:
    """p50 / p99 latency and k-mer throughput over requests[skip:] (by arrival)."""
    rs = sorted(requests, key=lambda r: r.arrival_s)[skip:]
    if not rs:
        return {}
    lat = np.array([r.latency_s for r in rs]) * 1e3
    span = max(r.done_s for r in rs) - min(r.arrival_s for r in rs)
    kmers = sum(r.n_kmers for r in rs)
    return dict(requests=len(rs), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                max_ms=float(lat.max()), kmers=int(kmers), span_s=float(span),
                kmers_per_s=float(kmers / span) if span > 0 else None,
                failed=int(sum(1 for r in rs if r.status != 0)))
