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
(``dbg_pack_ascii``), then built (``dbg_build``); an event recorded after the
build marks completion.  The computation is the plain build's, launch for launch,
so a request's tables do not depend on what else is in flight.  Results are
dropped when the request completes unless ``keep_results`` asks to keep them:
"device" keeps the output tables on the device and keeps their bytes charged to
the HBM budget (``Request.release()`` gives them back), "host" copies them to
host memory and releases the device budget.

Failures stay with their request: a request that needs more than the budget
(alone, or beside the results kept on the device) is rejected, one whose device
memory cannot be allocated fails, a waiting request can be cancelled
(``Request.cancel()``, or a ``deadline_s`` after arrival), and the loop goes on
with the others.  Waiting requests are admitted in arrival order, except that a
smaller request may pass one that does not fit yet, at most ``max_bypass`` times
for any one request.

Latency is measured on the host clock, from the request's arrival to the first
poll of the loop that finds its completion event done.
"""

from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api


# Request.status: a build's dbg_status (0 = DBG_OK), or one of the server's own
# outcomes (negative).
PENDING = -1       # not finished
REJECTED = -2      # needs more device memory than the budget leaves it
ALLOC_FAILED = -3  # its device buffers could not be allocated
CANCELLED = -4     # cancelled (or past its deadline) while waiting


@dataclass
class Request:
    rid: int
    bases: torch.Tensor        # pinned uint8 ASCII reads
    offsets: torch.Tensor      # pinned int64 read offsets (n_reads + 1)
    k: int
    arrival_s: float           # seconds after the loop starts
    deadline_s: float | None = None  # cancelled if still waiting this long after arrival
    n_kmers: int = 0
    need_bytes: int = 0
    out_bytes: int = 0         # the output tables' share of need_bytes
    admit_s: float = -1.0      # host time of admission
    done_s: float = -1.0       # host time the loop saw the build complete
    slot: int = -1
    graph: api.Graph | None = None
    status: int = PENDING
    error: str | None = None
    bypassed: int = 0          # later requests admitted while this one waited
    _bufs: dict = field(default_factory=dict, repr=False)
    _done: torch.cuda.Event | None = field(default=None, repr=False)
    _cancel: bool = field(default=False, repr=False)
    _server: "Server | None" = field(default=None, repr=False)

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s

    def cancel(self):
        """Cancel the request if it is still waiting (no effect once admitted)."""
        self._cancel = True

    def release(self):
        """Drop results kept on the device and give their bytes back to the
        server's budget."""
        if self._server is not None and self.graph is not None and self.out_bytes:
            self._server.kept -= self.out_bytes
        self.graph = None
        self._server = None


def pin_read_set(bases: np.ndarray, offsets: np.ndarray):
    """Copy a host read set into pinned (page-locked) host tensors."""
    b = torch.empty(max(1, len(bases)), dtype=torch.uint8, pin_memory=True)
    b[:len(bases)].copy_(torch.from_numpy(np.ascontiguousarray(bases, np.uint8)))
    o = torch.empty(len(offsets), dtype=torch.int64, pin_memory=True)
    o.copy_(torch.from_numpy(np.ascontiguousarray(offsets, np.uint64).view(np.int64)))
    return b[:len(bases)], o


def _r(x):
    return (int(x) + 511) // 512 * 512


def output_bytes(n_kmers: int, k: int, zkey: bool) -> int:
    """Device bytes of one build's output tables at the worst-case capacity (one
    row per k-mer position), rounded up to the allocator's 512-byte blocks."""
    w = 8 * api.key_words(k)
    cap = max(n_kmers, 1)
    out = _r(cap * w) + _r(cap * 4) + 2 * _r(cap * w) + _r(cap) + _r(cap * 4)
    return out + (_r(cap * w) if zkey else 0)


def request_bytes(n_bases: int, n_reads: int, n_kmers: int, k: int, zkey: bool) -> int:
    """Device bytes one build holds while in flight: ASCII staging, packed reads,
    offsets, workspace, output tables, result records."""
    return (_r(max(n_bases, 1)) + _r(max(1, (n_bases + 31) // 32) * 8) + _r((n_reads + 1) * 8)
            + _r(api.workspace_bytes(n_reads, 1, n_kmers, k)) + output_bytes(n_kmers, k, zkey)
            + 2 * _r(24))


class Server:
    """Continuous-batching request loop over ``dbg_build`` on one GPU.

    ``slots`` streams bound the builds in flight; ``hbm_budget`` (bytes) bounds
    the device memory they hold together with the results kept on the device
    (default: 80% of the free HBM when the server is created).  ``slots=1``
    gives the first-in first-out server that runs one build at a time.
    ``keep_results``: False (drop the tables), "device" or "host" (see the
    module notes; True means "device")."""

    def __init__(self, slots: int = 8, hbm_budget: int | None = None, device: int = 0,
                 keep_results=False, zkey: bool = False, poll_s: float = 50e-6,
                 max_bypass: int = 8):
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
        self.keep = "device" if keep_results is True else (keep_results or None)
        if self.keep not in (None, "device", "host"):
            raise ValueError("keep_results must be False, True, 'device' or 'host'")
        self.zkey = zkey
        self.poll_s = poll_s
        self.max_bypass = max_bypass
        self.kept = 0  # bytes of results kept on the device

    def _launch(self, req: Request, slot: int) -> bool:
        """Allocate the request's buffers and enqueue its build on the slot's
        stream.  On an allocation failure (or a build refused on the host) the
        request fails, whatever it allocated is dropped, and False is returned."""
        s = self.streams[slot]
        n_bases = int(req.bases.numel())
        n_reads = int(req.offsets.numel()) - 1
        try:
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
                done = torch.cuda.Event()
                done.record(s)
        except torch.cuda.OutOfMemoryError as e:
            req.status, req.error = ALLOC_FAILED, f"device memory: {e}".splitlines()[0]
        except api.DbgError as e:
            req.status, req.error = e.code, str(e)
        if req.status != PENDING:
            s.synchronize()  # nothing of the request is left in flight
            torch.cuda.empty_cache()
            return False
        req._bufs = dict(ascii=ascii_d, offs=offs, packed=packed, pres=pres, ws=ws, out=out,
                         result=result)
        req._done = done
        req.slot = slot
        return True

    def _retire(self, req: Request, now: float):
        req.done_s = now
        b = req._bufs
        n_nodes, n_edges, status = api.read_result(b["result"])
        _, _, pst = api.read_result(b["pres"])
        req.status = pst if pst else status
        if self.keep:
            o = b["out"]
            g = api.Graph(req.k, o["node_kmer"], o["node_count"], o["edge_u"], o["edge_v"],
                          o["edge_orient"], o["edge_mult"], o["edge_zkey"], n_nodes, n_edges,
                          req.status)
            if self.keep == "host":
                nn, ne = min(n_nodes, o["node_count"].numel()), min(n_edges, o["edge_mult"].numel())
                cut = {"node_kmer": nn, "node_count": nn, "edge_u": ne, "edge_v": ne,
                       "edge_orient": ne, "edge_mult": ne, "edge_zkey": ne}
                h = {f: (o[f][:n].cpu() if o[f] is not None else None) for f, n in cut.items()}
                g = api.Graph(req.k, h["node_kmer"], h["node_count"], h["edge_u"], h["edge_v"],
                              h["edge_orient"], h["edge_mult"], h["edge_zkey"], n_nodes, n_edges,
                              req.status)
            else:
                self.kept += req.out_bytes
                req._server = self
            req.graph = g
        req._bufs = {}
        req._done = None

    def run(self, requests: list, on_retire=None) -> dict:
        """Serve ``requests`` (sorted by arrival) in real time; returns statistics.
        Each request's ``done_s`` and ``status`` (and ``graph`` when results are
        kept) are filled in; ``on_retire(req)`` is called as each one finishes,
        and may cancel waiting requests."""
        for r in requests:
            r.n_kmers, _ = api.bounds(r.offsets.numpy().view(np.uint64), r.k)
            r.out_bytes = output_bytes(r.n_kmers, r.k, self.zkey)
            r.need_bytes = request_bytes(int(r.bases.numel()), int(r.offsets.numel()) - 1,
                                         r.n_kmers, r.k, self.zkey)
            r.status, r.error, r.bypassed, r._cancel = PENDING, None, 0, False
        pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        waiting: list = []
        inflight: dict = {}
        free_slots = list(range(self.slots))[::-1]
        used = 0
        peak_inflight = 0
        busy_integral = 0.0
        torch.cuda.synchronize(self.dev)
        host0 = time.perf_counter()
        last = 0.0

        def finish(req, status, error, now):
            req.status, req.error, req.done_s = status, error, now
            if on_retire is not None:
                on_retire(req)

        while pending or waiting or inflight:
            now = time.perf_counter() - host0
            busy_integral += len(inflight) * (now - last)
            last = now
            while pending and pending[0].arrival_s <= now:
                waiting.append(pending.popleft())
            progressed = False
            for slot, req in list(inflight.items()):
                if req._done.query():
                    self._retire(req, time.perf_counter() - host0)
                    used -= req.need_bytes
                    del inflight[slot]
                    free_slots.append(slot)
                    progressed = True
                    if on_retire is not None:
                        on_retire(req)
            # drop what can never run: cancelled or past its deadline, or larger
            # than the budget leaves beside the results kept on the device
            for req in list(waiting):
                if req._cancel or (req.deadline_s is not None
                                   and now - req.arrival_s > req.deadline_s):
                    waiting.remove(req)
                    finish(req, CANCELLED, "cancelled while waiting", now)
                elif req.need_bytes > self.budget or (req.need_bytes > self.budget - self.kept
                                                      and not inflight):
                    waiting.remove(req)
                    finish(req, REJECTED, f"needs {req.need_bytes} bytes; the budget leaves "
                                          f"{self.budget - self.kept}", now)
            # admission: in arrival order; a request that does not fit yet may be
            # passed by smaller ones until it has been passed max_bypass times
            i = 0
            while i < len(waiting) and free_slots:
                req = waiting[i]
                if used + self.kept + req.need_bytes <= self.budget:
                    waiting.pop(i)
                    slot = free_slots.pop()
                    req.admit_s = time.perf_counter() - host0
                    for older in waiting[:i]:
                        older.bypassed += 1
                    if self._launch(req, slot):
                        inflight[slot] = req
                        used += req.need_bytes
                    else:
                        free_slots.append(slot)
                        finish(req, req.status, req.error, time.perf_counter() - host0)
                    progressed = True
                    continue
                if req.bypassed >= self.max_bypass:
                    break  # it waits for room; nothing behind it goes first
                i += 1
            peak_inflight = max(peak_inflight, len(inflight))
            if not progressed:
                if not inflight and not waiting and pending:
                    time.sleep(max(0.0, min(pending[0].arrival_s - now, 1e-3)))
                else:
                    time.sleep(self.poll_s)
        done = [r for r in requests if r.done_s >= 0]
        span = (max(r.done_s for r in done) - min(r.arrival_s for r in requests)) if done else 0.0
        return dict(makespan_s=span, peak_inflight=peak_inflight,
                    mean_inflight=busy_integral / max(last, 1e-9),
                    rejected=sum(r.status == REJECTED for r in requests),
                    alloc_failed=sum(r.status == ALLOC_FAILED for r in requests),
                    cancelled=sum(r.status == CANCELLED for r in requests))


def summarize(requests: list, skip: int = 0) -> dict:
    """p50 / p99 latency and k-mer throughput over the completed requests among
    requests[skip:] (by arrival); the others are counted as failed."""
    every = sorted(requests, key=lambda r: r.arrival_s)[skip:]
    rs = [r for r in every if r.status == 0]
    if not rs:
        return {"requests": 0, "failed": len(every)}
    lat = np.array([r.latency_s for r in rs]) * 1e3
    span = max(r.done_s for r in rs) - min(r.arrival_s for r in rs)
    kmers = sum(r.n_kmers for r in rs)
    return dict(requests=len(rs), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                max_ms=float(lat.max()), kmers=int(kmers), span_s=float(span),
                kmers_per_s=float(kmers / span) if span > 0 else None,
                failed=len(every) - len(rs))
