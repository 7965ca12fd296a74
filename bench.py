#!/usr/bin/env python3
"""Benchmark of the bi-directed de Bruijn graph build on one MI355X.

A step is one full build (edge table and node table) of the 40,000,000-read,
k = 63 workload (100,000,000-base genome with GC content 0.41, reads of length
150 at 60x, 1% substitutions: 3.52 G k-mer positions, 128-bit keys), inputs
already packed and resident in HBM.  Prints one JSON line: k-mers/s, the
roofline of the dominant kernel (timed live with per-stage HIP events on the
build stream), the HBM traffic of the sort + reduce stages, and the oracle timed
on a bounded sample of the same reads on the host.  The same line carries, as
extra keys, the 2,000,000-read k = 31 build, the batched build of 256 read sets
against per-set builds, and the served build against a first-in first-out loop
(``--no-extras`` leaves them out).

Other modes: ``--batched``, ``--served``, ``--slices N`` (their own lines),
``--copy-calibration`` (the copy that scales the HBM counters), and
``--summarize-counters`` / ``--summarize-stats``, which turn rocprofv3 output
into the summaries kept under profiles/.
"""

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (generator, k, key bytes)
    "plain_repeats_k31": ("plain_repeats", 31),
    "plain_small_k31": ("plain_small", 31),
    "plain_large_k63": ("plain_large", 63),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


STAGE_EVENTS = 24  # DBG_STAGE_EVENTS: 12 per table


def stage_names():
    """The intervals between a table's stage events (see dbg_set_stage_events)."""
    return ["start", "offsets", "enum_hist", "plan", "enum_scatter", "levels_in_tile",
            "seg_sort", "levels_rest", "local_sort", "emit_count", "emit_write", "end"]


def table_stages(intervals):
    """Stage times of one table from its event intervals {name: ms}: the
    partition levels before and after the digit-range bucket sort are one stage
    ("levels"); the bucket sort is its two launches, the digit ranges of in-tile
    buckets ("seg_sort") and the other batches ("local_sort_rest"), whose sum is
    "local_sort"."""
    out = {}
    for n in ("offsets", "enum_hist", "plan", "enum_scatter"):
        out[n] = intervals[n]
    out["levels"] = intervals["levels_in_tile"] + intervals["levels_rest"]
    out["seg_sort"] = intervals["seg_sort"]
    out["local_sort_rest"] = intervals["local_sort"]
    out["local_sort"] = intervals["seg_sort"] + intervals["local_sort"]
    for n in ("emit_count", "emit_write", "end"):
        out[n] = intervals[n]
    return out


def algorithmic_bytes(stage, n_keys, n_unique, n_bases, n_reads, w, row_bytes):
    """Bytes a kernel must move at minimum (reads of its inputs + writes of its
    outputs), per launch."""
    if stage == "enum_hist":
        return n_bases / 4 + 16 * n_reads
    if stage == "enum_scatter":
        return n_bases / 4 + 16 * n_reads + n_keys * w
    if stage == "local_sort":  # keys in; distinct keys, their 32-bit counts and the run bitmap out
        return n_keys * w + n_unique * (w + 4) + n_keys / 8
    if stage == "emit_write":  # distinct keys, counts and the bitmap in; table rows out
        return n_unique * (w + 4) + n_keys / 8 + n_unique * row_bytes
    return None


KERNEL_SOURCES = ("paper_1003_1940_amd/csrc/dbg_kernels.hip",
                  "paper_1003_1940_amd/csrc/dbg_device.h",
                  "paper_1003_1940_amd/csrc/dbg_internal.h")


def kernel_source_hash():
    """sha256 over the kernel sources: counter readings taken on other sources are
    not reported as this build's traffic."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def run_copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of known size, for scaling the HBM counters."""
    import torch
    dev = torch.device("cuda", 0)
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(7)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def run_cpu_baseline(rs, k, target_s=12.0):
    """The oracle, as is, on a bounded prefix of the reads (host cores): prefixes
    grow until one takes a second or more, then one prefix sized for about
    target_s seconds is timed."""
    import oracle
    oracle.build(force=False)
    threads = oracle.host_threads(0)
    n = 2000

    def timed(n_):
        sub_ = rs.subset(np.arange(min(n_, rs.n_reads)))
        t0 = time.perf_counter()
        oracle.build_graph(sub_.bases, sub_.offsets, k, threads=threads)
        return sub_, time.perf_counter() - t0

    while True:
        sub, dt = timed(n)
        if dt >= 1.0 or n >= rs.n_reads:
            break
        n = int(min(rs.n_reads, n * max(2.0, min(8.0, 1.5 / max(dt, 1e-3)))))
    if n < rs.n_reads:
        sub, dt = timed(int(min(rs.n_reads, n * target_s / dt)))
    kmers = sub.kmer_count(k)
    return {"value": kmers / dt, "unit": "k-mers/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sub.n_reads} reads of the workload ({kmers} k-mer positions), "
                      f"{dt:.1f} s wall", "cpu": cpu_model()}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), for the baseline record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_batched(args):
    """256 independent read sets (batched-build workload): one dbg_build_batched
    launch sequence against 256 sequential dbg_build calls on the same stream."""
    import torch
    from paper_1003_1940_amd import api, synth
    k = 31
    log(f"generating {args.n_sets} read sets (scale {args.scale})")
    sets = synth.batched_sets(n_sets=args.n_sets, scale=args.scale,
                              workers=max(1, min(16, os.cpu_count() or 1)))
    bases = np.concatenate([s.bases for s in sets])
    lens = np.concatenate([np.diff(s.offsets.astype(np.int64)) for s in sets])
    offsets = np.zeros(len(lens) + 1, np.uint64)
    np.cumsum(lens, out=offsets[1:])
    sro = np.zeros(len(sets) + 1, np.uint64)
    np.cumsum([s.n_reads for s in sets], out=sro[1:])
    set_kmers = [s.kmer_count(k) for s in sets]
    n_k = int(sum(set_kmers))
    log(f"{len(sets)} sets, {len(lens)} reads, {int(offsets[-1])} bases, {n_k} k-mers")
    dev = torch.device("cuda", 0)
    packed, offs, n_bases = api.upload(bases, offsets, dev)
    sets_d = torch.from_numpy(sro.view(np.int64).copy()).to(dev)
    out = api.alloc_outputs(k, n_k, n_k, dev, zkey=True)
    ws = api.Workspace(len(lens), len(sets), n_k, k, dev)
    nso = torch.zeros(len(sets) + 1, dtype=torch.int64, device=dev)
    eso = torch.zeros(len(sets) + 1, dtype=torch.int64, device=dev)
    res = torch.zeros(3, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def batched():
        api.build_async(packed, n_bases, offs, k, n_k, out, n_k, n_k, res, ws, stream,
                        set_offsets=sets_d, node_set_offsets=nso, edge_set_offsets=eso)

    # plain per-set builds: each set's reads are a slice of the same device stream
    per = []
    max_keys = max(set_kmers)
    max_reads = max(s.n_reads for s in sets)
    ws1 = api.Workspace(max_reads, 1, max_keys, k, dev)
    out1 = api.alloc_outputs(k, max_keys, max_keys, dev, zkey=True)
    res1 = torch.zeros(3, dtype=torch.int64, device=dev)
    set_offs, set_packed = [], []
    for i, srs in enumerate(sets):
        p, o, nb = api.upload(srs.bases, srs.offsets, dev)
        set_packed.append((p, o, nb))

    def plain_all():
        for (p, o, nb), kk in zip(set_packed, set_kmers):
            api.build_async(p, nb, o, k, kk, out1, kk, kk, res1, ws1, stream)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    log("timing batched")
    t_b = timed(batched, args.steps, args.warmup)
    n_nodes, n_edges, status = api.read_result(res)
    if status:
        raise SystemExit(f"device status {status}: {api.strerror(status)}")
    log("timing plain per-set builds")
    t_p = timed(plain_all, max(1, args.steps // 4), 1)
    del out, ws
    torch.cuda.empty_cache()
    log("capturing the batched build as a HIP graph")
    cap = api.CapturedBuild(packed, n_bases, offs, k, n_k, set_offsets=sets_d)
    t_g = timed(cap.replay, args.steps, 1)
    gn, ge, gst = api.read_result(cap.result)
    if (gn, ge, gst) != (n_nodes, n_edges, 0):
        raise SystemExit(f"graph replay gave {(gn, ge, gst)}, eager {(n_nodes, n_edges, 0)}")
    line = {
        "metric": "k-mers/s into bi-directed graph (batched build)",
        "value": n_k / (t_b / 1e3), "unit": "k-mers/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_b, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batched_k31", "sets": len(sets), "reads": int(len(lens)),
                   "kmers": n_k, "nodes": n_nodes, "edges": n_edges, "scale": args.scale},
        "plain_per_set": {"ms_for_all_sets": t_p, "value": n_k / (t_p / 1e3),
                          "unit": "k-mers/s"},
        "batched_over_plain": t_p / t_b,
        "graph_replay": {"ms": t_g, "value": n_k / (t_g / 1e3), "unit": "k-mers/s"},
    }
    del cap, set_packed, out1, ws1
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return line


def run_served(args):
    """Served-build workload: a Poisson stream of requests (mean 200/s; read sets
    from a pool of 256, k of 31 or 63) served by the continuous-batching loop and by
    a first-in first-out loop of single builds, on the same trace; then the same
    requests all at once, for the throughput each loop sustains."""
    import torch
    from paper_1003_1940_amd import synth
    from paper_1003_1940_amd.serve import Request, Server, pin_read_set, summarize
    n_req = args.requests + args.warmup_requests
    workers = max(1, min(16, os.cpu_count() or 1))
    log(f"generating the request pool (256 sets, {workers} workers) and {n_req} arrivals")
    arrivals, which, ks, pool = synth.served_trace(n_req, rate=args.rate, pool_size=256,
                                                   scale=args.scale, workers=workers)
    log(f"pool: {sum(p.n_bases for p in pool)} bases; pinning")
    pinned = [pin_read_set(p.bases, p.offsets) for p in pool]
    del pool

    def trace(burst):
        return [Request(i, pinned[w][0], pinned[w][1], int(k), 0.0 if burst else float(a))
                for i, (a, w, k) in enumerate(zip(arrivals, which, ks))]

    out = {}
    for name, slots in (("continuous", args.slots), ("fifo", 1)):
        for burst in (False, True):
            reqs = trace(burst)
            log(f"{name} ({slots} slots), {'all at once' if burst else 'Poisson arrivals'}")
            st = Server(slots=slots).run(reqs)
            summ = summarize(reqs, skip=0 if burst else args.warmup_requests)
            summ.update(mean_inflight=round(st["mean_inflight"], 2),
                        peak_inflight=st["peak_inflight"])
            out[f"{name}_{'burst' if burst else 'poisson'}"] = summ
            log(f"  {summ}")
            del reqs
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    c, f = out["continuous_poisson"], out["fifo_poisson"]
    line = {
        "metric": "k-mers/s into bi-directed graph (served build)",
        "value": c["kmers_per_s"], "unit": "k-mers/s", "n_gpus": 1,
        "steps": args.requests, "warmup": args.warmup_requests,
        "ms_per_step": c["span_s"] * 1e3 / max(1, c["requests"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64+u128", "data": "synthetic",
        "config": {"workload": "served_poisson", "rate_per_s": args.rate, "pool": 256,
                   "requests": args.requests, "warmup_requests": args.warmup_requests,
                   "slots": args.slots, "scale": args.scale},
        "latency_ms": {"p50": c["p50_ms"], "p99": c["p99_ms"]},
        "fifo": {"p50_ms": f["p50_ms"], "p99_ms": f["p99_ms"], "kmers_per_s": f["kmers_per_s"]},
        "saturated_kmers_per_s": {"continuous": out["continuous_burst"]["kmers_per_s"],
                                  "fifo": out["fifo_burst"]["kmers_per_s"]},
        "modes": out,
    }
    return line


def run_sliced(args):
    """The out-of-memory build: the workload built in key-space slices whose keys
    fit a budget (the larger table's positions over --slices), each slice's rows
    copied to pinned host memory while the next slice builds.  Timed from reads
    resident in HBM (packed) to all rows in host memory: the prefix counts and
    the slices; the upload before and any host-side joining after are reported
    apart."""
    import torch
    from paper_1003_1940_amd import api, sliced, synth
    gen_name, k = WORKLOADS[args.workload]
    log(f"generating {args.workload} (scale {args.scale})")
    workers = max(1, min(16, os.cpu_count() or 1))
    gen = getattr(synth, gen_name)
    rs = gen(scale=args.scale, workers=workers) if gen_name == "plain_large" else gen(scale=args.scale)
    n_k = sliced.positions(rs.offsets, k)
    times = []
    for it in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        s = sliced.build_sliced(rs.bases, rs.offsets, k, n_slices=args.slices, concatenate=False)
        # reads in HBM to tables in pinned host memory: prefix counts + slices
        dt = s.seconds["prefix_counts"] + s.seconds["slices"]
        if it >= args.warmup:
            times.append((dt, s.seconds))
        log(f"run {it}: {dt * 1e3:.1f} ms, {s.seconds}")
        del s.parts
    med = sorted(times, key=lambda x: x[0])[len(times) // 2]
    one_ws = int(api.load().dbg_workspace_bytes(len(rs.offsets) - 1, 1, n_k, k))
    # the one-shot build brought to the same end state (rows in pinned host memory)
    one_ms = None
    if one_ws + 2 * n_k * 40 < torch.cuda.mem_get_info()[0]:
        packed, offs, n_bases = api.upload(rs.bases, rs.offsets)
        out = api.alloc_outputs(k, n_k, n_k, "cuda", False)
        ws = api.Workspace(len(rs.offsets) - 1, 1, n_k, k)
        res = torch.zeros(3, dtype=torch.int64, device="cuda")
        copy = torch.cuda.Stream()
        ts = []
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            api.build_async(packed, n_bases, offs, k, n_k, out, n_k, n_k, res, ws)
            n_nodes, n_edges, _ = api.read_result(res)
            copy.wait_stream(torch.cuda.current_stream())
            rows = sliced._host_rows(out, n_nodes, n_edges, copy)
            copy.synchronize()
            if it >= args.warmup:
                ts.append(time.perf_counter() - t0)
            del rows
        one_ms = round(float(np.median(ts)) * 1e3, 3)
        del out, ws
    log(f"one-shot build + rows to host: {one_ms} ms")
    line = {
        "metric": "k-mers/s into bi-directed graph (sliced, tables to host memory)",
        "value": n_k / med[0], "unit": "k-mers/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": med[0] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64" if k <= 31 else "u128",
        "data": "synthetic",
        "config": {"workload": args.workload, "scale": args.scale, "k": k, "kmers": n_k,
                   "slices_asked": args.slices, "slices": len(s.slices), "budget_keys": s.budget,
                   "nodes": int(sum(r[0] for r in s.rows)),
                   "edges": int(sum(r[1] for r in s.rows))},
        "seconds": {k_: round(v, 4) for k_, v in med[1].items()},
        "workspace_bytes": {"slice": s.workspace_bytes, "one_shot": one_ws},
        "one_shot_rows_to_host_ms": one_ms,
    }
    print(json.dumps(line), flush=True)




def plain_measure(workload, scale, steps, warmup, cap_frac, zkey, node_route="auto",
                  tune=False, after=True, cpu=True):
    """One plain build of a workload, timed: returns the bench line's fields."""
    import torch
    from paper_1003_1940_amd import api, synth

    if node_route != "auto":
        api.set_tuning(node_path={"kmers": api.NODES_KMERS,
                                  "endpoints": api.NODES_ENDPOINTS}[node_route])
    gen_name, k = WORKLOADS[workload]
    log(f"generating {workload} (scale {scale})")
    workers = max(1, min(16, os.cpu_count() or 1))
    gen = getattr(synth, gen_name)
    rs = gen(scale=scale, workers=workers) if gen_name == "plain_large" else gen(scale=scale)
    n_reads, n_bases = rs.n_reads, rs.n_bases
    n_k = rs.kmer_count(k)
    n_e = rs.kmer_count(k + 1)
    w = 8 if k <= 31 else 16
    log(f"{n_reads} reads, {n_bases} bases, {n_k} k-mers, {n_e} (k+1)-mers")

    dev = torch.device("cuda", 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    packed, offs, _ = api.upload(rs.bases, rs.offsets, dev)
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - t0
    # output capacity: one row per k-mer position unless cap_frac lowers it
    # (memory-tight mode: the build reports DBG_E_CAPACITY if it was too low)
    cap = max(1, int(n_k * cap_frac))
    out = api.alloc_outputs(k, cap, cap, dev, zkey=zkey)
    ws = api.Workspace(n_reads, 1, n_k, k, dev)
    result = torch.zeros(3, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    lib = api.load()
    lib.dbg_set_stage_events.restype = ctypes.c_int
    lib.dbg_set_stage_events.argtypes = [ctypes.c_void_p, ctypes.c_int]

    def step():
        api.build_async(packed, n_bases, offs, k, n_k, out, cap, cap, result, ws, stream)

    tuning = None
    if tune:
        from paper_1003_1940_amd import autotune
        log("autotuning (every candidate is checked to build identical tables)")
        tr = autotune.tune(rs.bases, rs.offsets, k, reps=3,
                           genome_hint=rs.params.get("genome"))
        api.set_tuning(**tr.best)
        tuning = {"best": tr.best, "best_ms": round(tr.best_ms, 4),
                  "default_ms": round(tr.default_ms, 4), "class": tr.input_class,
                  "candidates": len(tr.timings_ms)}
        log(f"tuned: {tuning}")
        torch.cuda.empty_cache()

    log(f"warmup {warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    n_nodes, n_edges, status = api.read_result(result)
    if status != 0:
        raise SystemExit(f"device status {status}: {api.strerror(status)}")

    # per-step stage events (HIP events recorded by the library on `stream`)
    NE = STAGE_EVENTS
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(NE)] for _ in range(steps)]
    for step_ev in ev:  # torch creates the HIP event on first record
        for e in step_ev:
            e.record(stream)
    torch.cuda.synchronize()
    handles = [(ctypes.c_void_p * NE)(*[e.cuda_event for e in step_ev]) for step_ev in ev]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    log(f"timing {steps} steps")
    start.record(stream)
    for s_ in range(steps):
        lib.dbg_set_stage_events(ctypes.cast(handles[s_], ctypes.c_void_p), NE)
        step()
    stop.record(stream)
    torch.cuda.synchronize()
    lib.dbg_set_stage_events(None, 0)
    ms = start.elapsed_time(stop) / steps
    n_nodes, n_edges, status = api.read_result(result)
    if status != 0:
        raise SystemExit(f"device status {status}: {api.strerror(status)}")
    node_route_run = ("endpoints" if api.read_flags(result) & api.FLAG_NODES_FROM_ENDPOINTS
                      else "kmers")

    names = stage_names()
    stages = {}
    half = NE // 2
    for tbl, base in (("edges", 0), ("nodes", half)):
        iv = {}
        for i in range(1, half):
            vals = [ev[s_][base + i - 1].elapsed_time(ev[s_][base + i]) for s_ in range(steps)]
            iv[names[i]] = float(np.mean(vals))
        for n_, v in table_stages(iv).items():
            stages[f"{tbl}.{n_}"] = v
    log("stages (ms): " + ", ".join(f"{k_}={v:.3f}" for k_, v in stages.items()))

    # dominant single-kernel stage and its roofline
    row_bytes = {"edges": (3 if zkey else 2) * w + 5, "nodes": w + 4}
    uniq = {"edges": n_edges, "nodes": n_nodes}
    keys = {"edges": n_e, "nodes": n_k}
    best = None
    for name, t in stages.items():
        tbl, st = name.split(".")
        b = algorithmic_bytes(st, keys[tbl], uniq[tbl], n_bases, n_reads, w, row_bytes[tbl])
        if b is not None and (best is None or t > best[1]):
            best = (name, t, b)
    kname, kms, kbytes = best
    achieved = kbytes / (kms / 1e3) / 1e9
    counters = read_counter_summary(workload) if scale == 1.0 and node_route == "auto" else None
    traffic = None
    if counters is not None and kname in counters.get("stages", {}):
        traffic = counters["stages"][kname]["bytes"]
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic),
                "algorithmic_bytes": round(kbytes), "ms": round(kms, 4)}

    # the sort + reduce stages: everything after the enumeration histogram until
    # the table's rows are written (bucket planning, the level-0 scatter, further
    # partition levels, the LDS bucket sort, run counting, the run-length write)
    sr_ms = sum(v for n_, v in stages.items() if n_.split(".")[1] in SORT_REDUCE_STAGES)
    sort_reduce = None
    if counters is not None and "sort_reduce" in counters:
        b = counters["sort_reduce"]["bytes"]
        sort_reduce = {"bytes": round(b), "ms": round(sr_ms, 4),
                       "achieved": round(b / (sr_ms / 1e3) / 1e9, 1), "unit": "GB/s",
                       "frac": round(b / (sr_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    build_traffic = None
    if counters is not None and "build_total" in counters:
        tb = counters["build_total"]["bytes"]
        build_traffic = {"bytes": round(tb), "achieved": round(tb / (ms / 1e3) / 1e9, 1),
                         "unit": "GB/s", "frac": round(tb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}

    # The bytes an 8-bit LSD radix sort of both tables would move (per key and
    # table: one enumeration write, one histogram read, a read and a write per
    # digit pass, one run-length read; distinct keys and counts written; the edge
    # decode read and rows written), divided by this build's time: the rate an
    # LSD implementation would have to sustain to match it.  It is not this
    # build's traffic and can exceed the HBM peak.
    def lsd_bytes(n, u, bits):
        passes = (bits + 7) // 8
        return n * w * (1 + 1 + 2 * passes + 1) + u * (w + 4)
    lsd = (lsd_bytes(n_e, n_edges, 2 * k + 2) + n_edges * (w + 4) + n_edges * (2 * w + 5)
           + lsd_bytes(n_k, n_nodes, 2 * k))
    lsd_equivalent = {"bytes": round(lsd), "rate": round(lsd / (ms / 1e3) / 1e9, 1),
                      "unit": "GB/s"}

    # STEP-4 adjacency lists and the Sec. 7 chain compaction of the built graph
    # (not part of the timed build)
    adjacency = compaction = None
    if after and status == 0 and cap_frac >= 1.0:  # memory-tight runs leave no room for them
        g = api.Graph(k, out["node_kmer"], out["node_count"], out["edge_u"], out["edge_v"],
                      out["edge_orient"], out["edge_mult"], out["edge_zkey"], n_nodes, n_edges, 0)

        def timed(fn, reps=5):
            ts, r = [], None
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                r = fn()
                e1.record(stream)
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            return float(np.median(ts)), r

        a = api.adjacency(g, edge_buckets=True)  # warm-up (and workspace sizing)
        a_ms, a = timed(lambda: api.adjacency_async(g, stream, edge_buckets=True))
        # node keys read once (index build), each edge's endpoints and orientation
        # read, the two bucket ids written, counted, read back and placed, the
        # offsets written and read, the entries written and sorted in place, the
        # node rows of both ends written
        a_bytes = (n_nodes * w + n_edges * (2 * w + 1) + 2 * n_edges * 4 * 3
                   + (2 * n_nodes + 1) * 8 * 2 + 2 * n_edges * 5 * 2 + 2 * n_edges * 4)
        adjacency = {"ms": round(a_ms, 4), "bytes": a_bytes,
                     "achieved_GBs": round(a_bytes / (a_ms / 1e3) / 1e9, 1)}
        log(f"adjacency: {adjacency}")
        c = api.compact(g, a, 3)  # warm-up, outputs reused below
        cw = c.workspace
        c_ms, _ = timed(lambda: api.compact_async(g, a, 3, stream, out=c._full, workspace=cw))
        clen = c.chain_len.to(torch.int64)
        compaction = {"ms": round(c_ms, 4), "min_nodes": 3, "chains": c.n_chains,
                      "merged_chains": int((clen >= 3).sum()),
                      "nodes_in_merged_chains": int(clen[clen >= 3].sum()),
                      "kept_edges": c.n_kept, "cycles": c.n_cyclic,
                      "longest_chain": int(clen.max()) if c.n_chains else 0,
                      "nodes_per_s": round(n_nodes / (c_ms / 1e3))}
        log(f"compaction: {compaction}")
        del a, c, g, cw
    del out, ws, packed, offs, result
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    cpu_line = None
    if cpu:
        log("cpu baseline (oracle on a bounded sample)")
        cpu_line = run_cpu_baseline(rs, k)
    if node_route != "auto":
        api.set_tuning(node_path=api.NODES_AUTO)

    return {
        "metric": "k-mers/s into bi-directed graph",
        "value": n_k / (ms / 1e3),
        "keys_per_s": (n_k + n_e) / (ms / 1e3),
        "unit": "k-mers/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64" if w == 8 else "u128",
        "data": "synthetic",
        "config": {"workload": workload, "reads": n_reads, "read_len": rs.params.get("read_len"),
                   "k": k, "genome": rs.params.get("genome"), "kmers": n_k, "kplus1mers": n_e,
                   "nodes": n_nodes, "edges": n_edges, "scale": scale,
                   "node_route": node_route_run, "output_rows": cap, "edge_zkey": zkey},
        "roofline": roofline,
        "cpu_baseline": cpu_line,
        "stages_ms": {k_: round(v, 4) for k_, v in stages.items()},
        "sort_reduce_ms": round(sr_ms, 4),
        "sort_reduce_traffic": sort_reduce,
        "build_traffic": build_traffic,
        "lsd_equivalent_rate": lsd_equivalent,
        "adjacency": adjacency,
        "compaction": compaction,
        "tuning": tuning if tuning is not None else api.get_tuning(),
        "h2d_upload_and_pack_s": round(h2d_s, 4),
    }


SORT_REDUCE_STAGES = ("plan", "enum_scatter", "levels", "local_sort", "emit_count",
                      "emit_write")


def default_cap(workload, scale):
    """Output rows as a fraction of the k-mer positions, and whether edge keys are
    exported: the full-size k = 63 build needs 0.55 and no edge keys to fit 288 GB."""
    big = workload == "plain_large_k63" and scale > 0.5
    return (0.55, False) if big else (1.0, True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_large_k63", choices=sorted(WORKLOADS))
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="leave out the extra keys (2M-read k=31 build, batched, served)")
    ap.add_argument("--batched", action="store_true",
                    help="the batched-build workload (many read sets in one launch sequence)")
    ap.add_argument("--n-sets", type=int, default=256)
    ap.add_argument("--served", action="store_true",
                    help="the served-build workload (Poisson request stream)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--warmup-requests", type=int, default=100)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--node-route", choices=("auto", "kmers", "endpoints"), default="auto",
                    help="how the node table is built (default: the library's choice)")
    ap.add_argument("--cap-frac", type=float, default=None,
                    help="output rows as a fraction of the k-mer positions (default 1; 0.55 "
                         "without edge keys for the full-size k=63 workload, which needs it "
                         "to fit 288 GB)")
    ap.add_argument("--no-zkey", action="store_true", help="do not export edge (k+1)-mer keys")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner on the workload first and time the chosen setting")
    ap.add_argument("--slices", type=int, default=0,
                    help="build in this many key-space slices, tables to host memory")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a 1 GiB device copy (scale for the HBM byte counters)")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH",
                                                               "COPY_WRITE"),
                    help="rocprofv3 --pmc output folders (FETCH_SIZE and WRITE_SIZE passes of "
                         "a bench run and of --copy-calibration): writes "
                         "profiles/hbm_traffic_<workload>.md")
    ap.add_argument("--summarize-stats", metavar="TRACE_DIR",
                    help="rocprofv3 --kernel-trace --stats output folder: writes "
                         "profiles/<workload>_kernel_stats.md")
    ap.add_argument("--command", default="",
                    help="the profiled command, recorded in the summary (with --summarize-*)")
    args = ap.parse_args()
    cap_frac, zkey = default_cap(args.workload, args.scale)
    if args.cap_frac is not None:
        cap_frac = args.cap_frac
    zkey = zkey and not args.no_zkey
    args.cap_frac, args.no_zkey = cap_frac, not zkey
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is described in DESIGN.md and not implemented.",
              file=sys.stderr)
        sys.exit(2)

    if args.summarize_counters:
        summarize_counters(args)
        return
    if args.summarize_stats:
        summarize_stats(args)
        return
    if args.copy_calibration:
        run_copy_calibration()
        return
    if args.batched:
        print(json.dumps(run_batched(args)), flush=True)
        return
    if args.served:
        print(json.dumps(run_served(args)), flush=True)
        return
    if args.slices:
        run_sliced(args)
        return

    line = plain_measure(args.workload, args.scale, args.steps, args.warmup, cap_frac, zkey,
                         args.node_route, args.tune, after=True, cpu=not args.no_cpu_baseline)
    if not args.no_extras and args.workload == "plain_large_k63":
        c2 = plain_measure("plain_repeats_k31", 1.0, args.steps, args.warmup, 1.0, True,
                           after=True, cpu=False)
        line["plain_repeats_k31"] = {k_: c2[k_] for k_ in (
            "value", "unit", "ms_per_step", "dtype", "config", "roofline", "stages_ms",
            "sort_reduce_ms", "sort_reduce_traffic", "build_traffic", "lsd_equivalent_rate",
            "adjacency", "compaction")}
        b = argparse.Namespace(**vars(args))
        b.steps, b.warmup, b.scale = 10, 2, 1.0
        bl = run_batched(b)
        line["batched"] = {k_: bl[k_] for k_ in ("value", "unit", "ms_per_step", "config",
                                                 "plain_per_set", "batched_over_plain",
                                                 "graph_replay")}
        sl = run_served(b)
        line["served"] = {k_: sl[k_] for k_ in ("value", "unit", "config", "latency_ms",
                                                "fifo", "saturated_kmers_per_s")}
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------------------
# rocprofv3 output -> the summaries under profiles/.

def _csv_rows(folder, suffix):
    import csv
    rows = []
    for root, _, files in os.walk(folder):
        for f in sorted(files):
            if f.endswith(suffix):
                with open(os.path.join(root, f), newline="") as fh:
                    # column names differ in case between rocprofv3's writers
                    rows.extend({k.lower(): v for k, v in r.items()} for r in csv.DictReader(fh))
    return rows


def _dispatches(folder):
    """Per dispatch (in dispatch order): kernel name and counter value."""
    rows = _csv_rows(folder, "counter_collection.csv")
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    key = "dispatch_id" if "dispatch_id" in rows[0] else "correlation_id"
    acc = {}
    for r in rows:
        d = int(r[key])
        acc.setdefault(d, [r["kernel_name"], 0.0])
        acc[d][1] += float(r["counter_value"])
    return [tuple(acc[d]) for d in sorted(acc)]


def _short(name):
    """Kernel name without its return type and argument list."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    depth, out = 0, []
    for ch in name:
        if ch == "(" and depth == 0:
            break
        out.append(ch)
        depth += ch == "<"
        depth -= ch == ">"
    return "".join(out).strip()


def _segment(dispatches):
    """Split the dispatches of a bench run into builds (each starts with k_init)
    and tables (each starts with k_table_reset: edges, then nodes); returns a
    list of builds, each {"edges": [(name, value)], "nodes": [...]}."""
    builds = []
    cur = None
    tbl = None
    for name, val in dispatches:
        s = _short(name)
        if s.endswith("k_init"):
            cur = {"edges": [], "nodes": []}
            builds.append(cur)
            tbl = None
            continue
        if cur is None or not s.startswith("dbg::"):
            continue
        if s.endswith("k_table_reset"):
            tbl = "edges" if tbl is None else "nodes"
        if s.endswith("k_write_result"):  # a build's last kernel: what follows is not
            cur = None                      # part of it (graph kernels timed after it)
            continue
        if tbl is not None:
            cur[tbl].append((s, val))
    return builds


# single-kernel stages (for the roofline's traffic) and the kernels of the sort +
# reduce stages (after the enumeration histogram, through the per-set rows)
SINGLE_STAGE = {"enum_hist": "k_enum_hist", "enum_scatter": "k_enum_scatter",
                "local_sort": "k_local_sort", "emit_write": "k_emit_write"}


def _stage_of(short_name):
    """The single-kernel stage a kernel is, or None."""
    base = short_name.split("::")[-1].split("<")[0]
    for st, kern in SINGLE_STAGE.items():
        if base.startswith(kern):
            return st
    return None


def _table_bytes(seq, scale):
    """One table's dispatches (name, KiB): bytes of each single-kernel stage (the
    sum over its launches: the bucket sort is launched for the digit ranges of
    in-tile buckets and for the other batches, and a table of the endpoint route
    also launches the other route's kernels, which return at once), and of the
    sort + reduce part."""
    stages, sr, inside = {}, 0.0, False
    for s, v in seq:
        b = v * 1024 * scale
        st = _stage_of(s)
        if st is not None:
            stages[st] = stages.get(st, 0.0) + b
        if inside:
            sr += b
        base = s.split("::")[-1].split("<")[0]
        if base == "k_enum_hist":
            inside = True
        elif base == "k_emit_write":
            inside = False
    return stages, sr


def summarize_counters(args):
    fetch_dir, write_dir, cfetch_dir, cwrite_dir = args.summarize_counters
    copy_bytes = 1 << 30

    def copy_scale(folder):
        d = [v for n, v in _dispatches(folder) if "copy" in n.lower()]
        if not d:
            raise SystemExit(f"no copy dispatch under {folder}")
        big = max(d)
        return copy_bytes / (big * 1024), big

    fs, fkib = copy_scale(cfetch_dir)
    ws_, wkib = copy_scale(cwrite_dir)
    per = {}  # part -> {"fetch": [per build], "write": [...]}

    def put(part, kind, b):
        per.setdefault(part, {"fetch": [], "write": []})[kind].append(b)

    n_builds = 0
    for kind, folder, scale in (("fetch", fetch_dir, fs), ("write", write_dir, ws_)):
        builds = _segment(_dispatches(folder))
        if not builds:
            raise SystemExit(f"no build found under {folder}")
        n_builds = len(builds)
        for bld in builds:
            sr_build = total = 0.0
            for tbl in ("edges", "nodes"):
                st, sr = _table_bytes(bld[tbl], scale)
                for name, b in st.items():
                    put(f"{tbl}.{name}", kind, b)
                sr_build += sr
                total += sum(v * 1024 * scale for _, v in bld[tbl])
            put("sort_reduce", kind, sr_build)
            put("build_total", kind, total)

    def mean(xs):
        return float(np.mean(xs)) if xs else 0.0

    def row(v):
        f, w_ = mean(v["fetch"]), mean(v["write"])
        return {"fetch_bytes": round(f), "write_bytes": round(w_), "bytes": round(f + w_)}

    data = {
        "workload": args.workload,
        "kernel_source_sha256": kernel_source_hash(),
        "fetch_scale": round(fs, 6), "write_scale": round(ws_, 6),
        "builds": n_builds,
        "stages": {n: row(v) for n, v in sorted(per.items())
                   if n not in ("sort_reduce", "build_total")},
        "sort_reduce": row(per["sort_reduce"]),
        "build_total": row(per["build_total"]),
    }
    lines = [f"# HBM traffic per build and per stage: {args.workload}", "",
             "Counters from two `rocprofv3 --pmc` passes over the same short benchmark run "
             "(FETCH_SIZE, then WRITE_SIZE), and the same two passes over a plain 1 GiB device "
             "copy that calibrates them.", "", "Commands (from `/tmp`, repository at "
             "`/root/repo`):", "", "```", args.command.strip(), "```", "",
             f"Calibration: the 1 GiB copy reads FETCH_SIZE = {fkib:.0f} KiB and WRITE_SIZE = "
             f"{wkib:.0f} KiB per dispatch, so fetch bytes = FETCH_SIZE x 1024 x {fs:.4f} and "
             f"write bytes = WRITE_SIZE x 1024 x {ws_:.4f}.", "",
             f"Mean over the run's {n_builds} builds (a build is every dispatch from `k_init` "
             "on; a table every dispatch from its `k_table_reset` on, edges first):", "",
             "| part | fetch GB | write GB | HBM GB |", "|---|---|---|---|"]
    for n, v in list(data["stages"].items()) + [("sort_reduce", data["sort_reduce"]),
                                                ("build_total", data["build_total"])]:
        lines.append(f"| {n} | {v['fetch_bytes'] / 1e9:.3f} | {v['write_bytes'] / 1e9:.3f} | "
                     f"{v['bytes'] / 1e9:.3f} |")
    lines += ["", "sort_reduce: both tables' kernels after the enumeration histogram through "
              "the run-length write (bucket planning and the endpoint records, the level-0 "
              "scatter, the further partition levels, the LDS bucket sort, the run counting "
              "and the writing of the rows).  build_total: every kernel of a build.", "",
              "`bench.py` reads the block below; it reports the traffic only while the "
              "kernel sources hash to `kernel_source_sha256`.", "", "```json",
              json.dumps(data, indent=1), "```", ""]
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{args.workload}.md")
    with open(path, "w") as f:
        f.write("\n".join(lines))
    print(path)


def read_counter_summary(workload):
    """The counter summary of a workload (profiles/hbm_traffic_<workload>.md), or
    None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    a = text.find("```json")
    if a < 0:
        return None
    b = text.find("```", a + 7)
    data = json.loads(text[a + 7:b])
    if data.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return data


def summarize_stats(args):
    rows = _csv_rows(args.summarize_stats, "kernel_stats.csv")
    if not rows:
        raise SystemExit(f"no kernel_stats.csv under {args.summarize_stats}")
    trace = _csv_rows(args.summarize_stats, "kernel_trace.csv")
    lines = [f"# Kernel time: {args.workload}", "",
             "rocprofv3 kernel trace of a short benchmark run (warm-up and timed builds). "
             "Command (from `/tmp`, repository at `/root/repo`):", "", "```",
             args.command.strip(), "```", "",
             "| kernel | calls | avg us | min us | max us | total ms | % |",
             "|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["totaldurationns"])):
        lines.append(f"| `{_short(r['name'])}` | {r['calls']} | "
                     f"{float(r['averagens']) / 1e3:.1f} | {float(r['minns']) / 1e3:.1f} | "
                     f"{float(r['maxns']) / 1e3:.1f} | {float(r['totaldurationns']) / 1e6:.3f} | "
                     f"{float(r['percentage']):.2f} |")
    if trace:
        disp = sorted(((int(r.get("dispatch_id", r.get("correlation_id", 0))), r["kernel_name"],
                        (int(r["end_timestamp"]) - int(r["start_timestamp"])) / 1e3)
                       for r in trace))
        builds = _segment([(n, d) for _, n, d in disp])
        per = {}
        for bld in builds:
            for tbl in ("edges", "nodes"):
                tot = {}
                for s, d in bld[tbl]:
                    st = _stage_of(s)
                    if st is not None:
                        tot[st] = tot.get(st, 0.0) + d
                for st, d in tot.items():
                    per.setdefault(f"{tbl}.{st}", []).append(d)
        if per:
            lines += ["", f"Single-kernel stages per table (mean over the {len(builds)} builds; "
                      "a stage is the sum of its kernel's launches in the table: the bucket sort "
                      "runs once over the digit ranges of in-tile buckets and once over the other "
                      "batches; the bench line's live durations of the same stages come from HIP "
                      "events on the build stream):", "", "| stage | avg us |", "|---|---|"]
            for n, v in sorted(per.items()):
                lines.append(f"| {n} | {np.mean(v):.1f} |")
    path = os.path.join(ROOT, "profiles", f"{args.workload}_kernel_stats.md")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


if __name__ == "__main__":
    main()
