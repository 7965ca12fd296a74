#!/usr/bin/env python3
"""Benchmark of the bi-directed de Bruijn graph build on one MI355X.

A step is one full build (edge table and node table) of the 2,000,000-read,
k = 31 workload (5,000,000-base genome with 200 copies of a 1,000-base repeat,
reads of length 100, 0.5% substitutions), inputs already packed and resident in
HBM.  Prints one JSON line: k-mers/s, the roofline of the dominant kernel
(timed live with per-stage HIP events on the build stream) and the oracle timed
on a bounded sample of the same reads on the host.
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


def stage_names():
    return ["start", "offsets", "enum_hist", "plan", "enum_scatter", "levels", "local_sort",
            "emit_count", "emit_write", "end"]


def algorithmic_bytes(stage, n_keys, n_unique, n_bases, n_reads, w, row_bytes):
    """Bytes a kernel must move at minimum (reads of its inputs + writes of its
    outputs), per launch."""
    if stage == "enum_hist":
        return n_bases / 4 + 16 * n_reads
    if stage == "enum_scatter":
        return n_bases / 4 + 16 * n_reads + n_keys * w
    if stage == "local_sort":  # keys in; distinct keys + counts and the run bitmap out
        return n_keys * w + 2 * n_unique * w + n_keys / 8
    if stage == "emit_write":  # distinct keys + counts and the bitmap in; table rows out
        return 2 * n_unique * w + n_keys / 8 + n_unique * row_bytes
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


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` ("edges.local_sort", ...) from the counter
    summary profiles/hbm_traffic_<workload>.md: FETCH_SIZE and WRITE_SIZE per
    dispatch, each scaled by the factor a plain copy of known size gave.  None if
    there is no summary, it lacks the kernel, or the kernels changed since."""
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
    row = data.get("kernels", {}).get(kernel)
    if row is None:
        return None
    return row["fetch_kib"] * 1024 * data["fetch_scale"] + row["write_kib"] * 1024 * data["write_scale"]


def measured_build_traffic(workload):
    """HBM bytes of one whole build (every build kernel, both tables) from the
    counter summary, scaled like measured_traffic; None when absent or stale."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    a = text.find("```json")
    if a < 0:
        return None
    b = text.find("```", a + 7)
    data = json.loads(text[a + 7:b])
    if data.get("kernel_source_sha256") != kernel_source_hash() or "build_total" not in data:
        return None
    return data["build_total"]["bytes"]


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


def run_cpu_baseline(rs, k, target_s=15.0):
    """The oracle, as is, on a bounded prefix of the reads (host cores)."""
    import oracle
    oracle.build(force=False)
    threads = oracle.host_threads(0)
    n = 2000
    while True:
        sub = rs.subset(np.arange(min(n, rs.n_reads)))
        t0 = time.perf_counter()
        oracle.build_graph(sub.bases, sub.offsets, k, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= target_s / 4 or n >= rs.n_reads:
            break
        n = int(min(rs.n_reads, n * max(2.0, min(8.0, target_s / 2 / max(dt, 1e-3)))))
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
    print(json.dumps(line), flush=True)


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
    print(json.dumps(line), flush=True)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_repeats_k31", choices=sorted(WORKLOADS))
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    args = ap.parse_args()
    if args.cap_frac is None:
        big = args.workload == "plain_large_k63" and args.scale > 0.5
        args.cap_frac = 0.55 if big else 1.0
        args.no_zkey = args.no_zkey or big
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is described in DESIGN.md and not implemented.",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        run_copy_calibration()
        return
    if args.batched:
        run_batched(args)
        return
    if args.served:
        run_served(args)
        return
    if args.slices:
        run_sliced(args)
        return

    import torch
    from paper_1003_1940_amd import api, synth

    if args.node_route != "auto":
        api.set_tuning(node_path={"kmers": api.NODES_KMERS,
                                  "endpoints": api.NODES_ENDPOINTS}[args.node_route])
    gen_name, k = WORKLOADS[args.workload]
    log(f"generating {args.workload} (scale {args.scale})")
    workers = max(1, min(16, os.cpu_count() or 1))
    gen = getattr(synth, gen_name)
    rs = gen(scale=args.scale, workers=workers) if gen_name == "plain_large" else gen(scale=args.scale)
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
    # output capacity: one row per k-mer position unless --cap-frac lowers it
    # (memory-tight mode: the build reports DBG_E_CAPACITY if it was too low)
    cap = max(1, int(n_k * args.cap_frac))
    zkey = not args.no_zkey
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
    if args.tune:
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

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    n_nodes, n_edges, status = api.read_result(result)
    if status != 0:
        raise SystemExit(f"device status {status}: {api.strerror(status)}")

    # per-step stage events (HIP events recorded by the library on `stream`)
    NE = 20
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(NE)] for _ in range(args.steps)]
    for step_ev in ev:  # torch creates the HIP event on first record
        for e in step_ev:
            e.record(stream)
    torch.cuda.synchronize()
    handles = [(ctypes.c_void_p * NE)(*[e.cuda_event for e in step_ev]) for step_ev in ev]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    start.record(stream)
    for s in range(args.steps):
        lib.dbg_set_stage_events(ctypes.cast(handles[s], ctypes.c_void_p), NE)
        step()
    stop.record(stream)
    torch.cuda.synchronize()
    lib.dbg_set_stage_events(None, 0)
    total_ms = start.elapsed_time(stop)
    ms = total_ms / args.steps
    n_nodes, n_edges, status = api.read_result(result)
    if status != 0:
        raise SystemExit(f"device status {status}: {api.strerror(status)}")
    node_route = ("endpoints" if api.read_flags(result) & api.FLAG_NODES_FROM_ENDPOINTS
                  else "kmers")

    names = stage_names()
    stages = {}
    for tbl, base in (("edges", 0), ("nodes", 10)):
        for i in range(1, 10):
            vals = [ev[s][base + i - 1].elapsed_time(ev[s][base + i]) for s in range(args.steps)]
            stages[f"{tbl}.{names[i]}"] = float(np.mean(vals))
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
    traffic = measured_traffic(args.workload, kname) if args.scale == 1.0 else None
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic),
                "algorithmic_bytes": round(kbytes), "ms": round(kms, 4)}

    # sort + reduce share of the build: partitions, LDS sort, emission of the tables
    sr_ms = sum(v for n_, v in stages.items()
                if n_.split(".")[1] in ("enum_scatter", "levels", "local_sort", "emit_count",
                                         "emit_write"))
    # The same build priced as the 8-bit LSD formulation would move it: per key and
    # table, one enumeration write, one histogram read, a read and a write per digit
    # pass, one run-length read; per distinct key a key and a count written; per
    # distinct edge the decode read and its row written.
    def lsd_bytes(n, u, bits):
        passes = (bits + 7) // 8
        return n * w * (1 + 1 + 2 * passes + 1) + u * (w + 4)
    lsd = (lsd_bytes(n_e, n_edges, 2 * k + 2) + n_edges * (w + 4) + n_edges * (2 * w + 5)
           + lsd_bytes(n_k, n_nodes, 2 * k))
    lsd_gbs = lsd / (ms / 1e3) / 1e9
    build_lsd = {"bytes": round(lsd), "achieved": round(lsd_gbs, 1), "unit": "GB/s",
                 "frac": round(lsd_gbs / HBM_PEAK_GBS, 4)}
    # the whole build's HBM bytes as the counters measured them (FETCH_SIZE +
    # WRITE_SIZE of every build kernel), over this run's build time
    tb = (measured_build_traffic(args.workload)
          if zkey and args.scale == 1.0 and args.node_route == "auto" else None)
    build_traffic = None if tb is None else {
        "bytes": tb, "achieved": round(tb / (ms / 1e3) / 1e9, 1), "unit": "GB/s",
        "frac": round(tb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}

    # STEP-4 adjacency lists and the Sec. 7 chain compaction of the built graph
    # (not part of the timed build)
    adjacency = compaction = None
    if status == 0 and args.cap_frac >= 1.0:  # memory-tight runs leave no room for them
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

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        cpu = run_cpu_baseline(rs, k)

    line = {
        "metric": "k-mers/s into bi-directed graph",
        "value": n_k / (ms / 1e3),
        "keys_per_s": (n_k + n_e) / (ms / 1e3),
        "unit": "k-mers/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64" if w == 8 else "u128",
        "data": "synthetic",
        "config": {"workload": args.workload, "reads": n_reads, "read_len": rs.params.get("read_len"),
                   "k": k, "genome": rs.params.get("genome"), "kmers": n_k, "kplus1mers": n_e,
                   "nodes": n_nodes, "edges": n_edges, "scale": args.scale,
                   "node_route": node_route, "output_rows": cap, "edge_zkey": zkey},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stages_ms": {k_: round(v, 4) for k_, v in stages.items()},
        "sort_reduce_ms": round(sr_ms, 4),
        "build_as_lsd_d8": build_lsd,
        "build_traffic": build_traffic,
        "adjacency": adjacency,
        "compaction": compaction,
        "tuning": tuning if tuning is not None else api.get_tuning(),
        "h2d_upload_and_pack_s": round(h2d_s, 4),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
