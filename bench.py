#!/usr/bin/env python3
"""Throughput of sliced tensor-network amplitude contraction on one MI355X.

One step = one qx_contract call over the whole slice range of the workload
(every slice of every bitstring), i.e. one pass of the whole hot path:
gather offsets, per-call sub-trees, then for every block of slices the
permutes, matrix-core products, small contractions and root inner products,
and the FP64 slice sum.  Inputs (plan, leaves, bitstrings) are resident on the
device before the timed region starts.

Prints one JSON line.  ``roofline`` is measured live: every launch in the timed
region is bracketed by HIP events on the stream it runs on, and the matrix-core
products' algorithmic flops (8 M N K each) are divided by their summed
durations.  ``cpu_baseline`` times the FP64 oracle on a bounded sample of the
same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "amplitudes/s + complex TFLOP/s (% MFMA peak) vs plain c64; p50/p99 latency"
# MI355X published dense peaks (per GPU)
PEAKS = {"c64": 157.3e12, "split_bf16": 2516.6e12, "split_fp16": 2516.6e12}
DTYPES = {"c64": "c64 (fp32 mfma)", "split_bf16": "bf16 hi+lo x3 (fp32 acc)", "split_fp16": "fp16 hi+lo x3 (fp32 acc)"}
HBM_PEAK = 8.0e12
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "gemm_traffic_c2_30q_d12.md")
KERNEL_NAMES = {"c64": "k_gemm_f32", "split_bf16": "k_gemm_bf16s", "split_fp16": "k_gemm_fp16s"}
COPY_BYTES = 1 << 30


def sources_digest():
    """Digest of the library sources: measured HBM traffic is only reported for the kernels it was taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2110_09894_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed counter summary, or None if stale or absent."""
    try:
        text = open(TRAFFIC_FILE).read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("sources_digest") != sources_digest():
        return None
    k = blob.get("kernels", {}).get(kernel)
    return None if k is None else k["traffic_bytes_per_launch"]


def copy_calibration():
    """A plain 1 GiB device-to-device copy: the reference dispatch for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES}), flush=True)


def summarize_traffic(run_dir):
    """Builds the traffic summary from four rocprofv3 --pmc databases under ``run_dir``:
    copy_fetch, copy_write (the calibration copy) and bench_fetch, bench_write (one timed c2 step of each
    precision).  FETCH_SIZE / WRITE_SIZE are KiB per dispatch; each is scaled by bytes-moved / counter reading
    of the copy, then averaged per launch over every launch of each matrix-product kernel."""
    import glob
    import sqlite3

    def per_dispatch(tag, counter, kernel=None):
        """[(kernel name, value)] for every dispatch of the copy run, or, with ``kernel``, for every dispatch
        of that kernel (and of the thin-product kernel, which serves every precision's thin products) in the
        last contract call that launches it (the dispatches after one call's
        k_block_finish up to the next one's): the timed call of that precision, after the warm-up call
        that ran the tile autotuner."""
        dbs = glob.glob(os.path.join(run_dir, tag, "**", "*results.db"), recursive=True)
        rows = []
        for db in dbs:
            con = sqlite3.connect(db)
            rows += con.execute("select dispatch_id, kernel_name, sum(value) from counters_collection "
                                "where counter_name = ? group by dispatch_id order by dispatch_id", (counter,)).fetchall()
        rows.sort()
        if kernel is None:
            return [(name, val) for _, name, val in rows]
        calls, cur = [], []
        for _, name, val in rows:
            if "k_block_finish" in name:
                # a call of this precision launches the family's own kernel and no other family's (thin-product
                # launches do not tell the precision; the split FP16 plan's creation also runs complex64 products)
                if {_family(n) for n, _ in cur} - {None} == {kernel}:
                    calls.append([(n, v) for n, v in cur if _is_product(n, kernel)])
                cur = []
            else:
                cur.append((name, val))
        return calls[-1] if calls else []

    cal = {}
    for counter, tag in (("FETCH_SIZE", "copy_fetch"), ("WRITE_SIZE", "copy_write")):
        d = per_dispatch(tag, counter)
        name, val = max(d, key=lambda t: t[1])
        cal[counter] = {"kernel": name[:80], "kib": val, "scale": COPY_BYTES / (val * 1024.0)}
    kernels = {}
    for short in KERNEL_NAMES.values():
        f = per_dispatch("bench_fetch", "FETCH_SIZE", short)
        w = per_dispatch("bench_write", "WRITE_SIZE", short)
        if not f or len(f) != len(w):
            continue
        fb = sum(v for _, v in f) / len(f) * 1024.0 * cal["FETCH_SIZE"]["scale"]
        wb = sum(v for _, v in w) / len(w) * 1024.0 * cal["WRITE_SIZE"]["scale"]
        kernels[short] = {"launches": len(f), "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                          "traffic_bytes_per_launch": fb + wb}
    blob = {"sources_digest": sources_digest(), "calibration": cal, "kernels": kernels}
    lines = ["# HBM traffic of the matrix-product kernels, c2 (30-qubit 5x6 grid, depth 12, 1024 slices, 256 bitstrings)",
             "",
             "Two counter passes over one timed `bench.py` step of each precision (every launch of each kernel inside",
             "the timed contract call; the warm-up call before it runs the tile autotuner), each scaled by the same",
             "counter read on a plain 1 GiB",
             "device copy (`bench.py --copy-calibration`):",
             "",
             "```",
             "cd /tmp && export TMPDIR=/tmp",
             "rocprofv3 --pmc FETCH_SIZE -d $R/gpurun_out/traffic/copy_fetch -- python3 $R/bench.py --copy-calibration",
             "rocprofv3 --pmc WRITE_SIZE -d $R/gpurun_out/traffic/copy_write -- python3 $R/bench.py --copy-calibration",
             "rocprofv3 --pmc FETCH_SIZE -d $R/gpurun_out/traffic/bench_fetch -- python3 $R/bench.py --steps 1 --warmup 1 "
             "--no-cpu-baseline --no-permute",
             "rocprofv3 --pmc WRITE_SIZE -d $R/gpurun_out/traffic/bench_write -- python3 $R/bench.py --steps 1 --warmup 1 "
             "--no-cpu-baseline --no-permute",
             "python3 $R/bench.py --summarize-traffic $R/gpurun_out/traffic",
             "```",
             "",
             "| kernel | launches | fetch MB/launch | write MB/launch | traffic MB/launch |",
             "|---|---|---|---|---|"]
    for k, v in kernels.items():
        lines.append(f"| {k} | {v['launches']} | {v['fetch_bytes_per_launch'] / 1e6:.1f} | "
                     f"{v['write_bytes_per_launch'] / 1e6:.1f} | {v['traffic_bytes_per_launch'] / 1e6:.1f} |")
    lines += ["", "Calibration: " + ", ".join(f"{c}: {v['kib']:.0f} KiB read for {COPY_BYTES >> 20} MiB copied "
                                           f"(scale {v['scale']:.3f})" for c, v in cal.items()),
              "", "bench.py reports `roofline.traffic` from this table only while the library sources still hash to",
              "`sources_digest`.", "", "```json", json.dumps(blob, indent=1), "```", ""]
    with open(TRAFFIC_FILE, "w") as f:
        f.write("\n".join(lines))
    print(TRAFFIC_FILE)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, tree, sliced, xs, seconds):
    """Oracle (complex128 tensordot) on as many (slice, bitstring) pairs as fit in ``seconds`` with the host
    BLAS's own thread count, then a third as long with one BLAS thread."""
    import oracle
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        info = threadpool_info()
        blas_threads = max([d.get("num_threads", 1) for d in info] or [1])
        blas = ", ".join(f"{d.get('internal_api')} {d.get('version')}" for d in info
                         if d.get("user_api") == "blas") or None
    except Exception:
        threadpool_limits, blas_threads, blas = None, None, None
    net = w.network()
    n_slices = 1 << len(sliced)

    def sample(budget):
        """Slice-amplitudes (slice s, bitstring b), slice-major from slice 0, until ``budget`` seconds pass
        (at least one slice-amplitude; a workload done sooner is run again); returns slice 0's values, the
        pairs done and the elapsed time."""
        vals, done = [], 0
        t0 = time.perf_counter()
        while True:
            for s in range(n_slices):
                for b in range(len(xs)):
                    v = oracle.contract_slice(net, tree, xs[b], sliced, s)
                    if s == 0 and len(vals) < len(xs):
                        vals.append(v)
                    done += 1
                    el = time.perf_counter() - t0
                    if el >= budget:
                        return vals, done, el

    def describe(done, el):
        return (f"{done} slice-amplitudes (slices from 0 upward x {len(xs)} bitstrings, repeated if the "
                f"workload is done sooner) in {el:.2f} s, scaled to {n_slices} slices per amplitude")

    vals, done, el = sample(seconds)
    out = {
        "value": done / el / n_slices,
        "unit": "amplitudes/s",
        "cores": blas_threads or len(os.sched_getaffinity(0)),
        "kind": "oracle",
        "sample": "FP64 oracle (numpy complex128 pairwise tensordot along the same tree): " + describe(done, el),
        "host_cpus": len(os.sched_getaffinity(0)),
        "cpu_model": cpu_model(),
        "blas": blas,
    }
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            _, d1, el1 = sample(seconds / 3)
        out["single_thread"] = {"value": d1 / el1 / n_slices, "unit": "amplitudes/s", "cores": 1,
                                "sample": describe(d1, el1)}
    return out, np.array(vals)


def serve_bench(args):
    """c5: saturation probe (all requests at once), then Poisson arrivals at 70% of it."""
    import torch
    from paper_2110_09894_amd.serve import Server
    from workloads.configs import SERVING

    torch.cuda.set_device(0)
    mix = SERVING
    circs = mix.circuits(reconfigure=args.serve_reconfigure, mem_weight=args.mem_weight)
    srv = Server(hbm_budget_bytes=args.serve_budget_gib << 30, max_replicas=args.max_replicas,
                 chunk_blocks=args.chunk_blocks)
    for name, circ, net, tree, sliced, st in circs:
        srv.register(name, net, tree, sliced, precision=args.precision, max_bitstrings=mix.max_bitstrings,
                     autotune=not args.no_autotune)
    srv.start()
    # warm-up: one request per circuit creates its plan (and tunes its tiles)
    for name, circ, *_ in circs:
        srv.submit_amplitudes(name, np.zeros(mix.max_bitstrings, np.uint64)).result()
    names = [c[0] for c in circs]

    def run(reqs, rate):
        srv.latencies.clear()
        srv.records.clear()
        t0 = time.monotonic()
        futs = []
        for i, (off, which, xs) in enumerate(reqs):
            if rate:
                delay = t0 + off / rate - time.monotonic()
                if delay > 0:
                    time.sleep(delay)
            futs.append(srv.submit_amplitudes(names[which], xs))
            if (i + 1) % 100 == 0:
                print(json.dumps({"progress": "submitted", "requests": i + 1,
                                  "seconds": round(time.monotonic() - t0, 1)}), file=sys.stderr, flush=True)
        for i, f in enumerate(futs):
            f.result()
            if (i + 1) % 100 == 0:
                print(json.dumps({"progress": "completed", "requests": i + 1,
                                  "seconds": round(time.monotonic() - t0, 1)}), file=sys.stderr, flush=True)
        el = time.monotonic() - t0
        lat = np.array(srv.latencies)
        st = srv.stats()
        return {"requests": len(reqs), "amplitudes": int(sum(len(x) for _, _, x in reqs)), "seconds": el,
                "amplitudes_per_s": sum(len(x) for _, _, x in reqs) / el, "requests_per_s": len(reqs) / el,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "queue": st["queue"], "service": st["service"], "by_circuit": st["by_circuit"]}

    sat = run(mix.requests(args.serve_probe), None)
    rate = 0.7 * sat["requests_per_s"]
    reqs = mix.requests(args.serve_probe + args.serve_requests)[args.serve_probe:]
    base = reqs[0][0]
    reqs = [(t - base, w, x) for t, w, x in reqs]
    pois = run(reqs, rate)
    st = srv.stats()
    srv.stop()
    out = {"metric": "amplitudes/s; p50/p99 latency (serving mix)", "value": pois["amplitudes_per_s"],
           "unit": "amplitudes/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
           "dtype": DTYPES[args.precision], "data": "synthetic (seeded circuits, Poisson arrivals, bitstrings)",
           "config": {"workload": f"{mix.name}: {mix.description}", "arrival_rate_per_s": rate,
                      "chunk_blocks": args.chunk_blocks, "max_replicas": args.max_replicas,
                      "planner_reconfigure": args.serve_reconfigure,
                      "flops_per_amplitude": {c[0]: c[5]["total_flops"] for c in circs},
                      "max_bitstrings_per_call": mix.max_bitstrings, "hbm_budget_gib": args.serve_budget_gib},
           "latency_ms": {"p50": pois["p50_ms"], "p99": pois["p99_ms"]},
           "poisson": pois, "saturation": sat, "max_concurrency": st["max_concurrency"],
           "rejected": st["rejected"], "failed": st["failed"], "replicas_built": st["replicas_built"],
           "replicas_evicted": st["replicas_evicted"], "resident_gib": st["resident_bytes"] / 2 ** 30,
           "argv": " ".join(sys.argv[1:])}
    print(json.dumps(out), flush=True)


def permute_measure(rank=26, reps=10):
    """k_permute alone on a 2^rank-element random bit permutation (seed 7): HBM roofline, 16 bytes per
    element (one read, one write), average over ``reps`` launches timed with events on the current stream."""
    import torch
    from paper_2110_09894_amd import qxtn
    rng = np.random.default_rng(7)
    in_pos = rng.permutation(rank).astype(np.int32)
    src = torch.randn(2 << rank, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    qxtn.permute_c64(src, dst, in_pos, 1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        qxtn.permute_c64(src, dst, in_pos, 1)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    gbs = 16.0 * (1 << rank) / sec / 1e9
    return {"kernel": "k_permute", "elements": 1 << rank, "avg_launch_ms": sec * 1e3, "achieved_gbs": gbs,
            "frac_of_hbm_peak": gbs * 1e9 / HBM_PEAK, "in_pos_seed": 7}


def cgemm_probe(args):
    """One large matrix product through qx_cgemm per forced tile (kernel-level measurement): 3 untimed calls,
    then the average of 5 timed with events on the current stream (the split precisions' calls include the
    operand split kernels; the kernel trace separates them)."""
    import torch
    from paper_2110_09894_amd import qxtn
    torch.cuda.set_device(0)
    M, N, K = args.cgemm_probe
    a = torch.randn(M * K * 2, device="cuda")
    b = torch.randn(K * N * 2, device="cuda")
    c = torch.empty(M * N * 2, device="cuda")
    out = {"probe": "qx_cgemm", "M": M, "N": N, "K": K, "precision": args.precision, "tiles": {}}
    for t in args.probe_tiles.split(","):
        for _ in range(3):
            qxtn.cgemm(a, b, c, M, N, K, K, 1, 1, K, 0, 0, 0, 1, args.precision, tile=t)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            qxtn.cgemm(a, b, c, M, N, K, K, 1, 1, K, 0, 0, 0, 1, args.precision, tile=t)
        e1.record()
        torch.cuda.synchronize()
        out["tiles"][t] = {"ms_per_call": e0.elapsed_time(e1) / 5}
        print(json.dumps({"tile": t, "ms_per_call": out["tiles"][t]["ms_per_call"]}), flush=True)
    print(json.dumps(out), flush=True)


def summarize_mfma(run_dir, out_name):
    """MFMA-pipe busy fraction and clock of the probe's products, from a kernel trace (run_dir/trace) and one
    counter pass per precision (run_dir/pmc_<precision>: SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE,
    SQ_INSTS_VALU_MFMA_MOPS_*).  GRBM_GUI_ACTIVE comes summed over the 8 XCDs; per XCD it is the active
    GPU cycles of the dispatch, so cycles / duration is the clock the kernel ran at.  The MFMA busy cycles
    are summed over all 1024 SIMDs."""
    import glob
    import sqlite3
    SIMDS, XCDS = 1024, 8
    rows = []
    for tdb in sorted(glob.glob(os.path.join(run_dir, "trace_*", "**", "*results.db"), recursive=True)):
        prec = tdb.split("trace_", 1)[1].split(os.sep, 1)[0]
        con = sqlite3.connect(tdb)
        durs = {}
        for name, dur in con.execute("select name, duration from kernels order by start"):
            if _family(name):
                durs.setdefault(name, []).append(dur)
        cnt = {}
        for pdb in glob.glob(os.path.join(run_dir, f"pmc_{prec}", "**", "*results.db"), recursive=True):
            pc = sqlite3.connect(pdb)
            for _, kname, cname, val in pc.execute(
                    "select dispatch_id, kernel_name, counter_name, sum(value) from counters_collection "
                    "group by dispatch_id, counter_name order by dispatch_id"):
                if _family(kname):
                    cnt.setdefault(kname, {}).setdefault(cname, []).append(val)
        for name, ds in durs.items():
            ds = ds[3:] or ds                      # the timed calls (3 untimed first)
            dur = sum(ds) / len(ds) * 1e-9
            c = cnt.get(name, {})
            busy = (sum(c["SQ_VALU_MFMA_BUSY_CYCLES"][3:]) / len(c["SQ_VALU_MFMA_BUSY_CYCLES"][3:])
                    if "SQ_VALU_MFMA_BUSY_CYCLES" in c else None)
            act = (sum(c["GRBM_GUI_ACTIVE"][3:]) / len(c["GRBM_GUI_ACTIVE"][3:]) / XCDS
                   if "GRBM_GUI_ACTIVE" in c else None)
            rows.append((prec, _tile_of(name), name, dur, busy, act))
    lines = [f"# MFMA-pipe occupancy and clock of single large products", "",
             "Commands (repository root, one MI355X), per precision P:", "", "```", "cd /tmp && export TMPDIR=/tmp",
             "rocprofv3 --kernel-trace --stats -d $R/gpurun_out/mfma/trace_P -o run -- python3 $R/bench.py "
             "--cgemm-probe 8192 8192 4096 --precision P --probe-tiles <tiles>",
             "rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE SQ_INSTS_VALU_MFMA_MOPS_BF16 "
             "SQ_INSTS_VALU_MFMA_MOPS_F16 SQ_INSTS_VALU_MFMA_MOPS_F32 -d $R/gpurun_out/mfma/pmc_P -o run -- python3 "
             "$R/bench.py --cgemm-probe 8192 8192 4096 --precision P --probe-tiles <tiles>",
             f"python3 $R/bench.py --summarize-mfma $R/gpurun_out/mfma {out_name}", "```", "",
             "`busy` = SQ_VALU_MFMA_BUSY_CYCLES / (active cycles x 1024 SIMDs); `clock` = active cycles per XCD /",
             "kernel duration; `% of nominal` = executed MFMA flops / duration / the dtype's dense peak at 2.4 GHz",
             "(= busy x clock / 2.4 GHz when the MFMAs run at their full rate).", "",
             "| precision | tile | kernel ms | busy | clock GHz | executed TFLOP/s | % of nominal |",
             "|---|---|---:|---:|---:|---:|---:|"]
    for prec, tile, name, dur, busy, act in rows:
        M = N = 8192
        K = 4096
        mult = 1 if prec == "c64" else 3
        ex = 8.0 * M * N * K * mult / dur
        b = f"{100 * busy / (act * SIMDS):.1f}%" if busy and act else "-"
        clk = f"{act / dur / 1e9:.2f}" if act else "-"
        lines.append(f"| {prec} | {tile} | {dur * 1e3:.3f} | {b} | {clk} | {ex / 1e12:.0f} | "
                     f"{100 * ex / PEAKS[prec]:.1f} |")
    path = os.path.join(PROFILES, out_name)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


def summarize_serving(out_name, logs):
    """Serving-mix summary from bench.py --workload c5 runs (one JSON line each): throughput and latency per
    phase, and per circuit the p50 / p99 of latency split into queue wait (arrival to first dispatch) and
    service (first dispatch to result)."""
    runs = [bench_line(p) for p in logs]
    lines = ["# Serving mix (c5): continuous batching over resident plans, one MI355X", "",
             "Commands (repository root):", "", "```"]
    lines += [f"python3 bench.py {r.get('argv', '')}" for r in runs]
    c0 = runs[0]["config"]
    lines += ["```", "", c0["workload"], "",
              f"Plans: trees refined by local sub-tree re-ordering of the best {c0.get('planner_reconfigure', 0)} "
              f"greedy trials per circuit, at most {c0.get('max_replicas', 2)} plan replicas per circuit and "
              f"{c0.get('max_bitstrings_per_call', '-')} bitstrings per call, "
              f"calls dispatched in chunks of {c0.get('chunk_blocks', '-')} slice block(s), "
              f"{c0.get('hbm_budget_gib', '-')} GiB HBM budget.  Complex flops per amplitude: "
              + ", ".join(f"{k} {v:.2e}" for k, v in c0.get("flops_per_amplitude", {}).items()) + ".", "",
              "Latency is arrival to result; queue = arrival to the request's first dispatch, service = first",
              "dispatch to result (a request larger than a call's capacity is served by several calls).", "",
              "| form | phase | requests | amplitudes | seconds | amplitudes/s | requests/s | p50 ms | p99 ms | "
              "queue p50 / p99 ms | service p50 / p99 ms |",
              "|---|---|---:|---:|---:|---:|---:|---:|---:|---|---|"]
    for r in runs:
        for ph in ("saturation", "poisson"):
            x = r[ph]
            lines.append(f"| {r['dtype']} | {ph} | {x['requests']} | {x['amplitudes']} | {x['seconds']:.1f} | "
                         f"{x['amplitudes_per_s']:.0f} | {x['requests_per_s']:.2f} | {x['p50_ms']:.0f} | "
                         f"{x['p99_ms']:.0f} | {x['queue']['p50_ms']:.0f} / {x['queue']['p99_ms']:.0f} | "
                         f"{x['service']['p50_ms']:.0f} / {x['service']['p99_ms']:.0f} |")
    for r in runs:
        lines += ["", f"Poisson phase per circuit, {r['dtype']} (arrival rate {r['config']['arrival_rate_per_s']:.2f}"
                      f"/s; max concurrent calls {r['max_concurrency']}, rejected {r['rejected']}, failed "
                      f"{r.get('failed', 0)}, replicas built {r.get('replicas_built', '-')}, evicted "
                      f"{r.get('replicas_evicted', '-')}, resident {r['resident_gib']:.1f} GiB):", "",
                  "| circuit | requests | p50 ms | p99 ms | queue p50 / p99 ms | service p50 / p99 ms |",
                  "|---|---:|---:|---:|---|---|"]
        for name, v in r["poisson"]["by_circuit"].items():
            lines.append(f"| {name} | {v['requests']} | {v['total']['p50_ms']:.0f} | {v['total']['p99_ms']:.0f} | "
                         f"{v['queue']['p50_ms']:.0f} / {v['queue']['p99_ms']:.0f} | "
                         f"{v['service']['p50_ms']:.0f} / {v['service']['p99_ms']:.0f} |")
        # which circuit sets the tail, and whether waiting or service time dominates it
        bc = r["poisson"]["by_circuit"]
        worst = max(bc, key=lambda k: bc[k]["total"]["p99_ms"])
        w = bc[worst]
        part = "queue wait" if w["queue"]["p99_ms"] > w["service"]["p99_ms"] else "service time"
        lines += ["", f"p99 attribution ({r['dtype']}): the overall p99 of {r['poisson']['p99_ms']:.0f} ms is set by "
                      f"{worst} (p99 {w['total']['p99_ms']:.0f} ms, the largest per-circuit tail), whose tail is "
                      f"mostly {part} (queue p99 {w['queue']['p99_ms']:.0f} ms, service p99 "
                      f"{w['service']['p99_ms']:.0f} ms); the other circuits' p99 stay at or below "
                      f"{max(v['total']['p99_ms'] for k, v in bc.items() if k != worst):.0f} ms."]
    path = os.path.join(PROFILES, out_name)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


def summarize_runs(out_name, title, logs):
    """Throughput table from bench.py runs (one JSON line each, the last line of each log): one row per
    precision the run timed (a 30-qubit run times complex64 and both split forms), with the tree, its width,
    executed complex TFLOP/s, the fraction of the form's peak (MFMA work for split precision) and the error
    against the FP64 oracle (reading 12 for the 30-qubit runs, reading 18 for the 49-qubit block)."""
    runs = [bench_line(p) for p in logs]
    lines = [f"# {title}", "", "Commands (repository root, one MI355X):", "", "```"]
    lines += [f"python3 bench.py {r.get('argv', '')}" for r in runs]
    lines += ["```", "",
              "| workload | tree | width | form | throughput | slice batch | complex TFLOP/s executed | "
              "fraction of peak | MFMA work / peak | error vs oracle | s per amplitude (all slices) |",
              "|---|---|---:|---|---:|---:|---:|---:|---:|---:|---:|"]

    def row(r, rr, prec):
        cfg = r["config"]
        tree = "refined" if r.get("planner", {}).get("reconfigure") else "greedy"
        ro = rr.get("roofline") or {}
        e = rr.get("error_vs_oracle") or {}
        err = e.get("max_abs_over_rms", e.get("abs_over_rss"))
        frac = rr.get("frac_of_peak", ro.get("frac"))
        ext = rr.get("extrapolated_seconds_per_amplitude")
        util = ro.get("mfma_util")
        cells = [cfg["workload"].split(":", 1)[0], tree, str(cfg.get("tree_width", "")), prec,
                 f"{rr['value']:.1f} {r['unit']}", str(rr.get("slice_batch", cfg.get("slice_batch", ""))),
                 f"{rr['complex_tflops']:.1f}", "" if frac is None else f"{frac:.3f}",
                 "" if util is None else f"{util:.3f}", "(not measured)" if err is None else f"{err:.1e}",
                 "" if ext is None else f"{ext:.0f}"]
        lines.append("| " + " | ".join(cells) + " |")
    for r in runs:
        prec = r["config"].get("precision", "c64")
        row(r, r, prec)
        for sub in ("split_bf16", "split_fp16"):
            if sub in r and isinstance(r[sub], dict) and "value" in r[sub]:
                row(r, r[sub], sub)
    lines += ["", "Workloads: " + "; ".join(sorted({r["config"]["workload"] for r in runs})) + "."]
    path = os.path.join(PROFILES, out_name)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


def refined_note(args):
    cost = f"roofline cost, {args.mem_weight:g} flops per element moved" if args.mem_weight else "flop cost"
    note = (f"; tree refined by local sub-tree re-ordering ({cost}) of the best {args.reconfigure} greedy trials"
            if args.reconfigure else "")
    if getattr(args, "open_qubits", 0):
        note += (f"; {args.open_qubits} highest-numbered qubits left open "
                 f"({1 << args.open_qubits} amplitudes per bitstring)")
    return note


def wait_with_progress(label, every=20.0):
    """Waits for the current stream's work by polling an event recorded after it, printing a progress line
    to stderr every ``every`` seconds (long single calls would otherwise print nothing)."""
    import torch
    ev = torch.cuda.Event()
    ev.record()
    t0 = time.monotonic()
    last = t0
    while not ev.query():
        time.sleep(0.002)
        now = time.monotonic()
        if now - last >= every:
            print(json.dumps({"progress": label, "seconds": round(now - t0, 1)}), file=sys.stderr, flush=True)
            last = now
    torch.cuda.synchronize()


def c4_golden(args, sliced, x):
    """Oracle values of slices 0..63 of the 49-qubit workload (tests/golden/c4_slices_<tree>.json, written by
    tests/golden/make_c4_oracle.py from the FP64 oracle), or None if absent or for other inputs."""
    kind = "greedy" if not args.reconfigure else ("refined" if (args.reconfigure, args.mem_weight) == (4, 16.0)
                                                    else None)
    if kind is None:
        return None
    path = os.path.join(ROOT, "tests", "golden", f"c4_slices_{kind}.json")
    try:
        g = json.load(open(path))
    except (OSError, ValueError):
        return None
    if [int(v) for v in g["sliced"]] != [int(v) for v in sliced] or int(g["bitstring"]) != int(x):
        return None
    return np.array([complex(*g["values"][str(s)]) for s in range(64)])


def c4_bench(args):
    """c4: a contiguous block of slices of the 49-qubit network for one bitstring."""
    import math
    import torch
    from paper_2110_09894_amd import qxtn
    from workloads import configs

    torch.cuda.set_device(0)
    w = configs.get("c4")
    tree, sliced, st = w.plan_inputs(reconfigure=args.reconfigure, mem_weight=args.mem_weight)
    xs = w.bitstrings()
    x = torch.from_numpy(np.ascontiguousarray(xs).view(np.int64)).cuda()
    print(json.dumps({"progress": "planning done, creating the plan"}), file=sys.stderr, flush=True)
    plan = qxtn.Plan(w.network(), tree, sliced, precision=args.precision, max_bitstrings=1,
                     autotune=not args.no_autotune)
    info = plan.info()
    bsz = 1 << info["slice_batch_log2"]
    n = max(bsz, (args.slices // bsz) * bsz)
    amp = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    print(json.dumps({"progress": "plan ready, warm-up"}), file=sys.stderr, flush=True)
    plan.contract(x, amp, (0, 2 * bsz))  # warm-up: two blocks (captures the block program)
    wait_with_progress("warm-up")
    print(json.dumps({"progress": f"timing {n} slices"}), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plan.contract(x, amp, (0, n))
    wait_with_progress("timed block")
    el = time.perf_counter() - t0
    flops = info["flops_block"] * (n // bsz) + info["flops_call"]
    total = 1 << len(sliced)
    out = {"metric": "slices/s + complex TFLOP/s (49-qubit block)", "value": n / el, "unit": "slices/s",
           "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": DTYPES[args.precision],
           "data": "synthetic (seeded circuit and bitstring)",
           "config": {"workload": f"c4: {w.description}{refined_note(args)}", "slices_timed": n, "slice_batch": bsz,
                      "tree_width": st["width"], "flops_per_slice": st["flops_per_slice"]},
           "seconds": el, "timed": "one contract call over the block, graph-replayed slice blocks",
           "complex_tflops": flops / el / 1e12,
           "frac_of_peak": flops / el / PEAKS[args.precision],
           "extrapolated_seconds_per_amplitude": el * total / n,
           "extrapolation_note": f"x{total // n} to all 2^{len(sliced)} slices"}
    if args.precision != "c64":
        out["mfma_util"] = 3 * flops / el / PEAKS[args.precision]
    out["call_sequence"] = {args.precision: ["warmup", "timed"]}
    out["planner"] = {"reconfigure": args.reconfigure, "mem_weight": args.mem_weight}
    out["argv"] = " ".join(sys.argv[1:])
    out["config"]["precision"] = args.precision
    out["config"]["bitstrings"] = 1
    if not args.no_timing:
        # one more block with per-launch HIP events (eager launches): roofline of the dominant kernel
        plan.set_timing(True)
        plan.get_timing(reset=True)
        a1 = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
        t1 = time.perf_counter()
        plan.contract(x, a1, (0, bsz))
        torch.cuda.synchronize()
        ev = time.perf_counter() - t1
        timing = plan.get_timing(reset=True)
        plan.set_timing(False)
        out.update(roofline_of(timing, args.precision, ev))
        out["evented_block_ms"] = 1e3 * ev
        out["call_sequence"][args.precision].append("evented")
    gold = c4_golden(args, sliced, xs[0])
    if gold is not None:
        # the first block's sum (Eq. 2 over slices 0..63) against the oracle's; normalised by the root sum of
        # squares of the oracle's slice values (the amplitude scale those slices contribute)
        a64 = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
        plan.contract(x, a64, (0, 64))
        torch.cuda.synchronize()
        got = complex(*a64.cpu().numpy()[0])
        want = complex(math.fsum(gold.real), math.fsum(gold.imag))
        out["call_sequence"][args.precision].append("check")
        out["error_vs_oracle"] = {"slices": "0..63", "bitstrings": 1,
                                  "abs_over_rss": abs(got - want) / float(np.sqrt(np.sum(np.abs(gold) ** 2))),
                                  "relative": abs(got - want) / abs(want)}
    print(json.dumps(out), flush=True)


FAMILY = {v: k for k, v in KERNEL_NAMES.items()}  # kernel family -> precision


def _family(name):
    for short in KERNEL_NAMES.values():
        if f"qx::{short}<" in name:
            return short
    return None


def _is_product(name, short):
    """A matrix-product launch of the family ``short``, or of the thin-product kernel (any precision)."""
    return _family(name) == short or "qx::k_gemm_thin<" in name


def _tile_of(name):
    """Work-group tile from a matrix-product kernel name: the first two template arguments, with "p<stages>"
    for the software-pipelined split-precision form (its last template argument); "thin" for the
    thin-product kernel."""
    if "qx::k_gemm_thin<" in name:
        return "thin"
    args = [a.strip() for a in name.split("<", 1)[1].split(">", 1)[0].split(",")]
    t = f"{args[0]}x{args[1]}"
    if len(args) == 8 and args[7] == "true":
        t += f"p{args[4]}"
    return t


def trace_calls(db_path):
    """Dispatches of a rocprofv3 kernel trace grouped into qx_contract calls (every call ends with
    k_block_finish; plan creation, pre-contraction and tile autotuning fall into the plan's first call):
    {precision: [[(kernel name, duration ns), ...] per call]} by the matrix-product kernel family a call
    launches."""
    import sqlite3
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, duration from kernels order by start").fetchall()
    calls, cur = {}, []
    for name, dur in rows:
        cur.append((name, dur))
        if "k_block_finish" in name:
            fams = {_family(n) for n, _ in cur} - {None}
            if len(fams) > 1:
                fams -= {KERNEL_NAMES["c64"]}  # a split FP16 plan's creation runs a complex64 calibration block
            prec = FAMILY[fams.pop()] if len(fams) == 1 else None
            calls.setdefault(prec, []).append(cur)
            cur = []
    return rows, calls


def bench_line(log_path):
    line = None
    for l in open(log_path):
        if l.startswith("{"):
            line = json.loads(l)
    return line


def _roofline_of_line(line, prec):
    if line is None:
        return None
    if prec == line.get("config", {}).get("precision"):
        return line.get("roofline")
    return line.get(prec, {}).get("roofline")


def summarize_trace(db_path, log_path, out_name):
    """Kernel-time summary of a ``rocprofv3 --kernel-trace --stats`` run of bench.py: whole-run totals per
    kernel, then the matrix-product kernels' average launch duration in the graph-replayed timed calls and
    in the evented call, beside bench.py's own event figure."""
    rows, calls = trace_calls(db_path)
    line = bench_line(log_path)
    top = {}
    for name, dur in rows:
        t = top.setdefault(name, [0, 0.0])
        t[0] += 1
        t[1] += dur * 1e-6
    total = sum(v[1] for v in top.values())
    seq = line.get("call_sequence", {}) if line else {}
    wl = line["config"]["workload"] if line else "?"
    out = [f"# Kernel time: {wl}", "", "Command (repository root, one MI355X):", "", "```",
           "cd /tmp && export TMPDIR=/tmp",
           f"rocprofv3 --kernel-trace --stats -d $R/gpurun_out/<dir> -o run -- python3 $R/bench.py {line.get('argv', '')}"
           f" > $R/gpurun_out/<dir>.log" if line else "",
           f"python3 $R/bench.py --summarize-trace $R/gpurun_out/<dir>/run_results.db $R/gpurun_out/<dir>.log {out_name}",
           "```", "",
           "Whole-run totals per kernel (plan creation, tile autotuning, warm-up, timed and evented calls):", "",
           "| kernel | calls | total ms | average ms | % of run |", "|---|---:|---:|---:|---:|"]
    for name, (n, ms) in sorted(top.items(), key=lambda kv: -kv[1][1])[:24]:
        out.append(f"| `{name[:90]}` | {n} | {ms:.0f} | {ms / n:.3f} | {100 * ms / total:.1f} |")
    out += ["", "Matrix-product kernels (all tile shapes) per call kind: `timed` calls replay the captured slice-block",
            "graph, the `evented` call launches eagerly with a HIP event pair around every launch (the launches",
            "bench.py's roofline averages over):", ""]
    for prec, cl in calls.items():
        if prec is None or prec not in seq:
            continue
        kinds = seq[prec]
        if len(kinds) != len(cl):
            out.append(f"* {prec}: {len(cl)} calls in the trace, {len(kinds)} in bench.py's sequence -- not matched")
            continue
        short = KERNEL_NAMES[prec]
        for kind in ("timed", "evented"):
            ds = [d for c, k in zip(cl, kinds) if k == kind for n, d in c if _is_product(n, short)]
            ncall = sum(1 for k in kinds if k == kind)
            if ds:
                out.append(f"* `{short}` ({prec}), {kind} calls ({ncall}): {len(ds)} launches, average "
                           f"{sum(ds) / len(ds) * 1e-6:.3f} ms, {sum(ds) * 1e-6 / ncall:.1f} ms per call")
        r = _roofline_of_line(line, prec)
        if r:
            out.append(f"  * bench.py events: {r['avg_launch_ms']:.3f} ms per launch, {r['achieved']:.1f} TFLOP/s "
                       f"algorithmic = {100 * r['frac']:.1f}% of {r['peak']:.1f} TFLOP/s (MFMA work "
                       f"{100 * r['mfma_util']:.1f}% of peak)")
    path = os.path.join(PROFILES, out_name)
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print(path)


def summarize_products(db_path, log_path, out_name):
    """Per-product table from a rocprofv3 kernel trace of bench.py and the plan's own op list
    (qx_plan_get_op_info on a host-only plan of the same inputs): for every matrix product of a step, its
    sizes, algorithmic flops and bytes, measured average duration over the graph-replayed timed calls,
    achieved rate against the dtype's peak, and whether it is GEMM-bound (flops / peak > bytes / HBM peak,
    executed flops for split precision)."""
    from paper_2110_09894_amd import qxtn
    from workloads import configs
    rows, calls = trace_calls(db_path)
    line = bench_line(log_path)
    cfg = line["config"]
    wname = cfg["workload"].split(":", 1)[0]
    w = configs.get(wname)
    pl = line.get("planner", {})
    tree, sliced, st = w.plan_inputs(reconfigure=pl.get("reconfigure", 0), mem_weight=pl.get("mem_weight", 16.0))
    B = cfg.get("bitstrings", 1)
    n_open = cfg.get("open_qubits", 0)
    open_q = list(range(w.n_qubits - n_open, w.n_qubits))
    seq = line["call_sequence"]
    out = [f"# Matrix products per step: {cfg['workload']}", "",
           "Commands (repository root, one MI355X):", "", "```", "cd /tmp && export TMPDIR=/tmp",
           f"rocprofv3 --kernel-trace --stats -d $R/gpurun_out/<dir> -o run -- python3 $R/bench.py {line.get('argv', '')}"
           f" > $R/gpurun_out/<dir>.log",
           f"python3 $R/bench.py --summarize-products $R/gpurun_out/<dir>/run_results.db $R/gpurun_out/<dir>.log "
           f"{out_name}", "```", "",
           "Durations are averages over every launch of the product in the graph-replayed timed calls (rocprofv3",
           "kernel trace); sizes, flops and bytes come from the plan (`qx_plan_get_op_info`).  Complex flops are",
           "8 M N K per product; bytes count each operand read once and the result written once.  `exec %` is the",
           "executed MFMA work (3 real products per term for split precision) against the dtype's dense peak;",
           "`bound` is `mfma` when flops / peak exceed bytes / 8 TB/s (GEMM-bound, Sec. IV-A's matrix-product",
           "steps), else `hbm`.", ""]
    for prec in [p for p in KERNEL_NAMES if p in seq and p in calls]:
        kinds = seq[prec]
        cl = calls[prec]
        if len(kinds) != len(cl):
            out += [f"{prec}: {len(cl)} calls in the trace against {len(kinds)} in bench.py's sequence; skipped", ""]
            continue
        sb = line[prec]["slice_batch"] if prec in line and "slice_batch" in line[prec] else cfg["slice_batch"]
        plan = qxtn.Plan(w.network(), tree, sliced, precision=prec, max_bitstrings=B,
                         slice_batch_log2=int(round(math.log2(sb))), open_qubits=open_q, dry_run=True)
        ops = [o for o in plan.ops() if o["op_class"] == "gemm" and o["phase"] >= 1]
        call_ops = [o for o in ops if o["phase"] == 1]
        block_ops = [o for o in ops if o["phase"] == 2]
        short = KERNEL_NAMES[prec]
        agg = {}
        n_timed = 0
        for c, k in zip(cl, kinds):
            if k != "timed":
                continue
            n_timed += 1
            g = [(n, d) for n, d in c if _is_product(n, short)]
            for j, (n, d) in enumerate(g):
                if j < len(call_ops):
                    key = ("call", j)
                elif block_ops:
                    key = ("block", (j - len(call_ops)) % len(block_ops))
                else:
                    continue
                a = agg.setdefault(key, {"n": 0, "ns": 0.0, "tile": _tile_of(n)})
                a["n"] += 1
                a["ns"] += d
        peak = PEAKS[prec]
        mult = 1 if prec == "c64" else 3
        total_ns = sum(a["ns"] for a in agg.values())
        out += [f"## {prec} (`{short}`), {n_timed} timed calls", "",
                "| # | phase | M | N | K | batch | tile | launches/step | GFLOP/launch | MB/launch | avg µs | TFLOP/s | "
                "% of peak | exec % | bound | % of product time |",
                "|---:|---|---:|---:|---:|---:|---|---:|---:|---:|---:|---:|---:|---:|---|---:|"]
        gb_ns = gb_flops = 0.0
        for key in sorted(agg, key=lambda k: -agg[k]["ns"]):
            a = agg[key]
            o = call_ops[key[1]] if key[0] == "call" else block_ops[key[1]]
            avg = a["ns"] / a["n"] * 1e-9
            rate = o["flops"] / avg
            bound = "mfma" if mult * o["flops"] / peak > o["bytes"] / HBM_PEAK else "hbm"
            if bound == "mfma":
                gb_ns += a["ns"]
                gb_flops += o["flops"] * a["n"]
            out.append(f"| {key[1]} | {key[0]} | {o['M']} | {o['N']} | {o['K']} | {o['batch']} | {a['tile']} | "
                       f"{a['n'] / n_timed:g} | {o['flops'] / 1e9:.1f} | {o['bytes'] / 1e6:.1f} | {avg * 1e6:.1f} | "
                       f"{rate / 1e12:.1f} | {100 * rate / peak:.1f} | {100 * mult * rate / peak:.1f} | {bound} | "
                       f"{100 * a['ns'] / total_ns:.1f} |")
        if gb_ns:
            r = gb_flops / (gb_ns * 1e-9)
            out += ["", f"GEMM-bound products together: {100 * gb_ns / total_ns:.1f}% of the product time, "
                        f"{r / 1e12:.1f} TFLOP/s useful = {100 * mult * r / peak:.1f}% of the dense MFMA peak in "
                        f"executed work.  All products: {total_ns * 1e-6 / n_timed:.1f} ms per step."]
        out.append("")
        plan.destroy()
    path = os.path.join(PROFILES, out_name)
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print(path)


def roofline_of(timing, precision, step_s, traffic=None):
    """Roofline of the dominant kernel from one evented step: algorithmic flops per launch over the average
    launch duration (HIP events on the launch's stream); plus the per-class device time of that step."""
    out = {"time_by_class_ms_per_step": {k: 1e3 * v["seconds"] for k, v in timing.items()}}
    g = timing["gemm"]
    if g["launches"] == 0:
        # no contraction reaches the matrix-core sizes: the call is a chain of small launches, bound by
        # launch latency; report the kernel class that takes the most device time
        dom = max(timing, key=lambda k: timing[k]["seconds"])
        d = timing[dom]
        kernel_s = sum(v["seconds"] for v in timing.values())
        out["roofline"] = {"bound": "latency", "achieved": None, "peak": None, "unit": None, "frac": None,
                           "traffic": None, "kernel": f"{dom} (largest class; no matrix-core launches)",
                           "launches_per_step": sum(v["launches"] for v in timing.values()),
                           "kernel_ms_per_step": 1e3 * kernel_s, "kernel_share_of_step": kernel_s / step_s,
                           "avg_launch_ms": 1e3 * d["seconds"] / max(1, d["launches"])}
        return out
    ach = g["flops"] / g["seconds"] if g["seconds"] > 0 else 0.0
    out["roofline"] = {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAKS[precision] / 1e12,
                       "unit": "TFLOP/s", "frac": ach / PEAKS[precision], "traffic": traffic,
                       "kernel": KERNEL_NAMES[precision],
                       "mfma_util": ach * (1 if precision == "c64" else 3) / PEAKS[precision],
                       "launches_per_step": g["launches"], "avg_launch_ms": 1e3 * g["seconds"] / g["launches"],
                       "measured_on": "one extra step with per-launch HIP events (eager launches)"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="c64", choices=sorted(PEAKS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="do not bracket launches with events")
    ap.add_argument("--no-autotune", action="store_true", help="default tile shapes instead of timed ones")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision comparison run")
    ap.add_argument("--no-permute", action="store_true", help="skip the standalone permute measurement")
    ap.add_argument("--slices", type=int, default=4096, help="c4: contiguous slices timed")
    ap.add_argument("--reconfigure", type=int, default=0, metavar="R",
                    help="c2/c4: refine the best R greedy trees by local sub-tree re-ordering "
                         "(a different, cheaper tree than the config's greedy one)")
    ap.add_argument("--open-qubits", type=int, default=0, metavar="M",
                    help="c2: leave the M highest-numbered qubits open (2^M amplitudes per bitstring)")
    ap.add_argument("--mem-weight", type=float, default=16.0,
                    help="with --reconfigure: flop:element ratio of the roofline cost (0 = flops only)")
    ap.add_argument("--serve-probe", type=int, default=100, help="c5: requests in the saturation probe")
    ap.add_argument("--serve-requests", type=int, default=1000, help="c5: requests in the Poisson phase")
    ap.add_argument("--serve-budget-gib", type=int, default=160, help="c5: HBM budget for resident plans")
    ap.add_argument("--chunk-blocks", type=int, default=1, help="c5: slice blocks per dispatched chunk of a call")
    ap.add_argument("--max-replicas", type=int, default=2, metavar="R",
                    help="c5: plan replicas per circuit (each runs one call at a time on its own stream)")
    ap.add_argument("--serve-reconfigure", type=int, default=2, metavar="R",
                    help="c5: plan the pool's circuits with the best R greedy trials refined (0 = greedy trees)")
    ap.add_argument("--copy-calibration", action="store_true", help="run only the 1 GiB copy used to scale counters")
    ap.add_argument("--cgemm-probe", type=int, nargs=3, metavar=("M", "N", "K"),
                    help="time one M x N x K product through qx_cgemm for each of --probe-tiles")
    ap.add_argument("--probe-tiles", default="128x128,128x128p3", help="tiles for --cgemm-probe")
    ap.add_argument("--summarize-runs", nargs="+", metavar="ARG",
                    help="OUT TITLE LOG...: throughput table of bench.py runs (one row per precision timed)")
    ap.add_argument("--summarize-serving", nargs="+", metavar="OUT_OR_LOG",
                    help="write the serving summary profiles/OUT from c5 bench logs (OUT LOG [LOG ...])")
    ap.add_argument("--summarize-mfma", nargs=2, metavar=("DIR", "OUT"),
                    help="write the MFMA occupancy / clock table profiles/OUT from probe traces and counters")
    ap.add_argument("--permute-only", action="store_true", help="time only k_permute (2^26 elements)")
    ap.add_argument("--summarize-traffic", metavar="DIR", help="write the HBM traffic summary from counter runs")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("DB", "LOG", "OUT"),
                    help="write the kernel-time summary profiles/OUT from a kernel trace and the bench log")
    ap.add_argument("--summarize-products", nargs=3, metavar=("DB", "LOG", "OUT"),
                    help="write the per-product table profiles/OUT from a kernel trace and the bench log")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(args.summarize_traffic)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_products:
        summarize_products(*args.summarize_products)
        return
    if args.summarize_mfma:
        summarize_mfma(*args.summarize_mfma)
        return
    if args.summarize_serving:
        summarize_serving(args.summarize_serving[0], args.summarize_serving[1:])
        return
    if args.summarize_runs:
        summarize_runs(args.summarize_runs[0], args.summarize_runs[1], args.summarize_runs[2:])
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.cgemm_probe:
        cgemm_probe(args)
        return
    if args.permute_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"permute": permute_measure(reps=args.steps * 10)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(slices shard across GPUs by contiguous ranges, but no multi-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "c5":
        serve_bench(args)
        return
    if args.open_qubits and args.workload != "c2":
        print("bench.py: --open-qubits applies to the c2 workload only", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        c4_bench(args)
        return

    import torch
    from paper_2110_09894_amd import qxtn
    from workloads import configs

    w = configs.get(args.workload)
    tree, sliced, st = w.plan_inputs(reconfigure=args.reconfigure, mem_weight=args.mem_weight)
    print(json.dumps({"progress": "planning done"}), file=sys.stderr, flush=True)
    xs = w.bitstrings()
    B = len(xs)
    net = w.network()
    torch.cuda.set_device(0)
    x = torch.from_numpy(np.ascontiguousarray(xs).view(np.int64)).cuda()
    n_slices = 1 << len(sliced)
    # open output qubits: the highest-numbered ones; each bitstring then yields 2^m amplitudes
    open_q = list(range(w.n_qubits - args.open_qubits, w.n_qubits))
    per_x = 1 << args.open_qubits

    # the oracle's sample (CPU baseline) first: its slice-0 values give each precision's error right after the
    # precision is timed, so every plan is destroyed before the next one is made and each gets the device's memory
    cb, ref = (None, None)
    if not args.no_cpu_baseline:
        cb, ref = cpu_baseline(w, tree, sliced, xs, args.cpu_seconds)

    def err(pl):
        k = len(ref)
        scale = np.sqrt(np.mean(np.abs(ref) ** 2))
        a0 = torch.zeros((k, per_x, 2), dtype=torch.float64, device="cuda")
        pl.contract(x[:k], a0, (0, 1))
        torch.cuda.synchronize()
        # with open qubits, the value whose open bits equal the bitstring's own is the closed amplitude
        own = [sum(((int(xs[b]) >> q) & 1) << i for i, q in enumerate(open_q)) for b in range(k)]
        got = a0.cpu().numpy()[np.arange(k), own]
        got = got[:, 0] + 1j * got[:, 1]
        return {"slice": 0, "bitstrings": k, "max_abs_over_rms": float(np.max(np.abs(got - ref)) / scale)}

    def run(precision):
        """Plan, warm up, time exactly args.steps full contractions (graph-replayed slice blocks, no per-launch
        events), then one more contraction with every launch bracketed by HIP events (eager launches) for the
        roofline and the per-class split; then the error on slice 0 against the oracle."""
        print(json.dumps({"progress": f"{precision}: creating the plan"}), file=sys.stderr, flush=True)
        plan = qxtn.Plan(net, tree, sliced, precision=precision, max_bitstrings=B,
                         autotune=not args.no_autotune, open_qubits=open_q)
        info = plan.info()
        print(json.dumps({"progress": f"{precision}: plan ready, timing"}), file=sys.stderr, flush=True)
        amp = torch.zeros((B, per_x, 2), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            plan.contract(x, amp)
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            starts[i].record()
            plan.contract(x, amp)
            ends[i].record()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        lat = np.array([s_.elapsed_time(e_) for s_, e_ in zip(starts, ends)])
        executed = info["flops_block"] * (n_slices >> info["slice_batch_log2"]) + info["flops_call"]
        r = {"value": B * per_x * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
             "complex_tflops": executed / (elapsed / args.steps) / 1e12,
             "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
             "slice_batch": 1 << info["slice_batch_log2"], "timed_steps": "graph-replayed slice blocks"}
        # work-group tiles of the largest matrix products (autotuned or default), largest first
        prods = sorted((o for o in plan.ops() if o["op_class"] == "gemm"), key=lambda o: -o["flops"])
        r["largest_product_tiles"] = [f"{o['M']}x{o['N']}x{o['K']}x{o['batch']}:{o['tile']}" for o in prods[:4]]
        if not args.no_timing:
            plan.set_timing(True)
            plan.get_timing(reset=True)
            t1 = time.perf_counter()
            plan.contract(x, amp)
            torch.cuda.synchronize()
            ev_el = time.perf_counter() - t1
            timing = plan.get_timing(reset=True)
            plan.set_timing(False)
            r.update(roofline_of(timing, precision, ev_el))
            r["evented_step_ms"] = 1e3 * ev_el
        if ref is not None:
            r["error_vs_oracle"] = err(plan)
        plan.destroy()
        return r

    main = run(args.precision)
    out = {
        "metric": METRIC,
        "value": main["value"],
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic (seeded random circuit, planner and bitstrings; no external dataset)",
        "config": {"workload": f"{w.name}: {w.description}{refined_note(args)}", "precision": args.precision,
                   "qubits": w.n_qubits, "depth": w.depth, "slices": n_slices, "bitstrings": B,
                   "open_qubits": args.open_qubits,
                   "slice_batch": main["slice_batch"], "tree_width": st["width"],
                   "flops_per_slice_amplitude": st["flops_per_slice"]},
        "complex_tflops": main["complex_tflops"],
        "latency_ms": main["latency_ms"],
    }
    for k in ("roofline", "time_by_class_ms_per_step", "evented_step_ms", "timed_steps", "largest_product_tiles"):
        if k in main:
            out[k] = main[k]
    # contract calls each plan makes, in order (read by the trace summaries)
    calls = ["warmup"] * args.warmup + ["timed"] * args.steps + ([] if args.no_timing else ["evented"])
    out["call_sequence"] = {args.precision: list(calls)}
    if "roofline" in out and out["roofline"]["bound"] == "mfma":
        # counters were taken on the 30-qubit workload only
        if args.workload == "c2" and not args.reconfigure and not args.open_qubits:
            out["roofline"]["traffic"] = measured_traffic(KERNEL_NAMES[args.precision])
    if ref is not None:
        calls.append("check")
        out["call_sequence"][args.precision] = list(calls)
        out["error_vs_oracle"] = main["error_vs_oracle"]
    if args.precision == "c64" and not args.no_split:
        for prec in ("split_bf16", "split_fp16"):
            r = run(prec)
            r["speedup_vs_c64"] = r["value"] / main["value"]
            out["call_sequence"][prec] = list(calls)
            if "roofline" in r and r["roofline"]["bound"] == "mfma" and args.workload == "c2" \
                    and not args.reconfigure and not args.open_qubits:
                r["roofline"]["traffic"] = measured_traffic(KERNEL_NAMES[prec])
            out[prec] = r

    # index-permute primitive on its own (the workload's plan needs none): HBM roofline
    if not args.no_permute:
        out["permute"] = permute_measure()

    if cb is not None:
        out["cpu_baseline"] = cb
    out["planner"] = {"reconfigure": args.reconfigure, "mem_weight": args.mem_weight}
    out["argv"] = " ".join(sys.argv[1:])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
