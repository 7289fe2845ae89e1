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
KERNEL_NAMES = {"c64": "k_gemm_f32", "split_bf16": "k_gemm_bf16s", "split_fp16": "k_gemm_split"}
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
        of that kernel in the last contract call that launches it (the dispatches after one call's
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
                if cur:
                    calls.append(cur)
                cur = []
            elif f"qx::{kernel}<" in name:
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
    circs = mix.circuits()
    srv = Server(hbm_budget_bytes=args.serve_budget_gib << 30, max_replicas=2)
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
        t0 = time.monotonic()
        futs = []
        for off, which, xs in reqs:
            if rate:
                delay = t0 + off / rate - time.monotonic()
                if delay > 0:
                    time.sleep(delay)
            futs.append(srv.submit_amplitudes(names[which], xs))
        for f in futs:
            f.result()
        el = time.monotonic() - t0
        lat = np.array(srv.latencies)
        return {"requests": len(reqs), "amplitudes": int(sum(len(x) for _, _, x in reqs)), "seconds": el,
                "amplitudes_per_s": sum(len(x) for _, _, x in reqs) / el, "requests_per_s": len(reqs) / el,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3)}

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
                      "max_bitstrings_per_call": mix.max_bitstrings, "hbm_budget_gib": args.serve_budget_gib},
           "latency_ms": {"p50": pois["p50_ms"], "p99": pois["p99_ms"]},
           "poisson": pois, "saturation": sat, "max_concurrency": st["max_concurrency"],
           "rejected": st["rejected"], "resident_gib": st["resident_bytes"] / 2 ** 30}
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


def refined_note(args):
    cost = f"roofline cost, {args.mem_weight:g} flops per element moved" if args.mem_weight else "flop cost"
    note = (f"; tree refined by local sub-tree re-ordering ({cost}) of the best {args.reconfigure} greedy trials"
            if args.reconfigure else "")
    if getattr(args, "open_qubits", 0):
        note += (f"; {args.open_qubits} highest-numbered qubits left open "
                 f"({1 << args.open_qubits} amplitudes per bitstring)")
    return note


def c4_bench(args):
    """c4: a contiguous block of slices of the 49-qubit network for one bitstring."""
    import torch
    from paper_2110_09894_amd import qxtn
    from workloads import configs

    torch.cuda.set_device(0)
    w = configs.get("c4")
    tree, sliced, st = w.plan_inputs(reconfigure=args.reconfigure, mem_weight=args.mem_weight)
    xs = w.bitstrings()
    x = torch.from_numpy(np.ascontiguousarray(xs).view(np.int64)).cuda()
    plan = qxtn.Plan(w.network(), tree, sliced, precision=args.precision, max_bitstrings=1,
                     autotune=not args.no_autotune)
    info = plan.info()
    bsz = 1 << info["slice_batch_log2"]
    n = max(bsz, (args.slices // bsz) * bsz)
    amp = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    plan.contract(x, amp, (0, bsz))  # warm-up: one block (captures the block program)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.contract(x, amp, (0, n))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    flops = info["flops_block"] * (n // bsz) + info["flops_call"]
    total = 1 << len(sliced)
    out = {"metric": "slices/s + complex TFLOP/s (49-qubit block)", "value": n / el, "unit": "slices/s",
           "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": DTYPES[args.precision],
           "data": "synthetic (seeded circuit and bitstring)",
           "config": {"workload": f"c4: {w.description}{refined_note(args)}", "slices_timed": n, "slice_batch": bsz,
                      "tree_width": st["width"], "flops_per_slice": st["flops_per_slice"]},
           "seconds": el, "complex_tflops": flops / el / 1e12,
           "frac_of_peak": flops / el / PEAKS[args.precision],
           "extrapolated_seconds_per_amplitude": el * total / n,
           "extrapolation_note": f"x{total // n} to all 2^{len(sliced)} slices"}
    print(json.dumps(out), flush=True)


def summarize_trace(db_path, log_path):
    """Kernel-time summary of a ``rocprofv3 --kernel-trace --stats`` run of bench.py (3 timed steps, 1 warm-up)."""
    import sqlite3
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, duration from kernels order by start").fetchall()
    top = {}
    for name, dur in rows:
        t = top.setdefault(name, [0, 0.0])
        t[0] += 1
        t[1] += dur * 1e-6
    total = sum(v[1] for v in top.values())
    # per kernel family, launches of the timed contract calls: a call is every dispatch after the previous
    # call's k_block_finish up to its own (per-call products included, as in bench.py's events); the first
    # call of each plan is the warm-up, which also holds that plan's autotuning trials
    fam, calls, cur = {}, 0, []
    for name, dur in rows:
        if "k_block_finish" not in name:
            cur.append((name, dur))
            continue
        calls += 1
        if calls % 4 != 1:
            for n, d in cur:
                for short in KERNEL_NAMES.values():
                    if f"qx::{short}<" in n:
                        f = fam.setdefault(short, [0, 0.0])
                        f[0] += 1
                        f[1] += d * 1e-6
        cur = []
    line = None
    for l in open(log_path):
        if l.startswith("{"):
            line = json.loads(l)
    out = ["# Kernel time on the 30-qubit workload (5x6 grid, depth 12, 1024 slices, 256 bitstrings)", "",
           "Command (repository root, one MI355X):", "", "```",
           "cd /tmp && export TMPDIR=/tmp",
           "rocprofv3 --kernel-trace --stats -d $R/gpurun_out/trace_c2 -o run -- python3 $R/bench.py --steps 3 "
           "--warmup 1 --no-cpu-baseline --no-permute",
           "python3 $R/bench.py --summarize-trace $R/gpurun_out/trace_c2/run_results.db $R/gpurun_out/trace_c2.log",
           "```", "",
           "The run makes a complex64 plan and a split-BF16 plan (both autotuned); each does 1 warm-up call (graph",
           "replay) and 3 timed calls (launches bracketed by events).  Whole-run totals per kernel:", "",
           "| kernel | calls | total ms | average ms | % of run |", "|---|---:|---:|---:|---:|"]
    for name, (n, ms) in sorted(top.items(), key=lambda kv: -kv[1][1])[:20]:
        out.append(f"| `{name[:90]}` | {n} | {ms:.0f} | {ms / n:.3f} | {100 * ms / total:.1f} |")
    out += ["", "Matrix-product kernels (all tile shapes) inside the timed calls, against what bench.py measured",
            "with HIP events in the same run:", ""]
    for prec, short in KERNEL_NAMES.items():
        if short not in fam:
            continue
        n, ms = fam[short]
        r = None
        if line is not None:
            r = line.get("roofline") if prec == line["config"].get("precision") else line.get(prec, {}).get("roofline")
        ev = f"bench.py: {r['avg_launch_ms']:.3f} ms per launch, {r['achieved']:.1f} TFLOP/s algorithmic = " \
             f"{100 * r['frac']:.1f}% of {r['peak']:.1f} TFLOP/s (MFMA work {100 * r['mfma_util']:.1f}% of peak)" if r else ""
        out.append(f"* `{short}` ({prec}): {n} launches, average {ms / n:.3f} ms.  {ev}")
    if line is not None:
        out += ["", "bench.py line of this run: c64 " + f"{line['value']:.1f} amplitudes/s"
                + (f", split_bf16 {line['split_bf16']['value']:.1f} amplitudes/s" if "split_bf16" in line else "")]
    path = os.path.join(PROFILES, "gemm_c2_30q_d12.md")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print(path)


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
    ap.add_argument("--serve-probe", type=int, default=24, help="c5: requests in the saturation probe")
    ap.add_argument("--serve-requests", type=int, default=120, help="c5: requests in the Poisson phase")
    ap.add_argument("--serve-budget-gib", type=int, default=160, help="c5: HBM budget for resident plans")
    ap.add_argument("--copy-calibration", action="store_true", help="run only the 1 GiB copy used to scale counters")
    ap.add_argument("--permute-only", action="store_true", help="time only k_permute (2^26 elements)")
    ap.add_argument("--summarize-traffic", metavar="DIR", help="write the HBM traffic summary from counter runs")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("DB", "LOG"), help="write the kernel-time summary")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(args.summarize_traffic)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.copy_calibration:
        copy_calibration()
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
    xs = w.bitstrings()
    B = len(xs)
    net = w.network()
    torch.cuda.set_device(0)
    x = torch.from_numpy(np.ascontiguousarray(xs).view(np.int64)).cuda()
    n_slices = 1 << len(sliced)
    # open output qubits: the highest-numbered ones; each bitstring then yields 2^m amplitudes
    open_q = list(range(w.n_qubits - args.open_qubits, w.n_qubits))
    per_x = 1 << args.open_qubits

    def run(precision):
        """Plan, warm up, then time exactly args.steps full contractions."""
        plan = qxtn.Plan(net, tree, sliced, precision=precision, max_bitstrings=B,
                         autotune=not args.no_autotune, open_qubits=open_q)
        info = plan.info()
        amp = torch.zeros((B, per_x, 2), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            plan.contract(x, amp)
        torch.cuda.synchronize()
        if not args.no_timing:
            plan.set_timing(True)
            plan.get_timing(reset=True)
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
        timing = None
        if not args.no_timing:
            timing = plan.get_timing(reset=True)
            plan.set_timing(False)
        lat = np.array([s_.elapsed_time(e_) for s_, e_ in zip(starts, ends)])
        executed = info["flops_block"] * (n_slices >> info["slice_batch_log2"]) + info["flops_call"]
        r = {"value": B * per_x * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
             "complex_tflops": executed / (elapsed / args.steps) / 1e12,
             "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
             "slice_batch": 1 << info["slice_batch_log2"]}
        if timing is not None and timing["gemm"]["launches"] == 0:
            # no contraction reaches the matrix-core sizes: the call is a chain of small launches, bound by
            # launch latency; report the kernel class that takes the most device time
            dom = max(timing, key=lambda k: timing[k]["seconds"])
            d = timing[dom]
            kernel_s = sum(v["seconds"] for v in timing.values()) / args.steps
            r["roofline"] = {"bound": "latency", "achieved": None, "peak": None, "unit": None, "frac": None,
                             "traffic": None, "kernel": f"{dom} (largest class; no matrix-core launches)",
                             "launches_per_step": sum(v["launches"] for v in timing.values()) / args.steps,
                             "kernel_ms_per_step": 1e3 * kernel_s,
                             "kernel_share_of_step": kernel_s / (elapsed / args.steps),
                             "avg_launch_ms": 1e3 * d["seconds"] / max(1, d["launches"])}
        elif timing is not None:
            g = timing["gemm"]
            ach = g["flops"] / g["seconds"] if g["seconds"] > 0 else 0.0
            r["roofline"] = {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAKS[precision] / 1e12,
                             "unit": "TFLOP/s", "frac": ach / PEAKS[precision],
                             # counters were taken on the 30-qubit workload only
                             "traffic": (measured_traffic(KERNEL_NAMES[precision])
                                         if args.workload == "c2" and not args.reconfigure
                                         and not args.open_qubits else None),
                             "kernel": KERNEL_NAMES[precision],
                             "mfma_util": ach * (1 if precision == "c64" else 3) / PEAKS[precision],
                             "launches_per_step": g["launches"] / args.steps,
                             "avg_launch_ms": 1e3 * g["seconds"] / max(1, g["launches"])}
            r["time_by_class_ms_per_step"] = {k: 1e3 * v["seconds"] / args.steps for k, v in timing.items()}
        return plan, r

    plan, main = run(args.precision)
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
    for k in ("roofline", "time_by_class_ms_per_step"):
        if k in main:
            out[k] = main[k]
    split_plans = {}
    if args.precision == "c64" and not args.no_split:
        for prec in ("split_bf16",):
            sp, r = run(prec)
            split_plans[prec] = sp
            r["speedup_vs_c64"] = r["value"] / main["value"]
            out[prec] = r

    # index-permute primitive on its own (the workload's plan needs none): HBM roofline
    if not args.no_permute:
        out["permute"] = permute_measure()

    # accuracy on slice 0 and the CPU baseline share the oracle sample
    if not args.no_cpu_baseline:
        cb, ref = cpu_baseline(w, tree, sliced, xs, args.cpu_seconds)
        out["cpu_baseline"] = cb
        k = len(ref)
        scale = np.sqrt(np.mean(np.abs(ref) ** 2))

        def err(pl):
            a0 = torch.zeros((k, per_x, 2), dtype=torch.float64, device="cuda")
            pl.contract(x[:k], a0, (0, 1))
            torch.cuda.synchronize()
            # with open qubits, the value whose open bits equal the bitstring's own is the closed amplitude
            own = [sum(((int(xs[b]) >> q) & 1) << i for i, q in enumerate(open_q)) for b in range(k)]
            got = a0.cpu().numpy()[np.arange(k), own]
            got = got[:, 0] + 1j * got[:, 1]
            return {"slice": 0, "bitstrings": k, "max_abs_over_rms": float(np.max(np.abs(got - ref)) / scale)}

        out["error_vs_oracle"] = err(plan)
        for prec, sp in split_plans.items():
            out[prec]["error_vs_oracle"] = err(sp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
