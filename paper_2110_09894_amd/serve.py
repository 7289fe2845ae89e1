"""Continuous-batching amplitude / sampling server over the C-ABI.

* Circuits are registered once; their plans stay resident on the device.  A
  circuit may have several plan replicas (each owns its own arena, so replicas
  run concurrently on their own streams); replicas are created on demand while
  the HBM budget allows and idle replicas of other circuits are evicted first.
* Requests arrive at any time.  The scheduler thread keeps a FIFO of pending work;
  whenever a replica is idle it takes the oldest pending work for that circuit and
  merges further pending requests of the same circuit into the same call, up to
  the plan's bitstring capacity (continuous batching).  Requests larger than the
  capacity are split.  Batch sizes are rounded up to a few buckets (padding with
  a repeated bitstring) so every replica replays one of a handful of captured
  block programs.
* Each bitstring's amplitude is computed independently of the others in its
  call, with the same plan inputs and kernels, so a request's result is the same
  alone and in a mix.
* A circuit registered with open output qubits answers every bitstring with the
  2^m amplitudes of all values of those qubits (one contraction, Sec. II); its
  results are [n, 2^m] arrays.
* Sampling requests run the empirical-supremum rejection sampler (Sec. III-B):
  each batch of candidates is one amplitude work item; accept / reject runs on
  the host when it completes and the next batch is queued.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future

import numpy as np

from . import qxtn


class AdmissionError(RuntimeError):
    pass


def _bucket(b: int, cap: int) -> int:
    """Round a batch size up to 1, 2, 4, ..., 64, then multiples of 64 (at most cap)."""
    r = 1
    while r < b and r < 64:
        r <<= 1
    if r < b:
        r = ((b + 63) // 64) * 64
    return min(r, cap)


class _Circuit:
    def __init__(self, name, network, tree, sliced, precision, max_bitstrings, slice_batch_log2, autotune,
                 plan_budget, open_qubits=()):
        self.name = name
        self.network = network
        self.tree = tree
        self.sliced = list(sliced)
        self.precision = precision
        self.max_b = int(max_bitstrings)
        self.autotune = autotune
        self.open_qubits = sorted(int(q) for q in open_qubits)
        self.per = 1 << len(self.open_qubits)   # amplitudes per bitstring
        # the slice batch is resolved once (within the per-plan budget) so every replica is the same plan
        dry = qxtn.Plan(network, tree, self.sliced, precision=precision, max_bitstrings=self.max_b,
                        slice_batch_log2=slice_batch_log2, dry_run=True, hbm_budget_bytes=plan_budget,
                        open_qubits=self.open_qubits)
        self.js = dry.info()["slice_batch_log2"]
        self.device_bytes = dry.info()["device_bytes"]
        self.n_slices = 1 << len(self.sliced)
        self.n_qubits = network.n_qubits
        self.replicas = []


class _Replica:
    def __init__(self, circ, device):
        import torch
        self.circ = circ
        self.stream = torch.cuda.Stream(device=device)
        with torch.cuda.stream(self.stream):
            self.plan = qxtn.Plan(circ.network, circ.tree, circ.sliced, precision=circ.precision,
                                  max_bitstrings=circ.max_b, slice_batch_log2=circ.js,
                                  autotune=circ.autotune, open_qubits=circ.open_qubits, stream=self.stream)
        self.device_bytes = self.plan.info()["device_bytes"]
        self.busy = None          # in-flight call, or None
        self.last_used = time.monotonic()

    def destroy(self):
        self.stream.synchronize()
        self.plan.destroy()


class _Request:
    _ids = 0

    def __init__(self, circuit, bitstrings=None, sample=None):
        _Request._ids += 1
        self.id = _Request._ids
        self.circuit = circuit
        self.arrival = time.monotonic()
        self.future = Future()
        self.sample = sample      # dict for sampling requests
        if bitstrings is not None:
            self.bitstrings = np.ascontiguousarray(np.asarray(bitstrings, dtype=np.uint64))
            self.result = None        # shaped by the circuit when enqueued
            self.remaining = len(self.bitstrings)
            self.next_off = 0


class Server:
    def __init__(self, hbm_budget_bytes: int = 64 << 30, max_replicas: int = 2, device: int = 0,
                 plan_budget_bytes: int | None = None):
        self.budget = int(hbm_budget_bytes)
        # one plan's share when its slice batch is chosen automatically
        self.plan_budget = int(plan_budget_bytes) if plan_budget_bytes else max(1 << 30, self.budget // 8)
        self.max_replicas = int(max_replicas)
        self.device = device
        self.circuits = {}
        self.pending = collections.deque()   # requests with bitstrings not yet dispatched
        self.lock = threading.Condition()
        self.running = False
        self.thread = None
        self.latencies = []
        self.completed_amplitudes = 0
        self.rejected = 0
        self.max_concurrency = 0
        self.used_bytes = 0

    # ------------------------------------------------------------------ setup
    def register(self, name, network, tree, sliced=(), precision="c64", max_bitstrings=1024,
                 slice_batch_log2=-1, autotune=False, open_qubits=()):
        circ = _Circuit(name, network, tree, sliced, precision, max_bitstrings, slice_batch_log2, autotune,
                        self.plan_budget, open_qubits)
        if circ.device_bytes > self.budget:
            raise AdmissionError(f"plan for {name} needs {circ.device_bytes} bytes, budget {self.budget}")
        with self.lock:
            self.circuits[name] = circ
        return circ.device_bytes

    def start(self):
        with self.lock:
            if self.running:
                return
            self.running = True
        self.thread = threading.Thread(target=self._loop, name="qx-server", daemon=True)
        self.thread.start()

    def stop(self):
        with self.lock:
            self.running = False
            self.lock.notify_all()
        if self.thread:
            self.thread.join()
        for circ in self.circuits.values():
            for r in circ.replicas:
                r.destroy()
            circ.replicas = []
        self.used_bytes = 0

    # --------------------------------------------------------------- requests
    def submit_amplitudes(self, name, bitstrings) -> Future:
        req = _Request(name, bitstrings=bitstrings)
        self._enqueue(req)
        return req.future

    def submit_sample(self, name, n_samples, candidates, uniforms, warmup=0, batch=256) -> Future:
        """Rejection-sample ``n_samples`` bitstrings from the given candidate / uniform streams."""
        req = _Request(name, sample={"n": int(n_samples), "cand": np.asarray(candidates, dtype=np.uint64),
                                     "u": np.asarray(uniforms, dtype=np.float64), "warmup": int(warmup),
                                     "batch": int(batch), "used": 0, "M": 1.0, "kept": []})
        self._enqueue_sample_batch(req)
        return req.future

    def _enqueue(self, req):
        circ = self.circuits.get(req.circuit)
        if circ is None:
            self.rejected += 1
            req.future.set_exception(AdmissionError(f"unknown circuit {req.circuit}"))
            return
        n = len(req.bitstrings)
        req.result = np.zeros((n, circ.per) if circ.per > 1 else n, dtype=np.complex128)
        with self.lock:
            self.pending.append(req)
            self.lock.notify_all()

    def _enqueue_sample_batch(self, req):
        s = req.sample
        cand = s["cand"][s["used"]:s["used"] + s["batch"]]
        if len(cand) == 0:
            self._finish_sample(req)
            return
        sub = _Request(req.circuit, bitstrings=cand)
        sub.arrival = req.arrival
        sub.parent = req
        self._enqueue(sub)

    def _finish_sample(self, req):
        s = req.sample
        self.latencies.append(time.monotonic() - req.arrival)
        req.future.set_result((np.array(s["kept"][:s["n"]], dtype=np.uint64),
                               {"candidates_used": s["used"], "M": s["M"]}))

    def _sample_step(self, sub):
        req = sub.parent
        s = req.sample
        circ = self.circuits[req.circuit]
        N = float(2.0 ** circ.n_qubits)
        vals = sub.result
        if circ.per > 1:
            # the candidate's amplitude is the value whose open bits are its own
            own = [sum(((int(x) >> q) & 1) << i for i, q in enumerate(circ.open_qubits)) for x in sub.bitstrings]
            vals = sub.result[np.arange(len(own)), own]
        for x, a in zip(sub.bitstrings, vals):
            if len(s["kept"]) >= s["n"]:
                break
            i = s["used"]
            ratio = float(abs(a) ** 2) * N
            if i >= s["warmup"] and s["u"][i] * s["M"] < ratio:
                s["kept"].append(int(x))
            s["M"] = max(s["M"], ratio)
            s["used"] = i + 1
        if len(s["kept"]) >= s["n"] or s["used"] >= len(s["cand"]):
            self._finish_sample(req)
        else:
            self._enqueue_sample_batch(req)

    # --------------------------------------------------------------- scheduler
    def _idle_replica(self, circ):
        for r in circ.replicas:
            if r.busy is None:
                return r
        if len(circ.replicas) >= self.max_replicas:
            return None
        # admit a new replica by HBM budget, evicting idle replicas of other circuits (LRU)
        while self.used_bytes + circ.device_bytes > self.budget:
            idle = [(r.last_used, r) for c in self.circuits.values() if c is not circ
                    for r in c.replicas if r.busy is None]
            if not idle:
                return None
            _, victim = min(idle, key=lambda t: t[0])
            victim.destroy()
            victim.circ.replicas.remove(victim)
            self.used_bytes -= victim.device_bytes
        rep = _Replica(circ, self.device)
        circ.replicas.append(rep)
        self.used_bytes += rep.device_bytes
        return rep

    def _dispatch(self, rep, parts):
        """parts: list of (request, offset, count).  One contract call over all of them."""
        import torch
        circ = rep.circ
        xs = np.concatenate([req.bitstrings[o:o + c] for req, o, c in parts])
        B = len(xs)
        Bp = _bucket(B, circ.max_b)
        if Bp > B:
            xs = np.concatenate([xs, np.repeat(xs[:1], Bp - B)])
        with torch.cuda.stream(rep.stream):
            hx = torch.from_numpy(xs.view(np.int64)).pin_memory()
            dx = hx.to(f"cuda:{self.device}", non_blocking=True)
            amp = torch.zeros((Bp, circ.per, 2), dtype=torch.float64, device=f"cuda:{self.device}")
            rep.plan.contract(dx, amp, (0, circ.n_slices), stream=rep.stream)
            host = torch.empty((Bp, circ.per, 2), dtype=torch.float64).pin_memory()
            host.copy_(amp, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(rep.stream)
        rep.busy = {"parts": parts, "host": host, "event": ev, "keep": (hx, dx, amp), "B": B}

    def _complete(self, rep):
        call = rep.busy
        h = call["host"].numpy()
        vals = h[..., 0] + 1j * h[..., 1]
        if vals.shape[1] == 1:
            vals = vals[:, 0]
        pos = 0
        now = time.monotonic()
        for req, o, c in call["parts"]:
            req.result[o:o + c] = vals[pos:pos + c]
            pos += c
            req.remaining -= c
            if req.remaining == 0:
                if getattr(req, "parent", None) is not None:
                    self._sample_step(req)
                else:
                    self.latencies.append(now - req.arrival)
                    self.completed_amplitudes += req.result.size
                    req.future.set_result(req.result)
        rep.busy = None
        rep.last_used = now

    def _loop(self):
        import torch
        torch.cuda.set_device(self.device)
        while True:
            progressed = False
            # completions
            for circ in list(self.circuits.values()):
                for rep in circ.replicas:
                    if rep.busy is not None and rep.busy["event"].query():
                        self._complete(rep)
                        progressed = True
            with self.lock:
                busy = sum(1 for c in self.circuits.values() for r in c.replicas if r.busy is not None)
                if not self.running and not self.pending and busy == 0:
                    return
                # admission: oldest pending first; merge same-circuit work into one call
                i = 0
                while i < len(self.pending):
                    req = self.pending[i]
                    circ = self.circuits[req.circuit]
                    try:
                        rep = self._idle_replica(circ)
                    except Exception as e:  # plan creation failed: reject the request
                        self.pending.remove(req)
                        self.rejected += 1
                        req.future.set_exception(e)
                        continue
                    if rep is None:
                        i += 1
                        continue
                    parts, room = [], circ.max_b
                    j = i
                    while j < len(self.pending) and room > 0:
                        r2 = self.pending[j]
                        if r2.circuit != req.circuit:
                            j += 1
                            continue
                        take = min(room, len(r2.bitstrings) - r2.next_off)
                        parts.append((r2, r2.next_off, take))
                        r2.next_off += take
                        room -= take
                        if r2.next_off == len(r2.bitstrings):
                            del self.pending[j]
                        else:
                            j += 1
                    self._dispatch(rep, parts)
                    progressed = True
                busy = sum(1 for c in self.circuits.values() for r in c.replicas if r.busy is not None)
                self.max_concurrency = max(self.max_concurrency, busy)
                if not progressed:
                    self.lock.wait(timeout=0.0005)

    # ------------------------------------------------------------------ stats
    def stats(self):
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return {"completed_amplitudes": self.completed_amplitudes, "rejected": self.rejected,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "max_concurrency": self.max_concurrency, "resident_bytes": self.used_bytes}
