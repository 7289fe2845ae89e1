"""Continuous-batching amplitude / sampling server over the C-ABI.

* Circuits are registered once; their plans stay resident on the device.  A
  circuit may have several plan replicas (each owns its own arena, so replicas
  run concurrently on their own streams).  Replicas are built by a worker
  thread: the scheduler only reserves HBM budget and hands the job over, so
  plan creation (allocation, pre-contraction, tile autotuning) never holds up
  dispatch or completion of other requests; the scheduler sees a replica once
  it is ready.  Idle replicas of other circuits are evicted (least recently
  used first) when the budget needs it; the scheduler destroys them outside its
  lock, and a destroy waits only for that replica's own last call.
* Admission counts a replica's plan (qx_plan_peak_bytes at the circuit's
  bitstring capacity and slice batch) plus the device buffers of its one call
  in flight (bitstrings and amplitudes at full capacity).
* Requests arrive at any time.  The scheduler thread keeps a FIFO of pending
  work; whenever a replica is idle it takes the oldest pending work for that
  circuit and merges further pending requests of the same circuit into the
  same call, up to the plan's bitstring capacity (continuous batching).
  Requests larger than the capacity are split.  Batch sizes are rounded up to
  a few buckets (padding with a repeated bitstring) so every replica replays
  one of a handful of captured block programs.
* A call runs as a sequence of slice-range chunks of at most chunk_blocks
  slice blocks each (Eq. 2: partial sums over disjoint ranges add), the
  replica's FP64 accumulator carrying over between chunks: every stream then
  holds at most a chunk's kernels at a time, so calls of small circuits are not
  queued behind the whole of a large circuit's call when streams share the
  device's hardware queues.
* Each bitstring's amplitude is computed independently of the others in its
  call, with the same plan inputs and kernels, so a request's result is the
  same alone and in a mix.
* A circuit registered with open output qubits answers every bitstring with
  the 2^m amplitudes of all values of those qubits (one contraction, Sec. II);
  its results are [n, 2^m] arrays.
* Sampling requests run the empirical-supremum rejection sampler (Sec. III-B):
  each batch of candidates is one amplitude work item; accept / reject runs on
  the host when it completes and the next batch is queued.
* Failures (plan creation, a launch, a copy) fail only the requests involved;
  the scheduler keeps running.  Every request records its queue wait (arrival
  to its first dispatch) and service time (first dispatch to result).
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
        self.block_slices = 1 << self.js
        self.plan_bytes = dry.peak_bytes(self.max_b, self.js)
        # device buffers of the one call a replica has in flight: bitstrings and amplitudes at capacity
        self.call_bytes = self.max_b * (8 + 16 * self.per)
        self.device_bytes = self.plan_bytes + self.call_bytes
        dry.destroy()
        self.n_slices = 1 << len(self.sliced)
        self.n_qubits = network.n_qubits
        self.replicas = []      # ready replicas
        self.building = 0       # replicas the worker is creating
        self.error = None       # plan creation failed: requests are rejected with this


class _Replica:
    def __init__(self, circ, device):
        import torch
        self.circ = circ
        self.stream = torch.cuda.Stream(device=device)
        with torch.cuda.stream(self.stream):
            self.plan = qxtn.Plan(circ.network, circ.tree, circ.sliced, precision=circ.precision,
                                  max_bitstrings=circ.max_b, slice_batch_log2=circ.js,
                                  autotune=circ.autotune, open_qubits=circ.open_qubits, stream=self.stream)
        self.device_bytes = circ.device_bytes
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
        self.first_dispatch = None
        self.future = Future()
        self.sample = sample      # dict for sampling requests
        self.parent = None        # sampling request a candidate batch belongs to
        self.failed = False
        if bitstrings is not None:
            self.bitstrings = np.ascontiguousarray(np.asarray(bitstrings, dtype=np.uint64))
            self.result = None        # shaped by the circuit when enqueued
            self.remaining = len(self.bitstrings)
            self.next_off = 0


class Server:
    def __init__(self, hbm_budget_bytes: int = 64 << 30, max_replicas: int = 2, device: int = 0,
                 plan_budget_bytes: int | None = None, chunk_blocks: int = 1):
        self.budget = int(hbm_budget_bytes)
        self.chunk_blocks = max(1, int(chunk_blocks))   # slice blocks per dispatched chunk of a call
        # one plan's share when its slice batch is chosen automatically
        self.plan_budget = int(plan_budget_bytes) if plan_budget_bytes else max(1 << 30, self.budget // 8)
        self.max_replicas = int(max_replicas)
        self.device = device
        self.circuits = {}
        self.pending = collections.deque()   # requests with bitstrings not yet dispatched
        self.lock = threading.Condition()
        self.running = False
        self.thread = None
        self.worker = None
        self.jobs = collections.deque()      # circuits whose next replica the worker builds
        self.evict = []                      # replicas the scheduler destroys after releasing its lock
        self.worker_stop = False             # set once the scheduler has drained
        self.latencies = []                  # seconds, arrival to result, per completed request
        self.records = []                    # per completed request: circuit, queue and service seconds
        self.completed_amplitudes = 0
        self.rejected = 0
        self.failed = 0
        self.max_concurrency = 0
        self.used_bytes = 0                  # replicas ready or being built
        self.built = 0
        self.evicted = 0

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
            self.worker_stop = False
        self.worker = threading.Thread(target=self._worker_loop, name="qx-server-worker", daemon=True)
        self.worker.start()
        self.thread = threading.Thread(target=self._loop, name="qx-server", daemon=True)
        self.thread.start()

    def stop(self):
        with self.lock:
            self.running = False
            self.lock.notify_all()
        if self.thread:
            self.thread.join()
        # the scheduler has drained every request (its last builds included): the worker may stop
        with self.lock:
            self.worker_stop = True
            self.lock.notify_all()
        if self.worker:
            self.worker.join()
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

    def _fail(self, req, exc):
        """Fails a request (its sampling parent, for a candidate batch) once."""
        target = req.parent if req.parent is not None else req
        req.failed = True
        if not target.future.done():
            self.failed += 1
            target.future.set_exception(exc)

    def _enqueue(self, req):
        circ = self.circuits.get(req.circuit)
        if circ is None or circ.error is not None:
            self.rejected += 1
            self._fail(req, AdmissionError(f"unknown circuit {req.circuit}") if circ is None else circ.error)
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
        sub.first_dispatch = req.first_dispatch
        sub.parent = req
        self._enqueue(sub)

    def _record(self, req, now):
        first = req.first_dispatch if req.first_dispatch is not None else now
        self.latencies.append(now - req.arrival)
        self.records.append({"circuit": req.circuit, "total": now - req.arrival, "queue": first - req.arrival,
                             "service": now - first})

    def _finish_sample(self, req):
        s = req.sample
        self._record(req, time.monotonic())
        req.future.set_result((np.array(s["kept"][:s["n"]], dtype=np.uint64),
                               {"candidates_used": s["used"], "M": s["M"]}))

    def _sample_step(self, sub):
        req = sub.parent
        if req.first_dispatch is None:
            req.first_dispatch = sub.first_dispatch
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

    # ------------------------------------------------------- replica worker
    def _worker_loop(self):
        import torch
        torch.cuda.set_device(self.device)
        while True:
            with self.lock:
                while not self.jobs and not self.worker_stop:
                    self.lock.wait(timeout=0.05)
                if not self.jobs:
                    return
                circ = self.jobs.popleft()
            try:
                rep = _Replica(circ, self.device)
                err = None
            except Exception as e:  # plan creation failed
                rep, err = None, e
            with self.lock:
                circ.building -= 1
                if rep is not None:
                    circ.replicas.append(rep)
                    self.built += 1
                else:
                    self.used_bytes -= circ.device_bytes
                    if not circ.replicas and circ.building == 0:
                        circ.error = err
                        # nothing can serve this circuit: reject its pending work
                        for req in [r for r in self.pending if r.circuit == circ.name]:
                            self.pending.remove(req)
                            self.rejected += 1
                            self._fail(req, err)
                self.lock.notify_all()

    # --------------------------------------------------------------- scheduler
    def _idle_replica(self, circ):
        """An idle ready replica of circ, or None.  With none idle and room for another replica, reserves its
        HBM (evicting idle replicas of other circuits, least recently used first, when the budget needs it:
        they are queued in self.evict for the scheduler to destroy once it has released the lock) and asks
        the worker to build it.  Called under the lock."""
        for r in circ.replicas:
            if r.busy is None:
                return r
        if circ.error is not None or len(circ.replicas) + circ.building >= self.max_replicas:
            return None
        need = circ.device_bytes
        while self.used_bytes + need > self.budget:
            idle = [(r.last_used, id(r), r) for c in self.circuits.values() if c is not circ
                    for r in c.replicas if r.busy is None]
            if not idle:
                return None
            _, _, victim = min(idle, key=lambda t: (t[0], t[1]))
            victim.circ.replicas.remove(victim)
            self.used_bytes -= victim.device_bytes
            self.evict.append(victim)
            self.evicted += 1
        if self.evict:
            return None  # build once the evicted replicas are destroyed (next pass of the scheduler)
        self.used_bytes += need
        circ.building += 1
        self.jobs.append(circ)
        self.lock.notify_all()
        return None

    def _dispatch(self, rep, parts):
        """parts: list of (request, offset, count).  One contract call over all of them."""
        import torch
        circ = rep.circ
        now = time.monotonic()
        for req, _, _ in parts:
            if req.first_dispatch is None:
                req.first_dispatch = now
        xs = np.concatenate([req.bitstrings[o:o + c] for req, o, c in parts])
        B = len(xs)
        Bp = _bucket(B, circ.max_b)
        if Bp > B:
            xs = np.concatenate([xs, np.repeat(xs[:1], Bp - B)])
        step = circ.block_slices * self.chunk_blocks
        chunks = [(lo, min(lo + step, circ.n_slices)) for lo in range(0, circ.n_slices, step)]
        with torch.cuda.stream(rep.stream):
            hx = torch.from_numpy(xs.view(np.int64)).pin_memory()
            dx = hx.to(f"cuda:{self.device}", non_blocking=True)
            amp = torch.zeros((Bp, circ.per, 2), dtype=torch.float64, device=f"cuda:{self.device}")
        rep.busy = {"parts": parts, "keep": (hx, dx, amp), "B": B, "chunks": chunks, "next": 0}
        self._next_chunk(rep)

    def _next_chunk(self, rep):
        """Enqueues the call's next slice-range chunk on the replica's stream (after the last one, the copy of
        the amplitudes to the host) and records the event the scheduler polls."""
        import torch
        call, circ = rep.busy, rep.circ
        hx, dx, amp = call["keep"]
        lo, hi = call["chunks"][call["next"]]
        call["next"] += 1
        with torch.cuda.stream(rep.stream):
            rep.plan.contract(dx, amp, (lo, hi), stream=rep.stream)
            if call["next"] == len(call["chunks"]):
                host = torch.empty(tuple(amp.shape), dtype=torch.float64).pin_memory()
                host.copy_(amp, non_blocking=True)
                call["host"] = host
            ev = torch.cuda.Event()
            ev.record(rep.stream)
        call["event"] = ev

    def _complete(self, rep):
        call = rep.busy
        if call["next"] < len(call["chunks"]):
            self._next_chunk(rep)
            return
        rep.busy = None
        rep.last_used = time.monotonic()
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
            if req.remaining == 0 and not req.failed:
                if req.parent is not None:
                    self._sample_step(req)
                else:
                    self._record(req, now)
                    self.completed_amplitudes += req.result.size
                    req.future.set_result(req.result)

    def _fail_call(self, rep, parts, exc):
        rep.busy = None
        rep.last_used = time.monotonic()
        for req, _, _ in parts:
            self._fail(req, exc)

    def _loop(self):
        import torch
        torch.cuda.set_device(self.device)
        while True:
            progressed = False
            # completions
            for circ in list(self.circuits.values()):
                for rep in list(circ.replicas):
                    if rep.busy is not None and rep.busy["event"].query():
                        parts = rep.busy["parts"]
                        try:
                            self._complete(rep)
                        except Exception as e:  # only the requests of this call fail
                            self._fail_call(rep, parts, e)
                        progressed = True
            with self.lock:
                busy = sum(1 for c in self.circuits.values() for r in c.replicas if r.busy is not None)
                if not self.running and not self.pending and busy == 0:
                    self.lock.notify_all()
                    return
                # admission: oldest pending first; merge same-circuit work into one call
                i = 0
                while i < len(self.pending):
                    req = self.pending[i]
                    circ = self.circuits[req.circuit]
                    if req.failed or circ.error is not None:
                        del self.pending[i]
                        if not req.failed:
                            self.rejected += 1
                            self._fail(req, circ.error)
                        continue
                    rep = self._idle_replica(circ)
                    if rep is None:
                        i += 1
                        continue
                    parts, room = [], circ.max_b
                    j = i
                    while j < len(self.pending) and room > 0:
                        r2 = self.pending[j]
                        if r2.circuit != req.circuit or r2.failed:
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
                    try:
                        self._dispatch(rep, parts)
                    except Exception as e:  # only the requests of this call fail
                        self._fail_call(rep, parts, e)
                    progressed = True
                busy = sum(1 for c in self.circuits.values() for r in c.replicas if r.busy is not None)
                self.max_concurrency = max(self.max_concurrency, busy)
                victims, self.evict = self.evict, []
                if not progressed and not victims:
                    self.lock.wait(timeout=0.0005)
            # evicted replicas (idle, no longer listed) are destroyed outside the lock, before the replica
            # they made room for is reserved and built
            for victim in victims:
                victim.destroy()

    # ------------------------------------------------------------------ stats
    def stats(self):
        def pct(v):
            v = np.asarray(v) if len(v) else np.zeros(1)
            return {"p50_ms": float(np.percentile(v, 50) * 1e3), "p99_ms": float(np.percentile(v, 99) * 1e3)}

        lat = self.latencies
        per = {}
        for rec in self.records:
            per.setdefault(rec["circuit"], []).append(rec)
        by_circuit = {name: {"requests": len(rs), "total": pct([r["total"] for r in rs]),
                             "queue": pct([r["queue"] for r in rs]), "service": pct([r["service"] for r in rs])}
                      for name, rs in sorted(per.items())}
        out = {"completed_amplitudes": self.completed_amplitudes, "rejected": self.rejected, "failed": self.failed,
               "max_concurrency": self.max_concurrency, "resident_bytes": self.used_bytes,
               "replicas_built": self.built, "replicas_evicted": self.evicted, "by_circuit": by_circuit,
               "queue": pct([r["queue"] for r in self.records]),
               "service": pct([r["service"] for r in self.records])}
        out.update(pct(lat))
        return out
