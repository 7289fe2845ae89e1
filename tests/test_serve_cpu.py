"""Scheduler logic of the server on the CPU: admission by HBM budget, replica building and eviction by the
worker thread, continuous batching and failure handling, with fake replicas standing in for device plans
(each fake call returns, for every bitstring, the bitstring's value as its amplitude)."""
import threading
import time

import numpy as np
import pytest

from paper_2110_09894_amd import serve
from workloads import circuit_to_network, random_grid_circuit, greedy_tree, ghz_circuit, tree_trimming


class _Event:
    def __init__(self, polls):
        self.left = polls

    def query(self):
        self.left -= 1
        return self.left <= 0


class _FakeReplica:
    made, destroyed = [], []
    lock = threading.Lock()

    def __init__(self, circ, device):
        if circ.name.startswith("broken"):
            raise RuntimeError("plan creation failed")
        time.sleep(0.01)
        self.circ = circ
        self.device_bytes = circ.device_bytes
        self.busy = None
        self.last_used = time.monotonic()
        with _FakeReplica.lock:
            _FakeReplica.made.append(circ.name)

    def destroy(self):
        time.sleep(0.01)
        with _FakeReplica.lock:
            _FakeReplica.destroyed.append(self.circ.name)


class _H:
    def __init__(self, a):
        self.a = a

    def numpy(self):
        return self.a


def _fake_dispatch(self, rep, parts):
    now = time.monotonic()
    for req, _, _ in parts:
        if req.first_dispatch is None:
            req.first_dispatch = now
    xs = np.concatenate([req.bitstrings[o:o + c] for req, o, c in parts])
    host = np.zeros((len(xs), rep.circ.per, 2))
    step = rep.circ.block_slices * self.chunk_blocks
    chunks = [(lo, min(lo + step, rep.circ.n_slices)) for lo in range(0, rep.circ.n_slices, step)]
    rep.busy = {"parts": parts, "keep": (xs, host), "B": len(xs), "chunks": chunks, "next": 0}
    self._next_chunk(rep)


def _fake_next_chunk(self, rep):
    """A chunk adds its share: after every chunk each bitstring's value is the bitstring itself."""
    call = rep.busy
    xs, host = call["keep"]
    lo, hi = call["chunks"][call["next"]]
    call["next"] += 1
    host[:, :, 0] += xs.astype(np.float64)[:, None] * (hi - lo) / rep.circ.n_slices
    if call["next"] == len(call["chunks"]):
        call["host"] = _H(host)
    call["event"] = _Event(2)
    self.chunks_run = getattr(self, "chunks_run", 0) + 1


@pytest.fixture()
def fake(monkeypatch):
    import torch
    monkeypatch.setattr(serve, "_Replica", _FakeReplica)
    monkeypatch.setattr(serve.Server, "_dispatch", _fake_dispatch)
    monkeypatch.setattr(serve.Server, "_next_chunk", _fake_next_chunk)
    monkeypatch.setattr(torch.cuda, "set_device", lambda d: None)
    _FakeReplica.made, _FakeReplica.destroyed = [], []
    return _FakeReplica


def _nets():
    out = {}
    for name, (r, c, d, s, k) in {"a": (2, 3, 4, 1, 0), "b": (3, 3, 4, 2, 2), "c": (2, 2, 3, 3, 0)}.items():
        net = circuit_to_network(random_grid_circuit(r, c, d, s))
        tree = greedy_tree(net, seed=s)
        out[name] = (net, tree, tree_trimming(net, tree, k, seed=s) if k else [])
    return out


def _check(res, xs):
    assert np.array_equal(np.real(res), xs.astype(np.float64))


def test_eviction_under_tight_budget_cpu(fake):
    nets = _nets()
    sizes = {n: serve.Server().register(n, *v, max_bitstrings=16) for n, v in nets.items()}
    srv = serve.Server(hbm_budget_bytes=max(sizes.values()) + 8, max_replicas=1)
    for n, v in nets.items():
        srv.register(n, *v, max_bitstrings=16)
    srv.start()
    order = ["a", "b", "c", "a", "b"]
    reqs = [(n, np.arange(i, i + 10, dtype=np.uint64)) for i, n in enumerate(order)]
    futs = [(xs, srv.submit_amplitudes(n, xs)) for n, xs in reqs]
    for xs, f in futs:
        _check(f.result(timeout=20), xs)
    st = srv.stats()
    srv.stop()
    assert st["resident_bytes"] <= max(sizes.values()) + 8
    assert st["replicas_evicted"] >= 2 and st["replicas_built"] >= 3
    assert len(fake.made) == len(fake.destroyed)  # stop() destroys what is left


def test_batching_merges_same_circuit_requests_cpu(fake):
    nets = _nets()
    srv = serve.Server(max_replicas=1)
    srv.register("a", *nets["a"], max_bitstrings=64)
    reqs = [np.arange(7 * i, 7 * i + 7, dtype=np.uint64) for i in range(20)]
    futs = [srv.submit_amplitudes("a", xs) for xs in reqs]  # queued before the scheduler starts
    srv.start()
    for xs, f in zip(reqs, futs):
        _check(f.result(timeout=20), xs)
    st = srv.stats()
    srv.stop()
    assert fake.made == ["a"]
    assert st["by_circuit"]["a"]["requests"] == 20
    # 140 bitstrings in calls of at most 64: the first nine requests share one call
    assert st["queue"]["p99_ms"] >= 0 and st["service"]["p50_ms"] >= 0


def test_failed_build_rejects_only_its_circuit_cpu(fake):
    nets = _nets()
    srv = serve.Server(max_replicas=1)
    srv.register("a", *nets["a"], max_bitstrings=16)
    srv.register("broken", *nets["a"], max_bitstrings=16)
    srv.start()
    xs = np.arange(5, dtype=np.uint64)
    bad = srv.submit_amplitudes("broken", xs)
    bad_sample = srv.submit_sample("broken", 3, xs, np.full(5, 0.5), batch=2)
    good = srv.submit_amplitudes("a", xs)
    with pytest.raises(RuntimeError):
        bad.result(timeout=20)
    with pytest.raises(RuntimeError):
        bad_sample.result(timeout=20)
    _check(good.result(timeout=20), xs)
    with pytest.raises(RuntimeError):
        srv.submit_amplitudes("broken", xs).result(timeout=20)
    st = srv.stats()
    srv.stop()
    assert st["failed"] == 3 and st["rejected"] >= 2


def test_failing_call_fails_its_requests_and_the_loop_continues_cpu(fake, monkeypatch):
    nets = _nets()
    srv = serve.Server(max_replicas=1)
    srv.register("a", *nets["a"], max_bitstrings=4)
    calls = {"n": 0}
    orig = serve.Server._dispatch

    def flaky(self, rep, parts):
        calls["n"] += 1
        if calls["n"] == 1:
            raise RuntimeError("launch failed")
        orig(self, rep, parts)
    monkeypatch.setattr(serve.Server, "_dispatch", flaky)
    srv.start()
    first = srv.submit_amplitudes("a", np.arange(3, dtype=np.uint64))
    with pytest.raises(RuntimeError):
        first.result(timeout=20)
    xs = np.arange(10, 13, dtype=np.uint64)
    _check(srv.submit_amplitudes("a", xs).result(timeout=20), xs)
    srv.stop()


def test_calls_run_in_slice_block_chunks_cpu(fake):
    """Circuit b has 2 sliced indices: with one slice per block a call runs as 4 chunks, whose partial sums
    add up (Eq. 2); the merged call of several requests is chunked once."""
    nets = _nets()
    srv = serve.Server(max_replicas=1)
    srv.register("b", *nets["b"], max_bitstrings=64, slice_batch_log2=0)
    reqs = [np.arange(5 * i, 5 * i + 5, dtype=np.uint64) for i in range(3)]
    futs = [srv.submit_amplitudes("b", xs) for xs in reqs]
    srv.start()
    for xs, f in zip(reqs, futs):
        assert np.allclose(np.real(f.result(timeout=20)), xs.astype(np.float64))
    srv.stop()
    assert srv.circuits["b"].n_slices == 4 and srv.chunks_run == 4
