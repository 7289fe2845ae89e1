"""Host-side parts of the benchmark: the oracle-timing leg, the single-GPU guard and the traffic gate."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle  # noqa: E402
from workloads import configs  # noqa: E402


def test_cpu_baseline_fields_and_slice0_values():
    w = configs.get("c1")
    tree, sliced, _ = w.plan_inputs()
    xs = w.bitstrings()
    cb, ref = bench.cpu_baseline(w, tree, sliced, xs, 0.3)
    assert cb["kind"] == "oracle" and cb["unit"] == "amplitudes/s"
    assert cb["value"] > 0 and cb["cores"] >= 1 and cb["host_cpus"] >= 1
    assert "slice-amplitudes" in cb["sample"]
    st = cb.get("single_thread")
    if st is not None:
        assert st["cores"] == 1 and st["value"] > 0
    # the values handed back are slice 0's amplitudes of the first bitstrings (no slicing here: the amplitudes)
    assert 1 <= len(ref) <= len(xs)
    want = oracle.amplitudes_statevector(w.circuit(), xs[:len(ref)])
    assert np.max(np.abs(ref - want)) < 1e-12


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_reported_only_for_matching_sources():
    with open(bench.TRAFFIC_FILE) as f:
        blob = json.loads(f.read().split("```json", 1)[1].split("```", 1)[0])
    got = bench.measured_traffic("k_gemm_f32")
    if blob.get("sources_digest") == bench.sources_digest():
        assert got == blob["kernels"]["k_gemm_f32"]["traffic_bytes_per_launch"]
    else:
        assert got is None
    assert bench.measured_traffic("no_such_kernel") is None


def test_trace_calls_groups_dispatches_by_contract_call(tmp_path):
    """The trace summaries split a kernel trace at every k_block_finish and label calls by the matrix-product
    kernel family they launch (host logic only, on a synthetic trace)."""
    import sqlite3
    db = tmp_path / "t.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, duration integer, start integer)")
    seq = ["void qx::k_gemm_f32<128, 64, true, true>(qx::GemmArgs)", "qx::k_simt(qx::SimtArgs)",
           "qx::k_block_finish(qx::BlockArgs, double*)",
           "void qx::k_gemm_bf16s<256, 128, 4, 2, 3, true, false>(qx::GemmArgs)",
           "qx::k_block_finish(qx::BlockArgs, double*)", "qx::k_block_finish(qx::BlockArgs, double*)"]
    for i, n in enumerate(seq):
        con.execute("insert into kernels values (?, ?, ?)", (n, 100 + i, i))
    con.commit()
    rows, calls = bench.trace_calls(str(db))
    assert len(rows) == 6
    assert [len(c) for c in calls["c64"]] == [3]
    assert [len(c) for c in calls["split_bf16"]] == [2]
    assert [len(c) for c in calls[None]] == [1]
    assert bench._tile_of(seq[3]) == "256x128" and bench._family(seq[0]) == "k_gemm_f32"
