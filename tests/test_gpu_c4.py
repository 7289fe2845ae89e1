"""49-qubit 7x7 depth-14 network with 24 sliced indices, one bitstring (GPU).

Runs the launch configuration bench.py times for this workload (autotuned tiles, graph-replayed slice
blocks) in every precision, on the configured greedy tree and on the refined tree, against FP64 oracle
values of single slices and of the first 64-slice block (tests/golden/c4_slices_*.json, written by
tests/golden/make_c4_oracle.py from the oracle alone).

Error metric for one bitstring (reading 18): a slice's value is one term of the amplitude's sum over
slices (Eq. 2).  With e_s = |got_s - want_s| / rms_{s' in S} |want_s'| over the 11 sampled slices S, every
e_s must be <= 3 tol and rms_s e_s <= tol; the first block's sum must satisfy
|got - want| / sqrt(sum_s |want_s|^2) <= tol.  tol = 1e-5 for complex64, 1e-4 for split precision.
"""
import json
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2110_09894_amd import qxtn  # noqa: E402
from workloads import configs  # noqa: E402
from tests._util import gpu_amplitudes  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = {"c64": 1e-5, "split_bf16": 1e-4, "split_fp16": 1e-4}


def _load(kind):
    with open(os.path.join(GOLDEN, f"c4_slices_{kind}.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module", params=["greedy", "refined"])
def c4(request):
    kind = request.param
    g = _load(kind)
    w = configs.get("c4")
    if kind == "greedy":
        tree, sl, _ = w.plan_inputs()
    else:
        # the refined tree is a plan input stored with its oracle values (planning it takes about a minute)
        tree = np.asarray(g["tree_ssa"], dtype=np.int32).reshape(-1, 2)
        sl = g["sliced"]
    assert [int(v) for v in sl] == [int(v) for v in g["sliced"]], "golden values were made for other slices"
    x = w.bitstrings()
    assert int(x[0]) == int(g["bitstring"])
    want = {int(s): complex(*v) for s, v in g["values"].items()}
    return kind, w, tree, sl, x, want


def _sample(want):
    """Slices 0 and 5, three more of the first block and the six seeded ones beyond it (some slice sets
    have exactly-zero slices, which the GPU must reproduce: their e_s is |got| / rms)."""
    extra = sorted(s for s in want if s >= 64)
    return [0, 5, 17, 38, 62] + extra


@pytest.mark.parametrize("precision", ["c64", "split_bf16", "split_fp16"])
def test_c4_slices_and_block_against_oracle(c4, precision):
    kind, w, tree, sl, x, want = c4
    tol = TOL[precision]
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=1, autotune=True, precision=precision)
    S = _sample(want)
    got = np.array([gpu_amplitudes(plan, x, (s, s + 1))[0] for s in S])
    ref = np.array([want[s] for s in S])
    e = np.abs(got - ref) / np.sqrt(np.mean(np.abs(ref) ** 2))
    print(f"c4 {kind} {precision}: per-slice e_s {np.array2string(e, precision=2)}, rms {np.sqrt(np.mean(e ** 2)):.2e}")
    assert np.all(e <= 3 * tol), (S, e)
    assert np.sqrt(np.mean(e ** 2)) <= tol, e
    # the first 64-slice block summed by the slice-sum kernel (Eq. 2)
    blk = gpu_amplitudes(plan, x, (0, 64))[0]
    vals = [want[s] for s in range(64)]
    wsum = complex(math.fsum(v.real for v in vals), math.fsum(v.imag for v in vals))
    rss = math.sqrt(sum(abs(v) ** 2 for v in vals))
    print(f"c4 {kind} {precision}: block 0..63 error / rss {abs(blk - wsum) / rss:.2e}")
    assert abs(blk - wsum) <= tol * rss
    plan.destroy()


def test_c4_slice_range_additivity(c4):
    kind, w, tree, sl, x, want = c4
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=1, autotune=True)
    whole = gpu_amplitudes(plan, x, (0, 16))[0]
    parts = gpu_amplitudes(plan, x, (0, 5))[0] + gpu_amplitudes(plan, x, (5, 16))[0]
    assert abs(whole - parts) <= 1e-9 * max(abs(whole), 1e-300)
    plan.destroy()
