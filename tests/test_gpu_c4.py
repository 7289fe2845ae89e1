"""49-qubit 7x7 depth-14 network with 24 sliced indices, one bitstring (GPU).

Runs the launch configuration bench.py times for this workload (autotuned tiles,
graph-replayed block program) and checks two single slices against the FP64
oracle, plus additivity of slice ranges.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2110_09894_amd import qxtn  # noqa: E402
from workloads import configs  # noqa: E402
from tests._util import gpu_amplitudes, rms_err  # noqa: E402


@pytest.fixture(scope="module")
def c4():
    w = configs.get("c4")
    tree, sl, st = w.plan_inputs()
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=1, autotune=True)
    return w, tree, sl, plan


def test_c4_single_slices_against_oracle(c4):
    """Slices 0 and 5 one at a time; error metric of the amplitude tests (max |err| over the values
    compared, divided by their rms), complex64 gate 1e-5."""
    w, tree, sl, plan = c4
    x = w.bitstrings()
    ids = [0, 5]
    got = np.array([gpu_amplitudes(plan, x, (s, s + 1))[0] for s in ids])
    want = np.array([oracle.contract_slice(w.network(), tree, x[0], sl, s) for s in ids])
    assert rms_err(got, want) < 1e-5, (got, want)


def test_c4_slice_range_additivity(c4):
    w, tree, sl, plan = c4
    x = w.bitstrings()
    whole = gpu_amplitudes(plan, x, (0, 16))[0]
    parts = gpu_amplitudes(plan, x, (0, 5))[0] + gpu_amplitudes(plan, x, (5, 16))[0]
    assert abs(whole - parts) <= 1e-9 * max(abs(whole), 1e-300)
