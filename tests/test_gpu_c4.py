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
from tests._util import gpu_amplitudes  # noqa: E402


@pytest.fixture(scope="module")
def c4():
    w = configs.get("c4")
    tree, sl, st = w.plan_inputs()
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=1, autotune=True)
    return w, tree, sl, plan


@pytest.mark.parametrize("slice_id", [0, 5])
def test_c4_single_slice_against_oracle(c4, slice_id):
    w, tree, sl, plan = c4
    x = w.bitstrings()
    got = gpu_amplitudes(plan, x, (slice_id, slice_id + 1))[0]
    want = oracle.contract_slice(w.network(), tree, x[0], sl, slice_id)
    assert abs(got - want) <= 1e-5 * abs(want) + 1e-30, (got, want)


def test_c4_slice_range_additivity(c4):
    w, tree, sl, plan = c4
    x = w.bitstrings()
    whole = gpu_amplitudes(plan, x, (0, 16))[0]
    parts = gpu_amplitudes(plan, x, (0, 5))[0] + gpu_amplitudes(plan, x, (5, 16))[0]
    assert abs(whole - parts) <= 1e-9 * max(abs(whole), 1e-300)
