"""End-to-end parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerance for complex64: max_b |a_b - ref_b| <= 1e-5 * rms_b |ref_b| over the
request's bitstrings (relative error against the batch's amplitude scale, so
near-zero amplitudes do not make the criterion meaningless).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2110_09894_amd import qxtn  # noqa: E402
from workloads import (circuit_to_network, random_grid_circuit, ghz_circuit, identity_circuit,  # noqa: E402
                       dense_chain_network, outer_thin_network, dot_pair_network,
                       mirror_circuit, greedy_tree, tree_trimming, all_bitstrings, random_bitstrings,
                       configs)
from tests._util import rms_err, gpu_amplitudes  # noqa: E402

TOL_C64 = 1e-5


def test_c1_all_64_amplitudes():
    w = configs.get("c1")
    net = w.network()
    tree, sl, _ = w.plan_inputs()
    xs = w.bitstrings()
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=len(xs))
    got = gpu_amplitudes(plan, xs)
    want = oracle.amplitudes_statevector(w.circuit(), xs)
    assert rms_err(got, want) < TOL_C64


def test_c1_deterministic_bitwise():
    w = configs.get("c1")
    tree, sl, _ = w.plan_inputs()
    xs = w.bitstrings()
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=len(xs))
    a = gpu_amplitudes(plan, xs)
    b = gpu_amplitudes(plan, xs)
    assert np.array_equal(a.view(np.float64), b.view(np.float64))


def test_normalisation_all_4096_bitstrings():
    w = configs.get("c1")
    tree, sl, _ = w.plan_inputs()
    xs = all_bitstrings(12)
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=len(xs))
    got = gpu_amplitudes(plan, xs)
    assert abs(np.sum(np.abs(got) ** 2) - 1.0) < 1e-5
    want = oracle.statevector(w.circuit()).transpose(list(range(11, -1, -1))).reshape(-1)
    assert rms_err(got, want) < TOL_C64


@pytest.mark.parametrize("js", [0, 1, 3, 4])
def test_sliced_small_network_all_js(js):
    circ = random_grid_circuit(3, 3, 6, 21)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=2)
    sl = tree_trimming(net, tree, 4, seed=2)
    xs = random_bitstrings(9, 16, 5)
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=16, slice_batch_log2=js)
    got = gpu_amplitudes(plan, xs)
    want = oracle.amplitudes_statevector(circ, xs)
    assert rms_err(got, want) < TOL_C64
    want3 = oracle.amplitudes_sliced(net, tree, xs, sl)
    assert rms_err(got, want3) < TOL_C64


@pytest.mark.parametrize("js", [6, 9])
def test_many_slices_per_block(js):
    """Blocks of 64 and 512 slices: each value's sum over a block is spread over a wavefront's lanes and
    joined in a fixed butterfly; full range against the state vector, a ragged range against the sliced
    oracle, and the same call twice bitwise."""
    circ = random_grid_circuit(4, 4, 8, 23)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=5)
    sl = tree_trimming(net, tree, 9, seed=5)
    xs = random_bitstrings(16, 8, 7)
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=8, slice_batch_log2=js)
    got = gpu_amplitudes(plan, xs)
    assert rms_err(got, oracle.amplitudes_statevector(circ, xs)) < TOL_C64
    assert np.array_equal(got.view(np.float64), gpu_amplitudes(plan, xs).view(np.float64))
    rag = gpu_amplitudes(plan, xs[:2], (5, 300))
    want = np.array([oracle.amplitude_sliced(net, tree, x, sl, (5, 300)) for x in xs[:2]])
    assert rms_err(rag, want) < TOL_C64


def test_ragged_slice_ranges_and_additivity():
    circ = random_grid_circuit(3, 4, 6, 22)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=4)
    sl = tree_trimming(net, tree, 5, seed=4)
    xs = random_bitstrings(12, 8, 6)
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=8, slice_batch_log2=2)
    full = gpu_amplitudes(plan, xs)
    parts = gpu_amplitudes(plan, xs, (0, 13)) + gpu_amplitudes(plan, xs, (13, 32))
    assert rms_err(parts, full) < 1e-6
    rag = gpu_amplitudes(plan, xs, (3, 11))
    want = np.array([oracle.amplitude_sliced(net, tree, x, sl, (3, 11)) for x in xs])
    assert rms_err(rag, want) < TOL_C64
    empty = gpu_amplitudes(plan, xs, (7, 7))
    assert np.all(empty == 0)
    # B smaller than max_bitstrings, and a single bitstring
    one = gpu_amplitudes(plan, xs[:1])
    assert abs(one[0] - full[0]) <= 1e-6 * np.sqrt(np.mean(np.abs(full) ** 2))


def test_ghz_49_qubits():
    net = circuit_to_network(ghz_circuit(49))
    tree = greedy_tree(net)
    ones = (1 << 49) - 1
    xs = np.array([0, ones, 1, 12345678901], dtype=np.uint64)
    plan = qxtn.Plan(net, tree, [], max_bitstrings=4)
    got = gpu_amplitudes(plan, xs)
    s = 1 / math.sqrt(2)
    assert abs(got[0] - s) < 1e-6 and abs(got[1] - s) < 1e-6
    assert np.max(np.abs(got[2:])) < 1e-7


@pytest.mark.parametrize("kind", ["empty", "sqrtx4", "cz2"])
def test_identity_circuits(kind):
    net = circuit_to_network(identity_circuit(6, kind))
    tree = greedy_tree(net, seed=1)
    xs = all_bitstrings(6)
    plan = qxtn.Plan(net, tree, [], max_bitstrings=64)
    got = gpu_amplitudes(plan, xs)
    want = np.zeros(64)
    want[0] = 1
    assert np.max(np.abs(got - want)) < 1e-6


def test_mirror_circuit_30_qubits_sliced():
    circ = mirror_circuit(5, 6, 6, 23)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=3)
    sl = tree_trimming(net, tree, 6, seed=3)
    xs = np.concatenate([[0], random_bitstrings(30, 7, 7)]).astype(np.uint64)
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=8)
    got = gpu_amplitudes(plan, xs)
    assert abs(got[0] - 1) < 1e-5
    assert np.max(np.abs(got[1:])) < 1e-5


@pytest.mark.parametrize("slice_id", [0, 777])
def test_c2_one_slice_against_oracle(slice_id):
    w = configs.get("c2")
    net = w.network()
    tree, sl, _ = w.plan_inputs()
    xs = w.bitstrings()
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=len(xs))
    got = gpu_amplitudes(plan, xs, (slice_id, slice_id + 1))
    # one slice, all 256 bitstrings of the workload
    want = np.array([oracle.contract_slice(net, tree, x, sl, slice_id) for x in xs])
    assert rms_err(got, want) < TOL_C64


def test_c2_full_amplitudes_two_bitstrings():
    """All 1024 slices summed (Eq. 2) for two bitstrings, against the oracle's slice sum."""
    w = configs.get("c2")
    net = w.network()
    tree, sl, _ = w.plan_inputs()
    xs = w.bitstrings()[:2]
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=256)
    got = gpu_amplitudes(plan, xs)
    want = oracle.amplitudes_sliced(net, tree, xs, sl)
    assert np.max(np.abs(got - want)) / np.sqrt(np.mean(np.abs(want) ** 2)) < TOL_C64


def test_errors_leave_plan_usable():
    w = configs.get("c1")
    tree, sl, _ = w.plan_inputs()
    xs = w.bitstrings(8)
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=8)
    x = torch.zeros(9, dtype=torch.int64, device="cuda")
    amp = torch.zeros((9, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(qxtn.QxError):
        plan.contract(x, amp)  # B > max_bitstrings
    with pytest.raises(qxtn.QxError):
        plan.contract(x[:8], amp, (0, 2))  # slice range beyond 2^0
    got = gpu_amplitudes(plan, xs)
    want = oracle.amplitudes_statevector(w.circuit(), xs)
    assert rms_err(got, want) < TOL_C64


TOL_SPLIT = 1e-4


@pytest.mark.parametrize("precision", ["split_bf16", "split_fp16"])
def test_split_precision_c1_and_sliced(precision):
    w = configs.get("c1")
    tree, sl, _ = w.plan_inputs()
    xs = w.bitstrings()
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=len(xs), precision=precision)
    got = gpu_amplitudes(plan, xs)
    want = oracle.amplitudes_statevector(w.circuit(), xs)
    assert rms_err(got, want) < TOL_SPLIT
    circ = random_grid_circuit(3, 3, 6, 21)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=2)
    sl = tree_trimming(net, tree, 4, seed=2)
    xs = random_bitstrings(9, 16, 5)
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=16, precision=precision, slice_batch_log2=2)
    assert rms_err(gpu_amplitudes(plan, xs), oracle.amplitudes_statevector(circ, xs)) < TOL_SPLIT


@pytest.mark.parametrize("precision", ["split_bf16", "split_fp16"])
def test_split_precision_c2_slice(precision):
    w = configs.get("c2")
    net = w.network()
    tree, sl, _ = w.plan_inputs()
    xs = w.bitstrings()
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=len(xs), precision=precision)
    got = gpu_amplitudes(plan, xs, (5, 6))
    want = np.array([oracle.contract_slice(net, tree, x, sl, 5) for x in xs])
    assert rms_err(got, want) < TOL_SPLIT


def test_mirror_circuit_split_bf16():
    circ = mirror_circuit(5, 6, 6, 23)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=3)
    sl = tree_trimming(net, tree, 6, seed=3)
    xs = np.concatenate([[0], random_bitstrings(30, 7, 7)]).astype(np.uint64)
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=8, precision="split_bf16")
    got = gpu_amplitudes(plan, xs)
    assert abs(got[0] - 1) < 1e-4
    assert np.max(np.abs(got[1:])) < 1e-4


def test_graph_replays_match_eager_bitwise():
    """The captured block program, replayed for every block of several calls with
    eager work in between, gives bitwise the same amplitudes as per-op launches."""
    circ = random_grid_circuit(4, 4, 8, 33)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=5)
    sl = tree_trimming(net, tree, 6, seed=5)
    xs = random_bitstrings(16, 12, 8)
    eager = qxtn.Plan(net, tree, sl, max_bitstrings=16, slice_batch_log2=2, eager=True)
    graph = qxtn.Plan(net, tree, sl, max_bitstrings=16, slice_batch_log2=2)
    want = gpu_amplitudes(eager, xs)
    for rep in range(3):
        got = gpu_amplitudes(graph, xs)
        assert np.array_equal(got.view(np.float64), want.view(np.float64)), rep
        torch.ones(1024, device="cuda").sum().item()  # unrelated eager work between replays
        # a different batch size captures and replays its own graph
        got5 = gpu_amplitudes(graph, xs[:5], (3, 60))
        want5 = gpu_amplitudes(eager, xs[:5], (3, 60))
        assert np.array_equal(got5.view(np.float64), want5.view(np.float64)), rep
    assert rms_err(want, oracle.amplitudes_statevector(circ, xs)) < TOL_C64


@pytest.fixture(scope="module")
def c2_slice777():
    """The c2 workload and the oracle's values of slice 777 for its 256 bitstrings."""
    w = configs.get("c2")
    net = w.network()
    tree, sl, _ = w.plan_inputs()
    xs = w.bitstrings()
    want = np.array([oracle.contract_slice(net, tree, x, sl, 777) for x in xs])
    return w, tree, sl, xs, want


@pytest.mark.parametrize("precision,tol", [("c64", TOL_C64), ("split_bf16", TOL_SPLIT), ("split_fp16", TOL_SPLIT)])
def test_autotuned_plan_matches_oracle(c2_slice777, precision, tol):
    """The launch configuration bench.py times (autotuned tiles, graph-replayed slice blocks), per precision."""
    w, tree, sl, xs, want = c2_slice777
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=len(xs), autotune=True, precision=precision)
    got = gpu_amplitudes(plan, xs, (777, 778))
    err = rms_err(got, want)
    print(f"c2 slice 777, {precision}, autotuned: max err / rms = {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("tile", qxtn.TILES)
@pytest.mark.parametrize("precision,tol", [("c64", TOL_C64), ("split_bf16", TOL_SPLIT), ("split_fp16", TOL_SPLIT)])
def test_c2_slice_every_forced_tile(c2_slice777, tile, precision, tol):
    """Every product of the 30-qubit plan run with one forced work-group tile, in every precision."""
    w, tree, sl, xs, want = c2_slice777
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=len(xs), precision=precision, gemm_tile=tile)
    got = gpu_amplitudes(plan, xs, (777, 778))
    assert rms_err(got, want) < tol


@pytest.fixture(scope="module")
def c2r_slice777():
    """The c2 network on the refined tree (four greedy trials re-ordered under the roofline cost), whose
    largest products are thin (one side of 16, K = 16), and the oracle's values of slice 777 for 16 bitstrings."""
    w = configs.get("c2")
    net = w.network()
    tree, sl, _ = w.plan_inputs(reconfigure=4, mem_weight=16.0)
    xs = w.bitstrings()[:16]
    want = np.array([oracle.contract_slice(net, tree, x, sl, 777) for x in xs])
    return w, tree, sl, xs, want


@pytest.mark.parametrize("tile", [None, "thin", "autotune"])
@pytest.mark.parametrize("precision,tol", [("c64", TOL_C64), ("split_bf16", TOL_SPLIT), ("split_fp16", TOL_SPLIT)])
def test_c2_refined_tree_thin_products(c2r_slice777, tile, precision, tol):
    """The refined tree's thin products in bit-scattered layouts (outputs permuted, split outputs written in
    chunks) on the default tiles, forced onto the thin kernel, and as the autotuner picks."""
    w, tree, sl, xs, want = c2r_slice777
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=len(xs), precision=precision,
                     gemm_tile=None if tile == "autotune" else tile, autotune=tile == "autotune")
    got = gpu_amplitudes(plan, xs, (777, 778))
    err = rms_err(got, want)
    print(f"c2 refined slice 777, {precision}, tile {tile}: max err / rms = {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("max_b,js", [(64, -1), (128, 0), (256, -1), (256, 0)])
def test_fp16_calibration_refined_c2(c2r_slice777, max_b, js):
    """Split FP16 scales of the refined c2 tree for plans sized for 64 to 256 bitstrings: with every
    bitstring zero its fSim-type gates leave whole batched tensors exactly zero, so the calibration
    passes use pseudo-random bitstrings; a tensor calibrated at zero would keep scale 1 and lose its
    low halves to FP16 subnormals (an error near 1e-2)."""
    w, tree, sl, xs, want = c2r_slice777
    plan = qxtn.Plan(w.network(), tree, sl, max_bitstrings=max_b, precision="split_fp16", slice_batch_log2=js)
    got = gpu_amplitudes(plan, xs, (777, 778))
    err = rms_err(got, want)
    print(f"c2 refined slice 777, split_fp16, max_bitstrings {max_b}, js {js}: max err / rms = {err:.2e}")
    assert err < TOL_SPLIT


@pytest.fixture(scope="module")
def outer_nets():
    """Long-times-short networks and the oracle's amplitudes of their one qubit."""
    out = {}
    for bits, short_first in [((17, 3, 2), False), ((17, 3, 2), True), ((18, 2, 1), False)]:
        net = outer_thin_network(*bits, seed=3, short_first=short_first)
        want = np.array([oracle.contract_slice(net, OUTER_TREE, x) for x in (0, 1)])
        out[(bits, short_first)] = (net, want)
    return out


OUTER_TREE = [(0, 1), (3, 2)]


@pytest.mark.parametrize("tile", [None] + qxtn.TILES)
@pytest.mark.parametrize("precision,tol", [("c64", TOL_C64), ("split_bf16", TOL_SPLIT), ("split_fp16", TOL_SPLIT)])
@pytest.mark.parametrize("case", [((17, 3, 2), False), ((17, 3, 2), True), ((18, 2, 1), False)])
def test_long_times_short_contraction(outer_nets, case, precision, tol, tile):
    """A 2^20-result contraction of a long operand (summed labels in the middle of its layout) with a short
    one of 4 or 8 rows over 2 or 4 terms, planned as a thin matrix product: default (thin) and every
    forced tile (split products of K 2 or 4 always run thin) against the oracle."""
    net, want = outer_nets[case]
    plan = qxtn.Plan(net, OUTER_TREE, [], max_bitstrings=2, precision=precision, gemm_tile=tile)
    got = gpu_amplitudes(plan, np.array([0, 1], np.uint64))
    err = rms_err(got, want)
    print(f"long x short {case}, {precision}, tile {tile}: max err / rms = {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("precision,tol", [("c64", TOL_C64), ("split_bf16", TOL_SPLIT)])
@pytest.mark.parametrize("bits,sliced", [((3, 3, 14), ()), ((3, 3, 14), (6, 7)), ((1, 2, 12), ()),
                                         ((2, 3, 10), ()), ((3, 1, 13), ()), ((2, 2, 16), (4, 5, 6))])
def test_long_inner_product_as_outer_product(bits, sliced, precision, tol):
    """A root inner product whose outputs are an outer product of A-only and B-only output wires (2 to 8 of
    each) per value of the varying sliced bits, on the kernel that reads each operand row once; with one
    slice block and 2^13 or more terms the sum is split over work-groups and the partial sums added in a
    second pass.  Every bitstring against the oracle's unsliced contraction."""
    net = dot_pair_network(*bits, seed=2)
    tree = [(0, 1)]
    n = bits[0] + bits[1]
    xs = all_bitstrings(n)
    want = np.array([oracle.contract_slice(net, tree, x) for x in xs])
    plan = qxtn.Plan(net, tree, list(sliced), max_bitstrings=len(xs), precision=precision,
                     slice_batch_log2=len(sliced))
    got = gpu_amplitudes(plan, xs)
    err = rms_err(got, want)
    print(f"outer dot {bits} sliced {sliced}, {precision}: max err / rms = {err:.2e}")
    assert err < tol


CHAIN_TREE = [(0, 1), (4, 2), (5, 3)]


@pytest.mark.parametrize("tile", [None] + qxtn.TILES)
@pytest.mark.parametrize("precision", ["c64", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("order", [(True, True, True, True), (True, False, True, False), (False, False, False, False)])
@pytest.mark.parametrize("sliced,js", [((), 0), ((5, 12), 2)])
def test_dense_leaves_as_matrix_product_operands(precision, order, sliced, js, tile):
    """Dense random leaves read directly by matrix-core products: leaves whose
    summed labels are (or are not) their fastest-varying ones, a product fed by a
    small contraction, and a varying sliced index shared by both operands; every
    work-group tile forced in turn."""
    net = dense_chain_network(5, order, seed=11)
    xs = random_bitstrings(10, 16, 12)
    plan = qxtn.Plan(net, CHAIN_TREE, list(sliced), max_bitstrings=64, precision=precision, slice_batch_log2=js,
                     gemm_tile=tile)
    got = gpu_amplitudes(plan, xs)
    want = oracle.amplitudes_sliced(net, CHAIN_TREE, xs, list(sliced))
    assert rms_err(got, want) < (TOL_C64 if precision == "c64" else TOL_SPLIT)


@pytest.mark.parametrize("mem_weight", [0.0, 16.0])
@pytest.mark.parametrize("precision,tol", [("c64", TOL_C64), ("split_bf16", TOL_SPLIT), ("split_fp16", TOL_SPLIT)])
def test_reconfigured_tree_against_statevector(precision, tol, mem_weight):
    # a tree refined by local sub-tree re-ordering (cheaper, different shapes) gives the same amplitudes
    from workloads import plan_network
    circ = random_grid_circuit(4, 4, 10, 61)
    net = circuit_to_network(circ)
    tree0, _, st0 = plan_network(net, 3, trials=4, seed=62)
    tree, sl, st = plan_network(net, 3, trials=4, seed=62, reconfigure=2, mem_weight=mem_weight)
    assert st["total_flops"] < st0["total_flops"] and not np.array_equal(tree, tree0)
    xs = random_bitstrings(16, 64, 63)
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=len(xs), precision=precision)
    got = gpu_amplitudes(plan, xs)
    want = oracle.amplitudes_statevector(circ, xs)
    assert rms_err(got, want) < tol


def _with_open_bits(xs, open_q):
    """Every bitstring with its open qubits replaced by each assignment j (bit i of j -> qubit open_q[i])."""
    mask = sum(1 << q for q in open_q)
    out = []
    for x in np.asarray(xs, dtype=np.uint64):
        for j in range(1 << len(open_q)):
            y = int(x) & ~mask
            for i, q in enumerate(open_q):
                y |= ((j >> i) & 1) << q
            out.append(y)
    return np.array(out, dtype=np.uint64)


@pytest.mark.parametrize("precision,tol", [("c64", TOL_C64), ("split_bf16", TOL_SPLIT), ("split_fp16", TOL_SPLIT)])
@pytest.mark.parametrize("open_q,js", [((0,), 0), ((2, 5, 7), 1), ((1, 3, 4, 8), 3)])
def test_open_output_qubits_against_statevector(precision, tol, open_q, js):
    # m open qubits: each bitstring yields the 2^m amplitudes of all values of those qubits
    circ = random_grid_circuit(3, 3, 8, 71)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=72)
    sl = tree_trimming(net, tree, 3, seed=72)
    xs = random_bitstrings(9, 16, 73)
    m = len(open_q)
    plan = qxtn.Plan(net, tree, sl, max_bitstrings=len(xs), precision=precision, open_qubits=open_q,
                     slice_batch_log2=js)
    assert plan.info()["n_open"] == m
    x = torch.from_numpy(np.ascontiguousarray(xs).view(np.int64)).cuda()
    amp = torch.zeros((len(xs), 1 << m, 2), dtype=torch.float64, device="cuda")
    plan.contract(x, amp, (0, 3))
    plan.contract(x, amp, (3, 8))  # disjoint slice ranges add (Eq. 2)
    torch.cuda.synchronize()
    h = amp.cpu().numpy()
    got = (h[..., 0] + 1j * h[..., 1]).reshape(-1)
    want = oracle.amplitudes_statevector(circ, _with_open_bits(xs, open_q))
    assert rms_err(got, want) < tol
    with pytest.raises(ValueError):
        plan.contract(x, torch.zeros((len(xs), 2), dtype=torch.float64, device="cuda") if m else amp[:1])


def test_all_qubits_open_gives_the_state():
    circ = random_grid_circuit(2, 3, 6, 74)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=75)
    plan = qxtn.Plan(net, tree, [], max_bitstrings=1, open_qubits=range(6))
    amp = torch.zeros((1, 64, 2), dtype=torch.float64, device="cuda")
    plan.contract(torch.zeros(1, dtype=torch.int64, device="cuda"), amp)
    torch.cuda.synchronize()
    h = amp.cpu().numpy()[0]
    want = oracle.amplitudes_statevector(circ, np.arange(64, dtype=np.uint64))
    assert rms_err(h[:, 0] + 1j * h[:, 1], want) < TOL_C64
    assert abs(np.sum(np.abs(want) ** 2) - 1.0) < 1e-12


@pytest.mark.parametrize("bits", [8, 9, 10, 14, 15])
@pytest.mark.parametrize("open_q", [(), (0, 1)])
def test_long_inner_products(bits, open_q):
    # two dense leaves sharing `bits` summed labels, one output wire each: the root is an inner product of
    # K = 2^bits terms (lane groups of 16 / 32 / 64 up to 2^14, a work-group per output above)
    from workloads import Network
    rng = np.random.default_rng(100 + bits)
    shape = (2,) * (bits + 1)
    t1 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    t2 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ks = tuple(range(bits))
    net = Network([t1, t2], [ks + (100,), ks + (101,)], [100, 101], 2)
    tree = np.array([[0, 1]], dtype=np.int32)
    xs = np.arange(4, dtype=np.uint64)
    plan = qxtn.Plan(net, tree, [], max_bitstrings=4, open_qubits=open_q)
    m = len(open_q)
    x = torch.from_numpy(xs.view(np.int64)).cuda()
    amp = torch.zeros((4, 1 << m, 2), dtype=torch.float64, device="cuda")
    plan.contract(x, amp)
    torch.cuda.synchronize()
    h = amp.cpu().numpy()
    got = (h[..., 0] + 1j * h[..., 1]).reshape(-1)
    want = np.array([oracle.contract_slice(net, tree, int(y)) for y in _with_open_bits(xs, open_q)])
    assert rms_err(got, want) < TOL_C64
