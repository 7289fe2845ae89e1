"""Pins of the FP64 oracle against closed forms, invariants and brute force (CPU only).

The paper prints no amplitude, so every value pin is mathematical: gate
algebra, single-gate closed forms, the three independent oracle computations
agreeing, normalisation, identity / mirror / GHZ circuits, slice additivity
(Eq. 2) and independence from the contraction order (Sec. III-A).  A few tests
plant a plausible mistake in an oracle input on the CPU and check that a pin
catches it.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from workloads import (circuit_to_network, random_grid_circuit, ghz_circuit, identity_circuit,
                       mirror_circuit, greedy_tree, tree_trimming, tree_stats, all_bitstrings,
                       random_bitstrings, Network, Circuit)
from workloads import circuits as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _amps(net, tree, xs, sliced=()):
    return oracle.amplitudes_sliced(net, tree, xs, sliced)


# ---------------------------------------------------------------- gate algebra
@pytest.mark.parametrize("m", [C.SQRT_X, C.SQRT_Y, C.SQRT_W, C.CZ, C.CNOT, C.H])
def test_gates_unitary(m):
    assert np.allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-15)


@pytest.mark.parametrize("root,p", [(C.SQRT_X, C.X), (C.SQRT_Y, C.Y), (C.SQRT_W, C.W)])
def test_principal_roots_square(root, p):
    assert np.allclose(root @ root, p, atol=1e-15)


def test_sqrt_matrices_closed_form():
    s = 1 / math.sqrt(2)
    assert np.allclose(C.SQRT_X, 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]]))
    assert np.allclose(C.SQRT_Y, 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]]))
    assert np.allclose(C.SQRT_W, np.array([[(1 + 1j) / 2, -1j * s], [s, (1 + 1j) / 2]]))


def test_cz_reshape_sign():
    t = C.CZ.reshape(2, 2, 2, 2)
    for a in range(2):
        for b in range(2):
            for c in range(2):
                for d in range(2):
                    want = (a == c) * (b == d) * (-1 if a and b else 1)
                    assert t[a, b, c, d] == want


def test_cz_counts():
    assert random_grid_circuit(3, 4, 8, 1).count("cz") == 34
    assert random_grid_circuit(5, 6, 12, 2).count("cz") == 147
    assert random_grid_circuit(7, 7, 14, 4).count("cz") == 294
    assert circuit_to_network(random_grid_circuit(3, 4, 8, 1)).n_tensors == 142
    assert circuit_to_network(random_grid_circuit(5, 6, 12, 2)).n_tensors == 537
    assert circuit_to_network(random_grid_circuit(7, 7, 14, 4)).n_tensors == 1029


# ---------------------------------------------------------------- closed forms
def _single(name, m, n=1, q=0):
    c = Circuit(n)
    c.add(name, (q,), m)
    return c


@pytest.mark.parametrize("gate,want", [
    (C.SQRT_X, [(1 + 1j) / 2, (1 - 1j) / 2]),
    (C.SQRT_Y, [(1 + 1j) / 2, (1 + 1j) / 2]),
    (C.SQRT_W, [(1 + 1j) / 2, 1 / math.sqrt(2)]),
    (C.H, [1 / math.sqrt(2), 1 / math.sqrt(2)]),
])
def test_single_gate_amplitudes(gate, want):
    circ = _single("g", gate)
    net = circuit_to_network(circ)
    tree = greedy_tree(net)
    for x in (0, 1):
        assert abs(oracle.contract_slice(net, tree, x) - want[x]) < 1e-15
        assert abs(oracle.amplitude_bruteforce(net, x) - want[x]) < 1e-15
        assert abs(oracle.amplitudes_statevector(circ, [x])[0] - want[x]) < 1e-15


def test_qubit_bit_order_and_cz_phase():
    # sqrt(X) on q0, sqrt(Y) on q1, then CZ(q0, q1):
    # a(x) = <x0|sqrtX|0> <x1|sqrtY|0> * (-1)^(x0 x1), with bit q of x = qubit q.
    circ = Circuit(2)
    circ.add("sqrt_x", (0,), C.SQRT_X).add("sqrt_y", (1,), C.SQRT_Y).add("cz", (0, 1), C.CZ)
    vx = [(1 + 1j) / 2, (1 - 1j) / 2]
    vy = [(1 + 1j) / 2, (1 + 1j) / 2]
    net = circuit_to_network(circ)
    tree = greedy_tree(net)
    for x in range(4):
        x0, x1 = x & 1, (x >> 1) & 1
        want = vx[x0] * vy[x1] * (-1 if x0 and x1 else 1)
        assert abs(oracle.contract_slice(net, tree, x) - want) < 1e-15
        assert abs(oracle.amplitude_bruteforce(net, x) - want) < 1e-15
        assert abs(oracle.amplitudes_statevector(circ, [x])[0] - want) < 1e-15
    # x = 0b11: -((1-i)/2)((1+i)/2) = -1/2
    assert abs(oracle.contract_slice(net, tree, 3) - (-0.5)) < 1e-15


# ------------------------------------------- three computations of one definition
@pytest.mark.parametrize("rows,cols,depth,seed", [(2, 2, 3, 11), (2, 3, 2, 12), (1, 4, 4, 13), (1, 3, 5, 14)])
def test_o1_o2_o3_agree(rows, cols, depth, seed):
    circ = random_grid_circuit(rows, cols, depth, seed)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=seed)
    xs = all_bitstrings(circ.n_qubits)
    a1 = oracle.amplitudes_statevector(circ, xs)
    a3 = _amps(net, tree, xs)
    assert np.max(np.abs(a1 - a3)) < 1e-14
    for x in xs[:: max(1, len(xs) // 4)]:
        assert abs(oracle.amplitude_bruteforce(net, x) - a1[int(x)]) < 1e-14


def test_c1_complete_against_statevector():
    circ = random_grid_circuit(3, 4, 8, 1)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=5)
    xs = random_bitstrings(12, 64, 1001)
    a1 = oracle.amplitudes_statevector(circ, xs)
    a3 = _amps(net, tree, xs)
    assert np.max(np.abs(a1 - a3)) < 1e-14


# ---------------------------------------------------------------- invariants
def test_normalisation_statevector_12q():
    psi = oracle.statevector(random_grid_circuit(3, 4, 8, 1))
    assert abs(np.sum(np.abs(psi) ** 2) - 1.0) < 1e-12


def test_normalisation_tree_6q():
    circ = random_grid_circuit(2, 3, 4, 21)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=3)
    a = _amps(net, tree, all_bitstrings(6))
    assert abs(np.sum(np.abs(a) ** 2) - 1.0) < 1e-13


@pytest.mark.parametrize("kind", ["empty", "sqrtx4", "cz2"])
def test_identity_circuits(kind):
    circ = identity_circuit(5, kind)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=1)
    a = _amps(net, tree, all_bitstrings(5))
    want = np.zeros(32)
    want[0] = 1
    assert np.max(np.abs(a - want)) < 1e-14


def test_mirror_circuit_sliced():
    circ = mirror_circuit(2, 3, 3, 7)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=2)
    sliced = tree_trimming(net, tree, 3, seed=2)
    xs = [0, 1, 5, 63, 42]
    a = _amps(net, tree, xs, sliced)
    assert abs(a[0] - 1) < 1e-13
    assert np.max(np.abs(a[1:])) < 1e-13


@pytest.mark.parametrize("n", [2, 3, 7, 20])
def test_ghz(n):
    circ = ghz_circuit(n)
    net = circuit_to_network(circ)
    tree = greedy_tree(net)
    ones = (1 << n) - 1
    s = 1 / math.sqrt(2)
    assert abs(oracle.contract_slice(net, tree, 0) - s) < 1e-15
    assert abs(oracle.contract_slice(net, tree, ones) - s) < 1e-15
    for x in [1, ones - 1, 1 << (n - 1), 5 % (1 << n)]:
        if x not in (0, ones):
            assert abs(oracle.contract_slice(net, tree, x)) < 1e-15


def test_ghz_width_matches_table_ii():
    # Table II lists the GHZ circuit with treewidth 2 (largest intermediate rank).
    for n in (8, 49):
        net = circuit_to_network(ghz_circuit(n))
        assert tree_stats(net, greedy_tree(net))["width"] == 2


def test_slice_additivity_eq2():
    circ = random_grid_circuit(2, 3, 4, 31)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=4)
    sliced = tree_trimming(net, tree, 4, seed=4)
    xs = random_bitstrings(6, 6, 3)
    full = _amps(net, tree, xs)
    sl = _amps(net, tree, xs, sliced)
    assert np.max(np.abs(full - sl)) < 1e-14
    # disjoint slice ranges add up to the full range
    for x in xs[:2]:
        lo = oracle.amplitude_sliced(net, tree, x, sliced, (0, 5))
        hi = oracle.amplitude_sliced(net, tree, x, sliced, (5, 16))
        assert abs(lo + hi - oracle.amplitude_sliced(net, tree, x, sliced)) < 1e-15


def test_order_invariance():
    circ = random_grid_circuit(2, 3, 4, 41)
    net = circuit_to_network(circ)
    t1 = greedy_tree(net, seed=1)
    t2 = greedy_tree(net, seed=2, alpha=0.3, temperature=2.0)
    assert not np.array_equal(t1, t2)
    # a third, naive left-to-right order
    n = net.n_tensors
    t3 = np.array([(0 if i == 0 else n + i - 1, i + 1) for i in range(n - 1)], dtype=np.int32)
    xs = random_bitstrings(6, 8, 4)
    a1, a2, a3 = (_amps(net, t, xs) for t in (t1, t2, t3))
    assert np.max(np.abs(a1 - a2)) < 1e-14 and np.max(np.abs(a1 - a3)) < 1e-14


# ------------------------------------------------------ worked examples Eq.1/Eq.2
def _letter_net(spec, seed):
    rng = np.random.default_rng(seed)
    names = sorted(spec["tensors"])
    tensors, indices = [], []
    for nm in names:
        ix = tuple(ord(ch) - ord("a") for ch in spec["tensors"][nm])
        t = rng.standard_normal((2,) * len(ix)) + 1j * rng.standard_normal((2,) * len(ix))
        tensors.append(t)
        indices.append(ix)
    outs = [ord(ch) - ord("a") for ch in spec["open"]]
    return Network(tensors, indices, outs, len(outs))


def test_eq1_example_network():
    spec = json.load(open(os.path.join(GOLDEN, "eq1_eq2_networks.json")))["eq1"]
    net = _letter_net(spec, 7)
    A, B, Cc, D, E = net.tensors
    tree = greedy_tree(net, seed=0)
    for x in range(4):
        l, m = x & 1, (x >> 1) & 1
        # Eq. (1) summed explicitly over g, h, i, j, k with nested loops
        want = 0j
        for g in range(2):
            for h in range(2):
                for i in range(2):
                    for j in range(2):
                        for k in range(2):
                            want += A[g, h] * B[h, i] * Cc[i, j] * D[g, k] * E[j, k, l, m]
        assert abs(oracle.contract_slice(net, tree, x) - want) < 1e-13
        assert abs(oracle.amplitude_bruteforce(net, x) - want) < 1e-13


def test_eq2_example_slicing():
    spec = json.load(open(os.path.join(GOLDEN, "eq1_eq2_networks.json")))["eq2"]
    net = _letter_net(spec, 8)
    A, B, Cc, D = net.tensors
    tree = greedy_tree(net, seed=0)
    g_label = ord(spec["sliced"]) - ord("a")
    want = sum(A[g, h] * B[h, i] * Cc[i, j] * D[g, j]
               for g in range(2) for h in range(2) for i in range(2) for j in range(2))
    parts = [oracle.contract_slice(net, tree, 0, [g_label], g) for g in range(2)]
    for g in range(2):
        inner = sum(A[g, h] * B[h, i] * Cc[i, j] * D[g, j]
                    for h in range(2) for i in range(2) for j in range(2))
        assert abs(parts[g] - inner) < 1e-13
    assert abs(sum(parts) - want) < 1e-13
    assert abs(oracle.amplitude_sliced(net, tree, 0, [g_label]) - want) < 1e-13


# ---------------------------------------------------- planted mistakes are caught
def test_planted_transposed_gate_is_caught():
    circ = random_grid_circuit(2, 2, 3, 51)
    net = circuit_to_network(circ)
    # transpose the first sqrt(Y)/sqrt(W) leaf (operand order mistake)
    bad = Network(net.tensors, net.indices, net.output_labels, net.n_qubits)
    for i, t in enumerate(bad.tensors):
        if t.ndim == 2 and not np.allclose(t, t.T):
            bad.tensors[i] = np.ascontiguousarray(t.T)
            break
    tree = greedy_tree(net, seed=1)
    xs = all_bitstrings(4)
    good = oracle.amplitudes_statevector(circ, xs)
    assert np.max(np.abs(_amps(bad, tree, xs) - good)) > 1e-3


def test_planted_cz_sign_is_caught():
    circ = random_grid_circuit(2, 2, 3, 52)
    net = circuit_to_network(circ)
    bad = Network(net.tensors, net.indices, net.output_labels, net.n_qubits)
    for i, t in enumerate(bad.tensors):
        if t.ndim == 4:
            bad.tensors[i] = np.abs(t)
            break
    tree = greedy_tree(net, seed=1)
    xs = all_bitstrings(4)
    good = oracle.amplitudes_statevector(circ, xs)
    assert np.max(np.abs(_amps(bad, tree, xs) - good)) > 1e-3


def test_planted_dropped_slice_is_caught():
    circ = random_grid_circuit(2, 3, 4, 53)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=4)
    sliced = tree_trimming(net, tree, 3, seed=4)
    xs = random_bitstrings(6, 4, 9)
    full = _amps(net, tree, xs)
    dropped = np.array([oracle.amplitude_sliced(net, tree, x, sliced, (0, 7)) for x in xs])
    assert np.max(np.abs(full - dropped)) > 1e-6
