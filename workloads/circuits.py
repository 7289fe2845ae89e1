"""Seeded synthetic quantum circuits (input generator; holds no contraction arithmetic).

A circuit is a list of gate applications ``(name, qubits, matrix)`` on ``n``
qubits that all start in |0>.  ``matrix`` is the gate's unitary as a complex128
array: 2x2 for one qubit, 4x4 for two qubits with the first listed qubit as the
more significant bit of the row/column index.

The random grid family follows the workload description used for the
benchmarks: an R x C qubit grid, ``depth`` layers, each layer applying a random
single-qubit gate from {sqrt(X), sqrt(Y), sqrt(W)} to every qubit and then CZ on
one of four alternating nearest-neighbour coupling patterns.  The paper itself
only names Boixo-style random circuits (Sec. IV-B) without defining them, so the
gate matrices, the pattern rule and the random draws below are this project's
reading:

* sqrt(P) is the principal square root ((1+i)/2) I + ((1-i)/2) P for
  P in {X, Y, W}, W = (X+Y)/sqrt(2);
* layer l uses coupling pattern l mod 4: 0 horizontal pairs with even column,
  1 horizontal with odd column, 2 vertical with even row, 3 vertical with odd
  row;
* each layer draws every qubit's gate uniformly and independently from
  numpy.random.Generator(PCG64(seed));
* qubit q = r * C + c (row-major).
"""
from __future__ import annotations

import numpy as np

_S2 = np.sqrt(2.0)

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
W = (X + Y) / _S2
H = (X + Z) / _S2


def principal_sqrt_pauli(p: np.ndarray) -> np.ndarray:
    """Principal square root of an involutory Hermitian 2x2 matrix P (P^2 = I)."""
    return 0.5 * (1 + 1j) * I2 + 0.5 * (1 - 1j) * p


SQRT_X = principal_sqrt_pauli(X)
SQRT_Y = principal_sqrt_pauli(Y)
SQRT_W = principal_sqrt_pauli(W)
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)

SINGLE_QUBIT_SET = (("sqrt_x", SQRT_X), ("sqrt_y", SQRT_Y), ("sqrt_w", SQRT_W))


class Circuit:
    """n qubits initialised to |0>, followed by ``ops`` in application order."""

    def __init__(self, n_qubits: int, ops=None, name: str = "circuit"):
        self.n_qubits = int(n_qubits)
        self.ops = list(ops or [])
        self.name = name

    def add(self, name: str, qubits, matrix) -> "Circuit":
        qubits = tuple(int(q) for q in qubits)
        m = np.asarray(matrix, dtype=np.complex128)
        assert m.shape == (2 ** len(qubits),) * 2
        assert all(0 <= q < self.n_qubits for q in qubits) and len(set(qubits)) == len(qubits)
        self.ops.append((name, qubits, m))
        return self

    def inverse(self) -> "Circuit":
        """Gates of the adjoint circuit U^dagger, in application order."""
        inv = Circuit(self.n_qubits, name=self.name + "_inv")
        for name, qs, m in reversed(self.ops):
            inv.add(name + "_dg", qs, m.conj().T)
        return inv

    def then(self, other: "Circuit") -> "Circuit":
        assert other.n_qubits == self.n_qubits
        return Circuit(self.n_qubits, self.ops + other.ops, name=self.name + "+" + other.name)

    def count(self, name: str) -> int:
        return sum(1 for o in self.ops if o[0] == name)

    def __len__(self):
        return len(self.ops)


def coupling_pattern(rows: int, cols: int, pattern: int):
    """Nearest-neighbour CZ pairs of one of the four alternating patterns."""
    pairs = []
    if pattern in (0, 1):
        for r in range(rows):
            for c in range(pattern, cols - 1, 2):
                pairs.append((r * cols + c, r * cols + c + 1))
    elif pattern in (2, 3):
        for r in range(pattern - 2, rows - 1, 2):
            for c in range(cols):
                pairs.append((r * cols + c, (r + 1) * cols + c))
    else:
        raise ValueError("pattern must be 0..3")
    return pairs


def random_grid_circuit(rows: int, cols: int, depth: int, seed: int) -> Circuit:
    """Random grid circuit: per layer, random sqrt(X|Y|W) on all qubits then a CZ pattern."""
    n = rows * cols
    rng = np.random.Generator(np.random.PCG64(seed))
    circ = Circuit(n, name=f"grid{rows}x{cols}_d{depth}_s{seed}")
    for layer in range(depth):
        choice = rng.integers(0, len(SINGLE_QUBIT_SET), size=n)
        for q in range(n):
            name, m = SINGLE_QUBIT_SET[int(choice[q])]
            circ.add(name, (q,), m)
        for a, b in coupling_pattern(rows, cols, layer % 4):
            circ.add("cz", (a, b), CZ)
    return circ


def ghz_circuit(n: int) -> Circuit:
    """H on qubit 0 then a CNOT chain 0->1->...->n-1: (|0..0> + |1..1>)/sqrt(2)."""
    circ = Circuit(n, name=f"ghz{n}")
    circ.add("h", (0,), H)
    for q in range(n - 1):
        circ.add("cnot", (q, q + 1), CNOT)
    return circ


def identity_circuit(n: int, kind: str = "empty") -> Circuit:
    """Circuits equal to the identity: no gates, sqrt(X)^4 on every qubit, or CZ twice."""
    circ = Circuit(n, name=f"identity_{kind}{n}")
    if kind == "empty":
        return circ
    if kind == "sqrtx4":
        for _ in range(4):
            for q in range(n):
                circ.add("sqrt_x", (q,), SQRT_X)
        return circ
    if kind == "cz2":
        for q in range(n):
            circ.add("sqrt_x", (q,), SQRT_X)
            circ.add("sqrt_x", (q,), SQRT_X)
            circ.add("sqrt_x", (q,), SQRT_X)
            circ.add("sqrt_x", (q,), SQRT_X)
        for q in range(n - 1):
            circ.add("cz", (q, q + 1), CZ)
            circ.add("cz", (q, q + 1), CZ)
        return circ
    raise ValueError(kind)


def mirror_circuit(rows: int, cols: int, depth: int, seed: int) -> Circuit:
    """A random grid circuit followed by its inverse: the identity up to rounding."""
    c = random_grid_circuit(rows, cols, depth, seed)
    m = c.then(c.inverse())
    m.name = f"mirror{rows}x{cols}_d{depth}_s{seed}"
    return m
