"""O1: state-vector simulation in complex128 (oracle; test infrastructure only).

The n-qubit state is kept as an array of shape (2,)*n whose axis q is qubit q,
so qubit 0 is the most significant bit of the flattened (Kronecker-order)
index.  Gates are applied in circuit order to |0...0>, as in the full-state
simulators described in Sec. II; the amplitude of bitstring x (bit q of x is
the value of qubit q) is psi[x_0, x_1, ..., x_{n-1}].
"""
from __future__ import annotations

import numpy as np


def statevector(circuit) -> np.ndarray:
    """Final state of ``circuit`` (shape (2,)*n, complex128)."""
    n = circuit.n_qubits
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for _name, qubits, matrix in circuit.ops:
        k = len(qubits)
        u = np.asarray(matrix, dtype=np.complex128).reshape((2,) * (2 * k))
        # contract the gate's input axes with the target qubits' axes
        psi = np.tensordot(u, psi, axes=(list(range(k, 2 * k)), list(qubits)))
        # the gate's output axes now lead; move them back to the qubits' slots
        psi = np.moveaxis(psi, list(range(k)), list(qubits))
    return psi


def amplitudes_statevector(circuit, bitstrings) -> np.ndarray:
    """<x|U|0...0> for every packed bitstring x (bit q = qubit q)."""
    psi = statevector(circuit)
    n = circuit.n_qubits
    out = np.empty(len(bitstrings), dtype=np.complex128)
    for i, x in enumerate(bitstrings):
        x = int(x)
        out[i] = psi[tuple((x >> q) & 1 for q in range(n))]
    return out
