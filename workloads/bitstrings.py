"""Seeded output bitstrings (input generator).

Bit q of the packed uint64 is the measured value of qubit q.  Bitstrings are
drawn uniformly and independently (duplicates allowed) from
numpy.random.Generator(PCG64(seed)).
"""
from __future__ import annotations

import numpy as np


def random_bitstrings(n_qubits: int, count: int, seed: int) -> np.ndarray:
    if not 0 < n_qubits <= 64:
        raise ValueError("n_qubits must be in 1..64")
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.integers(0, 2, size=(count, n_qubits), dtype=np.uint64)
    weights = np.left_shift(np.uint64(1), np.arange(n_qubits, dtype=np.uint64))
    return (bits * weights).sum(axis=1, dtype=np.uint64).astype(np.uint64)


def all_bitstrings(n_qubits: int) -> np.ndarray:
    return np.arange(2 ** n_qubits, dtype=np.uint64)


def bit(x, q: int) -> int:
    return (int(x) >> q) & 1
