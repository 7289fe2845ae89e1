"""Rejection sampling with the empirical-supremum bound, from exact probabilities
(oracle; test infrastructure only).

Sec. III-B: propose candidates uniformly; accept candidate X with probability
p(X) N / M where N is the number of possible bitstrings; start with M = 1 and
after each candidate set M to the larger of M and p(X) N; candidates of an
initial warm-up period are not kept.  Here p comes from the state vector (O1).
"""
from __future__ import annotations

import numpy as np

from .statevector import statevector


def probabilities(circuit):
    psi = statevector(circuit)
    n = circuit.n_qubits
    # flat index of psi has qubit 0 most significant; bitstring x has qubit q at bit q
    return np.abs(np.transpose(psi, list(range(n - 1, -1, -1))).reshape(-1)) ** 2


def empirical_supremum_sample(probs, n_qubits, candidates, uniforms, n_samples, warmup=0):
    N = 2.0 ** n_qubits
    M = 1.0
    kept = []
    decisions = []
    for i, (x, u) in enumerate(zip(candidates, uniforms)):
        if len(kept) >= n_samples:
            break
        r = probs[int(x)] * N
        if i < warmup:
            decisions.append(-1)
        else:
            accept = u < r / M
            decisions.append(1 if accept else 0)
            if accept:
                kept.append(int(x))
        M = max(M, r)
    return np.array(kept, dtype=np.uint64), np.array(decisions, dtype=np.int8)
