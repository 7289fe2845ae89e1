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


def empirical_supremum_sample(probs, n_qubits, candidates, uniforms, n_samples, warmup=0, return_bound=False):
    """Kept samples and per-candidate decisions (-1 warm-up, 0 rejected, 1 accepted); with ``return_bound``
    also the final bound M."""
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
    out = (np.array(kept, dtype=np.uint64), np.array(decisions, dtype=np.int8))
    return out + (M,) if return_bound else out


def empirical_supremum_sample_groups(probs, n_qubits, open_qubits, candidates, uniforms, choices, n_samples,
                                     warmup=0, return_bound=False):
    """Group rejection sampling with open outputs (an extension of Sec. III-B using the open-index
    contraction of Sec. II; not in the paper).  A candidate x names the group of the 2^m bitstrings that
    agree with x outside the m open qubits; groups are proposed uniformly (G = 2^(n - m) of them).  The
    group's probability P is the sum of its members' p; it is accepted with probability P G / M, M = 1 at
    first and max(M, P G) after every candidate, warm-up candidates only raising M.  An accepted group
    yields member j (bit i of j = value of the i-th open qubit, ascending) for the first j whose
    cumulative probability exceeds choice * P."""
    open_qubits = sorted(int(q) for q in open_qubits)
    m = len(open_qubits)
    G = 2.0 ** (n_qubits - m)
    mask = 0
    for q in open_qubits:
        mask |= 1 << q
    M = 1.0
    kept = []
    decisions = []
    for i, (x, u, c) in enumerate(zip(candidates, uniforms, choices)):
        if len(kept) >= n_samples:
            break
        members = []
        for j in range(1 << m):
            y = int(x) & ~mask
            for b, q in enumerate(open_qubits):
                if (j >> b) & 1:
                    y |= 1 << q
            members.append(y)
        pj = [float(probs[y]) for y in members]
        P = sum(pj)
        r = P * G
        if i < warmup:
            decisions.append(-1)
        else:
            accept = u < r / M
            decisions.append(1 if accept else 0)
            if accept:
                cum, pick = 0.0, members[-1]
                for y, p in zip(members, pj):
                    cum += p
                    if c * P < cum:
                        pick = y
                        break
                kept.append(pick)
        M = max(M, r)
    out = (np.array(kept, dtype=np.uint64), np.array(decisions, dtype=np.int8))
    return out + (M,) if return_bound else out
