"""Empirical-supremum rejection sampling of output bitstrings (Sec. III-B).

Candidates x are uniform over the N = 2^n bitstrings.  A candidate is accepted
with probability p(x) N / M, p(x) = |a(x)|^2 its output probability; after every
candidate the bound becomes M = max(M, p(x) N), starting from M = 1.  The first
``warmup`` candidates only update M and are discarded.

The random numbers are inputs: ``candidates`` (uint64 bitstrings, bit q = qubit q)
and ``uniforms`` (one in [0, 1) per candidate).  Amplitudes are computed a batch
of candidates at a time by ``amplitude_fn`` (the GPU path); accept / reject runs
in candidate order, so the result is the sequential algorithm's.
"""
from __future__ import annotations

import numpy as np


def rejection_sample(amplitude_fn, n_qubits: int, candidates, uniforms, n_samples: int, warmup: int = 0,
                     batch: int = 256):
    """Returns (samples, info).  Stops when ``n_samples`` are accepted or the candidates run out."""
    candidates = np.asarray(candidates, dtype=np.uint64)
    uniforms = np.asarray(uniforms, dtype=np.float64)
    if len(candidates) != len(uniforms):
        raise ValueError("one uniform per candidate")
    N = float(2.0 ** n_qubits)
    M = 1.0
    samples = []
    used = 0
    decisions = []
    while len(samples) < n_samples and used < len(candidates):
        cand = candidates[used:used + batch]
        amps = np.asarray(amplitude_fn(cand))
        for x, a, u in zip(cand, amps, uniforms[used:used + len(cand)]):
            if len(samples) >= n_samples:
                break
            ratio = float(abs(a) ** 2) * N
            if used < warmup:
                decisions.append(-1)
            else:
                ok = u * M < ratio
                decisions.append(int(ok))
                if ok:
                    samples.append(int(x))
            M = max(M, ratio)
            used += 1
    return np.array(samples, dtype=np.uint64), {"candidates_used": used, "M": M,
                                                 "decisions": np.array(decisions, dtype=np.int8)}
