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


def rejection_sample_groups(amplitude_fn, n_qubits: int, open_qubits, candidates, uniforms, choices,
                            n_samples: int, warmup: int = 0, batch: int = 256):
    """Group rejection sampling over m open output qubits: one contraction gives the 2^m amplitudes of a
    candidate's group (the bitstrings that agree with it outside the open qubits), proposed uniformly among
    the 2^(n - m) groups.  A group of probability P is accepted when u M < P 2^(n - m), after which M
    becomes max(M, P 2^(n - m)) (starting at 1; warm-up candidates only raise M), and yields the member
    where the running sum of probabilities first exceeds choice * P, members ordered by j (bit i of j =
    value of the i-th smallest open qubit).  ``amplitude_fn(cand)`` returns a [len(cand), 2^m] array.
    Returns (samples, info)."""
    candidates = np.asarray(candidates, dtype=np.uint64)
    uniforms = np.asarray(uniforms, dtype=np.float64)
    choices = np.asarray(choices, dtype=np.float64)
    if not (len(candidates) == len(uniforms) == len(choices)):
        raise ValueError("one uniform and one choice per candidate")
    qs = sorted(int(q) for q in open_qubits)
    m = len(qs)
    mask = 0
    for q in qs:
        mask |= 1 << q
    scale = float(2.0 ** (n_qubits - m))
    M = 1.0
    samples = []
    used = 0
    decisions = []
    while len(samples) < n_samples and used < len(candidates):
        cand = candidates[used:used + batch]
        probs = np.abs(np.asarray(amplitude_fn(cand)).reshape(len(cand), 1 << m)) ** 2
        for x, pj, u, c in zip(cand, probs, uniforms[used:used + len(cand)], choices[used:used + len(cand)]):
            if len(samples) >= n_samples:
                break
            P = float(np.sum(pj))
            ratio = P * scale
            if used < warmup:
                decisions.append(-1)
            else:
                ok = u * M < ratio
                decisions.append(int(ok))
                if ok:
                    cum = np.cumsum(pj)
                    hit = np.nonzero(c * P < cum)[0]
                    j = int(hit[0]) if len(hit) else (1 << m) - 1
                    y = int(x) & ~mask
                    for b, q in enumerate(qs):
                        y |= ((j >> b) & 1) << q
                    samples.append(y)
            M = max(M, ratio)
            used += 1
    return np.array(samples, dtype=np.uint64), {"candidates_used": used, "M": M,
                                                 "decisions": np.array(decisions, dtype=np.int8)}
