"""Random inputs of the rejection sampler: uniform candidate bitstrings and one
uniform variate per candidate, from numpy.random.Generator(PCG64(seed))."""
from __future__ import annotations

import numpy as np

from .bitstrings import random_bitstrings


def sampling_inputs(n_qubits: int, count: int, seed: int):
    cand = random_bitstrings(n_qubits, count, seed)
    u = np.random.Generator(np.random.PCG64(seed + 7919)).random(count)
    return cand, u


def group_sampling_inputs(n_qubits: int, count: int, seed: int):
    """Inputs of the open-output (group) sampler: candidates, an acceptance uniform per candidate and a
    second uniform per candidate that picks the member of an accepted group."""
    cand, u = sampling_inputs(n_qubits, count, seed)
    c = np.random.Generator(np.random.PCG64(seed + 104729)).random(count)
    return cand, u, c
