"""O2: literal index sum (oracle; test infrastructure only).

A tensor network's value is the product of its tensors summed over every
assignment of the indices they share (Eq. 1).  Closing each output wire with the
bitstring's qubit value (Sec. II) leaves a scalar: the amplitude.  This module
evaluates that sum term by term, vectorised over blocks of assignments, with no
contraction order at all.  Only usable for networks with about 24 or fewer
internal indices.
"""
from __future__ import annotations

import numpy as np


def amplitude_bruteforce(net, bitstring, fixed=None, block=1 << 16) -> complex:
    """Sum over all internal-index assignments of prod_v T_v (output wires fixed).

    ``fixed`` optionally maps further labels to a fixed value (a slice, Eq. 2).
    """
    x = int(bitstring)
    fix = {lab: (x >> q) & 1 for q, lab in enumerate(net.output_labels)}
    if fixed:
        fix.update({int(k): int(v) for k, v in fixed.items()})
    free = sorted({lab for ix in net.indices for lab in ix if lab not in fix})
    pos = {lab: i for i, lab in enumerate(free)}
    n_free = len(free)
    if n_free > 26:
        raise ValueError("too many internal indices for brute force")
    flat = [t.reshape(-1) for t in net.tensors]
    total = 0.0 + 0.0j
    n_assign = 1 << n_free
    for start in range(0, n_assign, block):
        a = np.arange(start, min(n_assign, start + block), dtype=np.int64)
        term = np.ones(a.shape[0], dtype=np.complex128)
        for t, ix in zip(flat, net.indices):
            r = len(ix)
            off = np.zeros(a.shape[0], dtype=np.int64)
            for j, lab in enumerate(ix):
                if lab in fix:
                    v = np.int64(fix[lab])
                else:
                    v = (a >> pos[lab]) & 1
                off += v << (r - 1 - j)
            term = term * t[off]
        total += term.sum()
    return complex(total)
