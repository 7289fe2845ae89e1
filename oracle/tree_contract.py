"""O3: pairwise tree contraction of sliced networks in complex128 (oracle; test infrastructure only).

* A slice fixes every sliced index to one value (Eq. 2): slice s sets the j-th
  sliced label to bit j of s.  The network's value is the sum over all slices.
* The bitstring closes the output wire of qubit q with value bit q of x
  (Sec. II).
* Each slice's network is then contracted as a sequence of pairwise
  contractions along the given tree (Sec. III-A): a pair of tensors is replaced
  by their product summed over the indices they share.

The tree is data (an SSA list of pairs), so any order can be checked against
any other.  Slice values are summed with math.fsum, real and imaginary parts
separately.
"""
from __future__ import annotations

import math

import numpy as np


def _fix_leaves(net, fixed):
    leaves = []
    for t, ix in zip(net.tensors, net.indices):
        sel = tuple(fixed[lab] if lab in fixed else slice(None) for lab in ix)
        leaves.append((np.asarray(t[sel], dtype=np.complex128),
                       tuple(lab for lab in ix if lab not in fixed)))
    return leaves


def contract_slice(net, tree, bitstring, sliced=(), slice_id=0) -> complex:
    """Value of one slice's closed network, contracted pairwise along ``tree``."""
    x = int(bitstring)
    fixed = {lab: (x >> q) & 1 for q, lab in enumerate(net.output_labels)}
    for j, lab in enumerate(sliced):
        if lab in fixed:
            raise ValueError("an output wire cannot be sliced")
        fixed[int(lab)] = (int(slice_id) >> j) & 1
    nodes = _fix_leaves(net, fixed)
    tree = np.asarray(tree, dtype=np.int64).reshape(-1, 2)
    if len(tree) != len(nodes) - 1:
        raise ValueError("tree must have n_tensors - 1 steps")
    for a, b in tree:
        ta, la = nodes[a]
        tb, lb = nodes[b]
        if ta is None or tb is None:
            raise ValueError("tree consumes a tensor twice")
        shared = [lab for lab in la if lab in lb]
        tc = np.tensordot(ta, tb, axes=([la.index(s) for s in shared], [lb.index(s) for s in shared]))
        lc = tuple(lab for lab in la if lab not in shared) + tuple(lab for lab in lb if lab not in shared)
        nodes[a] = (None, None)
        nodes[b] = (None, None)
        nodes.append((tc, lc))
    root, labels = nodes[-1]
    if labels:
        raise ValueError("root still carries open indices: %r" % (labels,))
    return complex(root)


def amplitude_sliced(net, tree, bitstring, sliced=(), slice_range=None) -> complex:
    """sum over slices in ``slice_range`` (default: all 2^k) of each slice's value."""
    k = len(sliced)
    lo, hi = slice_range if slice_range is not None else (0, 1 << k)
    vals = [contract_slice(net, tree, bitstring, sliced, s) for s in range(lo, hi)]
    return complex(math.fsum(v.real for v in vals), math.fsum(v.imag for v in vals))


def amplitudes_sliced(net, tree, bitstrings, sliced=(), slice_range=None) -> np.ndarray:
    return np.array([amplitude_sliced(net, tree, x, sliced, slice_range) for x in bitstrings],
                    dtype=np.complex128)
