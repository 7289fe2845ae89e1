"""Circuit -> tensor network construction (input generator, Sec. II / Fig. 3).

Each qubit starts as a rank-1 tensor |0> = (1, 0) carrying one open index.  A
one-qubit gate becomes a rank-2 tensor T[out, in]; a two-qubit gate's 4x4
matrix is reshaped to a rank-4 tensor T[a_out, b_out, a_in, b_in].  Gates are
attached to the open indices of the qubits they act on, in circuit order, and
the open index left on qubit q at the end is its output wire.  Index labels are
non-negative integers, every label has dimension 2, and every label appears in
exactly two tensors except output wires, which appear in one.

Tensors are stored row-major in the order of their label tuple (first label
slowest), which is the element order the C-ABI boundary expects.
"""
from __future__ import annotations

import numpy as np

from .circuits import Circuit


class Network:
    def __init__(self, tensors, indices, output_labels, n_qubits, name="network"):
        self.tensors = [np.ascontiguousarray(t, dtype=np.complex128) for t in tensors]
        self.indices = [tuple(int(x) for x in ix) for ix in indices]
        self.output_labels = [int(x) for x in output_labels]
        self.n_qubits = int(n_qubits)
        self.name = name
        for t, ix in zip(self.tensors, self.indices):
            assert t.shape == (2,) * len(ix), (t.shape, ix)

    @property
    def n_tensors(self) -> int:
        return len(self.tensors)

    def labels(self):
        out = set()
        for ix in self.indices:
            out.update(ix)
        return out

    def label_count(self):
        cnt = {}
        for ix in self.indices:
            for x in ix:
                cnt[x] = cnt.get(x, 0) + 1
        return cnt

    def to_csr(self):
        """Flat arrays for the C-ABI: (index_ptr, index_ids, data_ptr, data, output_index)."""
        index_ptr = np.zeros(self.n_tensors + 1, dtype=np.int64)
        data_ptr = np.zeros(self.n_tensors + 1, dtype=np.int64)
        for i, (t, ix) in enumerate(zip(self.tensors, self.indices)):
            index_ptr[i + 1] = index_ptr[i] + len(ix)
            data_ptr[i + 1] = data_ptr[i] + t.size
        index_ids = np.array([x for ix in self.indices for x in ix], dtype=np.int64)
        data = np.concatenate([t.reshape(-1) for t in self.tensors]) if self.tensors else \
            np.zeros(0, np.complex128)
        data = np.ascontiguousarray(data.astype(np.complex128)).view(np.float64)
        output_index = np.array(self.output_labels, dtype=np.int64)
        return index_ptr, index_ids, data_ptr, data, output_index


def circuit_to_network(circ: Circuit) -> Network:
    n = circ.n_qubits
    tensors, indices = [], []
    next_label = 0
    cur = []
    for q in range(n):
        tensors.append(np.array([1.0, 0.0], dtype=np.complex128))
        indices.append((next_label,))
        cur.append(next_label)
        next_label += 1
    for name, qs, m in circ.ops:
        k = len(qs)
        new = list(range(next_label, next_label + k))
        next_label += k
        tensors.append(m.reshape((2,) * (2 * k)))
        indices.append(tuple(new) + tuple(cur[q] for q in qs))
        for q, lab in zip(qs, new):
            cur[q] = lab
    return Network(tensors, indices, cur, n, name=circ.name)


def dense_chain_network(group_bits: int = 5, slow_first=(True, True, True, True), seed: int = 0) -> Network:
    """Four dense random leaves in a chain, A(q_lo, k) B(k, j) C(j, l) D(l, q_hi).

    Each group holds ``group_bits`` labels; q_lo / q_hi are the output wires of
    qubits 0..g-1 / g..2g-1.  ``slow_first[t]`` lists leaf t's first group
    slowest (else its second group slowest), which decides whether the labels a
    contraction sums over are the leaf's fastest-varying ones.  Entries are
    complex normal, scaled so amplitudes are of order 2^-g.
    """
    g = int(group_bits)
    groups = [list(range(i * g, (i + 1) * g)) for i in range(5)]
    rng = np.random.default_rng(seed)
    tensors, indices = [], []
    for t in range(4):
        first, second = groups[t], groups[t + 1]
        ix = first + second if slow_first[t] else second + first
        shape = (2,) * len(ix)
        data = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0 * (1 << g))
        tensors.append(data)
        indices.append(tuple(ix))
    return Network(tensors, indices, groups[0] + groups[4], 2 * g, name=f"chain{g}")


def outer_thin_network(long_bits: int, short_bits: int, sum_bits: int, seed: int = 0,
                       short_first: bool = False) -> Network:
    """Three dense random leaves: a long operand L(l, k), a short one S(s, k) and a closing leaf
    C(l, s, q) whose one open wire q is qubit 0.  Contracted along ((L, S), C), the first product has
    2^(long_bits + short_bits) entries summed over 2^sum_bits terms.  L lists its k labels between
    its l labels, so neither its fastest nor its slowest labels are all summed.  ``short_first``
    puts S first in the leaf list.  Entries are complex normal, scaled so the amplitudes are of order 1.
    """
    rng = np.random.default_rng(seed)
    lo = list(range(long_bits))
    sh = list(range(long_bits, long_bits + short_bits))
    ks = list(range(long_bits + short_bits, long_bits + short_bits + sum_bits))
    q = long_bits + short_bits + sum_bits
    half = long_bits // 2
    ix_l = tuple(lo[:half] + ks + lo[half:])
    ix_s = tuple(ks + sh)
    ix_c = tuple(sh + lo + [q])

    def rnd(n, scale):
        shape = (2,) * n
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale

    t_l = rnd(len(ix_l), 2.0 ** (-0.25 * sum_bits) / np.sqrt(2.0))
    t_s = rnd(len(ix_s), 2.0 ** (-0.25 * sum_bits) / np.sqrt(2.0))
    t_c = rnd(len(ix_c), 2.0 ** (-0.5 * (long_bits + short_bits)) / np.sqrt(2.0))
    tensors, indices = [t_l, t_s, t_c], [ix_l, ix_s, ix_c]
    if short_first:
        tensors[0], tensors[1] = tensors[1], tensors[0]
        indices[0], indices[1] = indices[1], indices[0]
    return Network(tensors, indices, [q], 1, name=f"outer{long_bits}x{short_bits}k{sum_bits}")


def dot_pair_network(a_bits: int, b_bits: int, sum_bits: int, seed: int = 0) -> Network:
    """Two dense random leaves A(qa, k) and B(qb, k) whose one contraction is a long inner product:
    qa are the output wires of qubits 0..a_bits-1, qb those of the next b_bits qubits, k the
    sum_bits summed labels (listed last, so fastest-varying).  Entries are complex normal, scaled
    so the amplitudes are of order 1."""
    rng = np.random.default_rng(seed)
    qa = list(range(a_bits))
    qb = list(range(a_bits, a_bits + b_bits))
    ks = list(range(a_bits + b_bits, a_bits + b_bits + sum_bits))
    scale = 2.0 ** (-0.25 * sum_bits) / np.sqrt(2.0)
    tensors, indices = [], []
    for q in (qa, qb):
        ix = tuple(q + ks)
        shape = (2,) * len(ix)
        tensors.append((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale)
        indices.append(ix)
    return Network(tensors, indices, qa + qb, a_bits + b_bits, name=f"dot{a_bits}x{b_bits}k{sum_bits}")
