"""FP64 CPU oracle for sliced tensor-network amplitude contraction.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or call anything in this package; the
product path never does, and this package imports nothing from the product
package.  It shares no code with the GPU path: only the seeded input
generators (``workloads``) feed both.

Three independent computations of one definition, all in complex128:

* ``statevector``  (O1) -- apply the circuit's gates in order to |0...0> and
  read psi[x] (Sec. II: the full-state picture the paper contrasts with).
* ``bruteforce``   (O2) -- the literal sum over every assignment of the
  network's internal indices of the product of all tensors, output wires fixed
  by the bitstring (Eq. 1 with the output closure of Sec. II).
* ``tree_contract`` (O3) -- pairwise contraction along a given tree
  (Sec. III-A) of each slice's network, slices summed (Eq. 2).
* ``sampling`` -- empirical-supremum rejection sampling (Sec. III-B) from the
  exact O1 probabilities, per bitstring and per group of bitstrings that share
  all but some open output qubits.

Every function here is pinned by tests against closed forms, invariants and the
other two computations; none is "parity unpinned".
"""
from .statevector import statevector, amplitudes_statevector
from .bruteforce import amplitude_bruteforce
from .tree_contract import contract_slice, amplitude_sliced, amplitudes_sliced
from .sampling import probabilities, empirical_supremum_sample, empirical_supremum_sample_groups

__all__ = ["statevector", "amplitudes_statevector", "amplitude_bruteforce", "contract_slice",
           "amplitude_sliced", "amplitudes_sliced", "probabilities",
           "empirical_supremum_sample", "empirical_supremum_sample_groups"]
