"""The benchmark workloads, as seeded synthetic inputs.

Each config fixes a circuit (grid, depth, seed), the number of sliced indices,
the bitstring batch and the planner's seed and trial count.  The contraction
tree and the sliced indices are plan INPUTS: any tree gives the same amplitudes
up to rounding, only the work changes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .bitstrings import random_bitstrings
from .circuits import random_grid_circuit
from .network import circuit_to_network
from .planner import plan_network


@dataclass
class Workload:
    name: str
    rows: int
    cols: int
    depth: int
    circuit_seed: int
    n_sliced: int
    n_bitstrings: int
    bitstring_seed: int
    planner_seed: int
    planner_trials: int
    width_cap: int | None = None
    description: str = ""
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def n_qubits(self):
        return self.rows * self.cols

    def circuit(self):
        if "circ" not in self._cache:
            self._cache["circ"] = random_grid_circuit(self.rows, self.cols, self.depth, self.circuit_seed)
        return self._cache["circ"]

    def network(self):
        if "net" not in self._cache:
            self._cache["net"] = circuit_to_network(self.circuit())
        return self._cache["net"]

    def plan_inputs(self):
        """(tree, sliced_labels, stats) from the seeded planner."""
        if "plan" not in self._cache:
            self._cache["plan"] = plan_network(self.network(), self.n_sliced, trials=self.planner_trials,
                                               seed=self.planner_seed, width_cap=self.width_cap)
        return self._cache["plan"]

    def bitstrings(self, count=None):
        return random_bitstrings(self.n_qubits, count or self.n_bitstrings, self.bitstring_seed)


CONFIGS = {
    "c1": Workload("c1", 3, 4, 8, 1, 0, 64, 1001, 101, 8,
                   description="12-qubit 3x4 grid, depth 8, no slicing, 64 bitstrings"),
    "c2": Workload("c2", 5, 6, 12, 2, 10, 256, 1002, 100, 40,
                   description="30-qubit 5x6 grid, depth 12, 10 sliced indices (1024 slices), 256 bitstrings"),
    "c4": Workload("c4", 7, 7, 14, 4, 24, 1, 1004, 104, 16, width_cap=30,
                   description="49-qubit 7x7 grid, depth 14, 24 sliced indices, 1 bitstring"),
}


def get(name: str) -> Workload:
    return CONFIGS[name]
