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

    def plan_inputs(self, reconfigure=0, mem_weight=0.0):
        """(tree, sliced_labels, stats) from the seeded planner; ``reconfigure`` = r > 0 refines the
        best r greedy trials by local sub-tree re-ordering under a flop (``mem_weight`` 0) or
        roofline cost (the configs themselves use the greedy tree)."""
        key = ("plan", reconfigure, mem_weight)
        if key not in self._cache:
            self._cache[key] = plan_network(self.network(), self.n_sliced, trials=self.planner_trials,
                                            seed=self.planner_seed, width_cap=self.width_cap,
                                            reconfigure=reconfigure, mem_weight=mem_weight)
        return self._cache[key]

    def bitstrings(self, count=None):
        return random_bitstrings(self.n_qubits, count or self.n_bitstrings, self.bitstring_seed)


CONFIGS = {
    "c1": Workload("c1", 3, 4, 8, 1, 0, 64, 1001, 101, 8,
                   description="12-qubit 3x4 grid, depth 8, no slicing, 64 bitstrings"),
    "c2": Workload("c2", 5, 6, 12, 2, 10, 256, 1002, 100, 40,
                   description="30-qubit 5x6 grid, depth 12, 10 sliced indices (1024 slices), 256 bitstrings"),
    "c4": Workload("c4", 7, 7, 14, 4, 24, 1, 1004, 104, 64, width_cap=30,
                   description="49-qubit 7x7 grid, depth 14, 24 sliced indices, 1 bitstring"),
}


def get(name: str) -> Workload:
    return CONFIGS[name]


@dataclass
class ServingMix:
    """Poisson stream of amplitude requests over a pool of resident circuits."""
    name: str
    pool: list            # (rows, cols, depth, circuit_seed, n_sliced)
    max_bitstrings: int
    request_max_bitstrings: int
    seed: int
    planner_trials: int = 8
    description: str = ""

    def circuits(self, reconfigure=2, mem_weight=16.0):
        """(name, circuit, network, tree, sliced labels, stats) per pool circuit; with ``reconfigure`` = r > 0
        the best r greedy trials are refined by local sub-tree re-ordering (as a server would plan the
        circuits it keeps resident), else the plain seeded greedy tree."""
        out = []
        for rows, cols, depth, cseed, k in self.pool:
            circ = random_grid_circuit(rows, cols, depth, cseed)
            net = circuit_to_network(circ)
            tree, sliced, st = plan_network(net, k, trials=self.planner_trials, seed=cseed + 7,
                                            reconfigure=reconfigure, mem_weight=mem_weight)
            out.append((f"{rows}x{cols}_d{depth}", circ, net, tree, sliced, st))
        return out

    def requests(self, count: int):
        """(arrival offset in units of 1/rate, circuit index, bitstrings) for ``count`` requests."""
        rng = np.random.Generator(np.random.PCG64(self.seed))
        gaps = rng.exponential(1.0, size=count)
        which = rng.integers(0, len(self.pool), size=count)
        sizes = rng.integers(1, self.request_max_bitstrings + 1, size=count)
        out, t = [], 0.0
        for i in range(count):
            t += gaps[i]
            rows, cols = self.pool[which[i]][0], self.pool[which[i]][1]
            xs = random_bitstrings(rows * cols, int(sizes[i]), self.seed * 1000 + i)
            out.append((t, int(which[i]), xs))
        return out


SERVING = ServingMix(
    "c5", pool=[(4, 5, 8, 51, 0), (4, 5, 14, 52, 0), (5, 6, 8, 53, 0), (5, 6, 10, 54, 2), (7, 7, 8, 55, 4)],
    max_bitstrings=256, request_max_bitstrings=1024, seed=5,
    description="Poisson amplitude requests of 1-1024 bitstrings over 20-, 30- and 49-qubit grids "
                "(4x5 d8, 4x5 d14, 5x6 d8, 5x6 d10, 7x7 d8), plans resident, admitted by HBM budget")
