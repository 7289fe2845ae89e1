"""Seeded synthetic inputs shared by the oracle and the GPU path.

Circuits, their tensor networks, contraction trees, sliced-index choices and
output bitstrings.  Nothing here contracts tensors: it only builds the inputs
that ``plan``/``contract`` and the oracle consume.
"""
from .circuits import (Circuit, random_grid_circuit, ghz_circuit, identity_circuit,
                       mirror_circuit, coupling_pattern)
from .network import Network, circuit_to_network, dense_chain_network, outer_thin_network, dot_pair_network
from .planner import greedy_tree, tree_trimming, plan_network, tree_stats, node_label_sets, local_reconfigure
from .bitstrings import random_bitstrings, all_bitstrings
from .sampling_inputs import sampling_inputs, group_sampling_inputs

__all__ = ["dense_chain_network", "outer_thin_network", "dot_pair_network", "Circuit", "random_grid_circuit", "ghz_circuit", "identity_circuit", "mirror_circuit",
           "coupling_pattern", "Network", "circuit_to_network", "greedy_tree", "tree_trimming",
           "plan_network", "tree_stats", "node_label_sets", "local_reconfigure", "random_bitstrings", "all_bitstrings",
           "sampling_inputs", "group_sampling_inputs"]
