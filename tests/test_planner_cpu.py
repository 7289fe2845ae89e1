"""Planner checks (CPU only): local sub-tree re-ordering keeps the tree valid,
never costs more, reaches the exhaustive optimum when its window covers the
whole tree, and leaves the amplitudes unchanged (Sec. III-A: any contraction
order gives the same result).
"""
import itertools

import numpy as np
import pytest

import oracle
from workloads import (circuit_to_network, random_grid_circuit, greedy_tree, tree_trimming, tree_stats,
                       local_reconfigure, plan_network, random_bitstrings, node_label_sets)


def _check_ssa(tree, n):
    tree = np.asarray(tree)
    assert tree.shape == (n - 1, 2)
    used = set()
    for t, (a, b) in enumerate(tree):
        assert a != b and a < n + t and b < n + t
        assert a not in used and b not in used
        used.update((int(a), int(b)))
    assert used == set(range(2 * n - 2))


@pytest.mark.parametrize("rows,cols,depth,seed,n_sliced", [(2, 3, 4, 7, 0), (3, 3, 6, 8, 2), (3, 4, 8, 9, 3)])
def test_reconfigure_valid_and_not_costlier(rows, cols, depth, seed, n_sliced):
    net = circuit_to_network(random_grid_circuit(rows, cols, depth, seed))
    tree = greedy_tree(net, seed=seed, alpha=0.6, temperature=1.0)
    sliced = tree_trimming(net, tree, n_sliced, seed=seed) if n_sliced else []
    before = tree_stats(net, tree, sliced)
    new = local_reconfigure(net, tree, sliced, window=6)
    _check_ssa(new, net.n_tensors)
    after = tree_stats(net, new, sliced)
    assert after["flops_per_slice"] <= before["flops_per_slice"]
    assert after["width"] <= before["width"]
    # the root keeps every label that stays open (none once outputs and slices are closed)
    assert node_label_sets(net, new, sliced)[-1] == node_label_sets(net, tree, sliced)[-1]


def _exhaustive_min_flops(net, cap):
    """Cheapest pairwise merge sequence over all orders (tiny networks only), no set wider than cap."""
    sets = node_label_sets(net, np.zeros((0, 2), dtype=np.int32))
    best = [np.inf]

    def rec(active, cost):
        if cost >= best[0]:
            return
        if len(active) == 1:
            best[0] = cost
            return
        for i, j in itertools.combinations(range(len(active)), 2):
            a, b = active[i], active[j]
            out = a ^ b
            if len(out) > cap:
                continue
            rest = [s for k, s in enumerate(active) if k not in (i, j)]
            rec(rest + [out], cost + 8 * 2 ** len(a | b))

    rec(list(sets), 0)
    return best[0]


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_full_window_reaches_exhaustive_optimum(seed):
    # 1x2 depth-2 grids give 6-7 leaves: small enough to try every merge order
    net = circuit_to_network(random_grid_circuit(1, 2, 2, seed))
    n = net.n_tensors
    assert n <= 7
    tree = greedy_tree(net, seed=seed, alpha=0.0, temperature=3.0)
    cap = tree_stats(net, tree)["width"]
    new = local_reconfigure(net, tree, window=n)
    assert tree_stats(net, new)["flops_per_slice"] == _exhaustive_min_flops(net, cap)


def test_reconfigured_tree_gives_same_amplitudes():
    circ = random_grid_circuit(3, 3, 6, 5)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=3, alpha=0.5, temperature=1.5)
    sliced = tree_trimming(net, tree, 2, seed=3)
    new = local_reconfigure(net, tree, sliced, window=8)
    assert not np.array_equal(new, tree)
    xs = random_bitstrings(9, 8, 77)
    want = oracle.amplitudes_statevector(circ, xs)
    got = oracle.amplitudes_sliced(net, new, xs, sliced)
    assert np.max(np.abs(got - want)) < 1e-14


def test_plan_network_refinement_never_worse():
    net = circuit_to_network(random_grid_circuit(3, 4, 8, 1))
    t0, s0, st0 = plan_network(net, 2, trials=4, seed=3)
    t1, s1, st1 = plan_network(net, 2, trials=4, seed=3, reconfigure=2)
    assert st1["total_flops"] <= st0["total_flops"]
    _check_ssa(t1, net.n_tensors)


def test_roofline_cost_and_refinement():
    from workloads.planner import contraction_cost, tree_cost
    a, b = frozenset({1, 2, 3}), frozenset({3, 4})
    assert contraction_cost(a, b) == 2.0 ** 4
    # memory term: 2^3 + 2^2 + 2^|{1,2,4}| = 20 elements
    assert contraction_cost(a, b, mem_weight=10.0) == 200.0
    assert contraction_cost(a, b, mem_weight=0.5) == 16.0
    circ = random_grid_circuit(3, 4, 8, 9)
    net = circuit_to_network(circ)
    tree = greedy_tree(net, seed=9, alpha=0.6, temperature=1.0)
    sliced = tree_trimming(net, tree, 2, seed=9)
    for mw in (4.0, 32.0):
        new = local_reconfigure(net, tree, sliced, window=6, mem_weight=mw)
        _check_ssa(new, net.n_tensors)
        assert tree_cost(net, new, sliced, mw) <= tree_cost(net, tree, sliced, mw)
        assert tree_stats(net, new, sliced)["width"] <= tree_stats(net, tree, sliced)["width"]
    xs = random_bitstrings(12, 6, 5)
    got = oracle.amplitudes_sliced(net, new, xs, sliced)
    assert np.max(np.abs(got - oracle.amplitudes_statevector(circ, xs))) < 1e-14


def test_refined_c2_tree_compiles_and_is_cheaper():
    # the 30-qubit configuration's refined tree (bench.py --reconfigure 4) compiles into a plan and does far
    # less work per slice than the greedy tree the configuration uses
    from paper_2110_09894_amd import qxtn
    from workloads import configs
    w = configs.get("c2")
    tree0, sl0, st0 = w.plan_inputs()
    tree, sl, st = w.plan_inputs(reconfigure=4, mem_weight=16.0)
    assert st["width"] <= st0["width"] and st["total_flops"] < st0["total_flops"] / 4
    p0 = qxtn.Plan(w.network(), tree0, sl0, max_bitstrings=256, slice_batch_log2=4, dry_run=True).info()
    p1 = qxtn.Plan(w.network(), tree, sl, max_bitstrings=256, slice_batch_log2=4, dry_run=True).info()
    assert p1["flops_per_slice"] < p0["flops_per_slice"] / 4
    assert p1["width"] == st["width"]
