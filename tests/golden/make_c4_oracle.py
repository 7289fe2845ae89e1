#!/usr/bin/env python3
"""Writes tests/golden/c4_slices_<tree>.json: FP64 oracle values of single slices of the 49-qubit
7x7 depth-14 workload (24 sliced indices, one bitstring), for the GPU parity tests of that workload.

Calls only the oracle (O3, pairwise tree contraction in complex128: Eq. 2 and the output closure of
Sec. II) on inputs from the seeded generators in ``workloads``.  A slice's value does not depend on
the contraction order (Sec. III-A), so the oracle contracts each slice along a cheaper order of the
same sliced network (local sub-tree re-ordering of the plan's tree with the sliced labels closed);
the GPU contracts along the plan's own tree.

Slices: the whole first block of 64 (0..63, the block the GPU computes in one pass) and six seeded
slices from [64, 4096).  Trees: ``greedy`` (the workload's configured tree) and ``refined`` (the
workload's tree refined by local re-ordering, which also re-selects the sliced indices).

Usage: python tests/golden/make_c4_oracle.py greedy|refined   (minutes per tree on a few cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import configs, local_reconfigure, tree_stats  # noqa: E402

SEED = 4004


def slice_ids():
    rng = np.random.Generator(np.random.PCG64(SEED))
    extra = sorted(int(s) for s in rng.choice(np.arange(64, 4096), size=6, replace=False))
    return list(range(64)) + extra


def main(kind):
    w = configs.get("c4")
    net = w.network()
    if kind == "greedy":
        tree, sliced, st = w.plan_inputs()
    elif kind == "refined":
        tree, sliced, st = w.plan_inputs(reconfigure=4, mem_weight=16.0)
    else:
        raise SystemExit("tree kind must be greedy or refined")
    x = int(w.bitstrings()[0])
    otree = tree
    for _ in range(3):
        otree = local_reconfigure(net, otree, sliced, sweeps=3, window=10)
    ost = tree_stats(net, otree, sliced)
    out = {"workload": "c4", "tree": kind, "sliced": [int(s) for s in sliced], "bitstring": str(x),
           "plan_tree_width": int(st["width"]), "plan_tree_flops_per_slice": float(st["flops_per_slice"]),
           "oracle_tree_flops_per_slice": float(ost["flops_per_slice"]), "values": {}}
    if kind == "refined":
        out["tree_ssa"] = np.asarray(tree).reshape(-1).astype(int).tolist()
    path = os.path.join(HERE, f"c4_slices_{kind}.json")
    t0 = time.time()
    for i, s in enumerate(slice_ids()):
        v = oracle.contract_slice(net, otree, x, sliced, s)
        out["values"][str(s)] = [v.real, v.imag]
        print(f"{kind} slice {s}: {v!r} ({i + 1}/{len(slice_ids())}, {time.time() - t0:.0f} s)", flush=True)
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=0)
    os.replace(path + ".tmp", path)
    print(path)


if __name__ == "__main__":
    main(sys.argv[1])
