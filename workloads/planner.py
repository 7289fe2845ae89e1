"""Contraction-order and slice selection (input generator; integer size bookkeeping only).

* ``greedy_tree`` -- a seeded greedy pairwise order.  The paper contracts a
  network as a sequence of pairwise contractions (Sec. III-A) and notes that
  many heuristics find good orders in bounded time; this is the "greedy
  min-size" family: repeatedly contract the adjacent pair whose result grows the
  stored size least, size(out) - alpha * (size(a) + size(b)), with seeded Gumbel
  noise for trial diversity.  Several noisy trials are run and the best kept.
* ``tree_trimming`` -- greedy slice selection as described in Sec. III-A:
  always slice an index of a largest intermediate; among those, prefer the
  index contained in the most largest intermediates, then the one whose slicing
  saves the most total intermediate memory, then a seeded random choice.

A tree is an int32 array of shape [n_tensors - 1, 2] in SSA form: step t
contracts ids (a, b) and creates id n_tensors + t.  Output-wire labels are
closed by the bitstring, so they never count towards sizes.
"""
from __future__ import annotations

import heapq
import math

import numpy as np


def _base_sets(net, exclude=()):
    ex = set(net.output_labels) | set(exclude)
    return [frozenset(x for x in ix if x not in ex) for ix in net.indices]


def node_label_sets(net, tree, exclude=()):
    """Label set of every node (leaves then internal), outputs and ``exclude`` removed."""
    sets = _base_sets(net, exclude)
    for a, b in np.asarray(tree).reshape(-1, 2):
        sets.append(sets[a] ^ sets[b])
    return sets


def tree_stats(net, tree, sliced=()):
    """Per-slice width (log2 elements of the largest intermediate) and complex flops (8 M N K)."""
    n = net.n_tensors
    sets = node_label_sets(net, tree, exclude=sliced)
    flops = 0
    width = 0
    steps = []
    for t, (a, b) in enumerate(np.asarray(tree).reshape(-1, 2)):
        allx = sets[a] | sets[b]
        k = len(sets[a] & sets[b])
        m = len(sets[a]) - k
        nn = len(sets[b]) - k
        f = 8 * (2 ** len(allx))
        flops += f
        width = max(width, len(sets[n + t]))
        steps.append((m, nn, k))
    return {"width": width, "flops_per_slice": flops, "n_slices": 2 ** len(sliced),
            "total_flops": flops * 2 ** len(sliced), "steps": steps}


def greedy_tree(net, seed=0, alpha=1.0, temperature=0.0):
    """One seeded greedy trial.  Returns an int32 SSA tree."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sets = _base_sets(net)
    n = len(sets)
    active = {}
    where = {}
    for i, s in enumerate(sets):
        active[i] = s
        for x in s:
            where.setdefault(x, set()).add(i)

    heap = []
    counter = [0]

    def score(a, b):
        sa, sb = active[a], active[b]
        sc = sa ^ sb
        cost = 2.0 ** len(sc) - alpha * (2.0 ** len(sa) + 2.0 ** len(sb))
        key = math.copysign(math.log2(1.0 + abs(cost)), cost)
        if temperature > 0:
            key -= temperature * -math.log(-math.log(rng.uniform(1e-300, 1.0)))
        return key

    def push(a, b):
        if a > b:
            a, b = b, a
        counter[0] += 1
        heapq.heappush(heap, (score(a, b), rng.random(), a, b))

    seen = set()
    for x, ids in where.items():
        ids = sorted(ids)
        for i in range(len(ids)):
            for j in range(i + 1, len(ids)):
                if (ids[i], ids[j]) not in seen:
                    seen.add((ids[i], ids[j]))
                    push(ids[i], ids[j])

    tree = []
    next_id = n
    while heap:
        _, _, a, b = heapq.heappop(heap)
        if a not in active or b not in active:
            continue
        sa, sb = active.pop(a), active.pop(b)
        sc = sa ^ sb
        for x in sa:
            where[x].discard(a)
        for x in sb:
            where[x].discard(b)
        c = next_id
        next_id += 1
        tree.append((a, b))
        active[c] = sc
        nbrs = set()
        for x in sc:
            nbrs |= where[x]
            where[x].add(c)
        for d in sorted(nbrs):
            push(d, c)
    # disconnected components: join smallest first
    while len(active) > 1:
        ids = sorted(active, key=lambda i: (len(active[i]), i))
        a, b = ids[0], ids[1]
        sa, sb = active.pop(a), active.pop(b)
        tree.append((a, b))
        active[next_id] = sa ^ sb
        next_id += 1
    return np.array(tree, dtype=np.int32).reshape(-1, 2)


def tree_trimming(net, tree, n_sliced, seed=0):
    """Greedy slice selection; returns the sliced labels in selection order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = net.n_tensors
    base = node_label_sets(net, tree)
    inter = base[n:]
    sliced = []
    sset = set()
    for _ in range(n_sliced):
        cur = [s - sset for s in inter]
        wmax = max(len(s) for s in cur)
        largest = [s for s in cur if len(s) == wmax]
        cand = set()
        for s in largest:
            cand |= s
        if not cand:
            raise ValueError("nothing left to slice")
        key1 = {e: 0 for e in cand}
        for s in largest:
            for e in s:
                key1[e] += 1
        key2 = {e: 0 for e in cand}
        for s in cur:
            sz = 2 ** len(s)
            for e in s:
                if e in key2:
                    key2[e] += sz
        best = max(sorted(cand), key=lambda e: (key1[e], key2[e], rng.random()))
        sliced.append(int(best))
        sset.add(best)
    return sliced


def plan_network(net, n_sliced, trials=16, seed=0, width_cap=None):
    """Best of ``trials`` noisy greedy trees, each sliced by tree trimming.

    Trial 0 is the plain greedy (alpha=1, no noise).  A tree is ranked by
    (sliced width above ``width_cap``, total sliced flops).  Returns
    (tree, sliced_labels, stats).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    best = None
    for t in range(trials):
        if t == 0:
            alpha, temp = 1.0, 0.0
        else:
            alpha = float(rng.uniform(0.5, 1.0))
            temp = float(rng.uniform(0.05, 1.5))
        tseed = int(rng.integers(0, 2 ** 31))
        tree = greedy_tree(net, seed=tseed, alpha=alpha, temperature=temp)
        sliced = tree_trimming(net, tree, n_sliced, seed=tseed + 1) if n_sliced else []
        st = tree_stats(net, tree, sliced)
        over = max(0, st["width"] - width_cap) if width_cap is not None else 0
        key = (over, st["total_flops"])
        if best is None or key < best[0]:
            st["trial"] = t
            best = (key, tree, sliced, st)
    return best[1], best[2], best[3]
