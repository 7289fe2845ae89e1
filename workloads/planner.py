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
* ``local_reconfigure`` -- local optimisation of sub-trees, the improvement the
  paper names as future work (Sec. V): under each expensive node a window of at
  most ``window`` sub-trees is re-ordered optimally (dynamic programming over
  the window's subsets, cost = per-slice flops with sliced and output labels
  closed), never creating an intermediate wider than the tree already has.
  ``plan_network`` can alternate it with tree trimming.

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


def greedy_tree(net, seed=0, alpha=1.0, temperature=0.0, exclude=()):
    """One seeded greedy trial.  Returns an int32 SSA tree.  Labels in ``exclude`` (e.g. sliced ones,
    whose values are fixed) do not count towards sizes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sets = _base_sets(net, exclude)
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


def contraction_cost(sa, sb, mem_weight=0.0):
    """Cost of contracting label sets sa and sb: 2^|sa | sb| (flops / 8), or with mem_weight = r > 0
    a roofline estimate max(2^|sa | sb|, r (2^|sa| + 2^|sb| + 2^|sa ^ sb|)), r being the flop:element
    ratio at which the device turns from memory- to compute-bound."""
    f = 2.0 ** len(sa | sb)
    if mem_weight > 0:
        f = max(f, mem_weight * (2.0 ** len(sa) + 2.0 ** len(sb) + 2.0 ** len(sa ^ sb)))
    return f


def tree_cost(net, tree, sliced=(), mem_weight=0.0):
    """Sum of contraction_cost over the tree's steps (per slice)."""
    sets = node_label_sets(net, tree, exclude=sliced)
    return sum(contraction_cost(sets[a], sets[b], mem_weight) for a, b in np.asarray(tree).reshape(-1, 2))


def local_reconfigure(net, tree, sliced=(), window=8, sweeps=2, mem_weight=0.0):
    """Re-orders small sub-trees optimally; returns an SSA tree of equal or lower per-slice flops.

    For every internal node, most expensive first, the window is grown from the node by repeatedly
    replacing its most expensive internal member with that member's two children, up to ``window``
    members.  The window's result has a fixed label set whatever the order inside, so only the
    window's own contractions change; the cheapest order over its members is found by dynamic
    programming over subsets (best[S] = min over splits S = A + B of best[A] + best[B] +
    cost(labels(A), labels(B)), cost = ``contraction_cost``) and replaces the old one when strictly
    cheaper.  Sets wider than the tree's widest intermediate are not allowed.
    """
    n = net.n_tensors
    tree = np.asarray(tree).reshape(-1, 2)
    base = _base_sets(net, sliced)
    lab = {i: base[i] for i in range(n)}
    kids = {}
    for t, (a, b) in enumerate(tree):
        kids[n + t] = (int(a), int(b))
        lab[n + t] = lab[int(a)] ^ lab[int(b)]
    root = n + len(tree) - 1 if len(tree) else 0
    wcap = max((len(lab[v]) for v in kids), default=0)
    next_id = n + len(tree)

    def cost(v):
        a, b = kids[v]
        return contraction_cost(lab[a], lab[b], mem_weight)

    for _ in range(sweeps):
        improved = False
        for v in sorted(kids, key=lambda u: -cost(u)):
            if v not in kids:
                continue
            front, inner = [v], []
            while len(front) < window:
                cand = [u for u in front if u in kids]
                if not cand:
                    break
                u = max(cand, key=lambda x: (cost(x), x))
                front.remove(u)
                inner.append(u)
                front += list(kids[u])
            if len(front) < 3:
                continue
            old = sum(cost(u) for u in inner)
            m = len(front)
            full = (1 << m) - 1
            ls = [frozenset()] * (1 << m)
            for S in range(1, full + 1):
                low = S & -S
                ls[S] = ls[S ^ low] ^ lab[front[low.bit_length() - 1]]
            best = [math.inf] * (1 << m)
            split = [0] * (1 << m)
            for i in range(m):
                best[1 << i] = 0.0
            for S in range(1, full + 1):
                if S & (S - 1) == 0 or (len(ls[S]) > wcap and S != full):
                    continue
                low = S & -S
                rest = S ^ low
                sub = rest
                while True:
                    A = low | sub
                    if A != S:
                        B = S ^ A
                        if best[A] < math.inf and best[B] < math.inf:
                            c = best[A] + best[B] + contraction_cost(ls[A], ls[B], mem_weight)
                            if c < best[S]:
                                best[S], split[S] = c, A
                    if sub == 0:
                        break
                    sub = (sub - 1) & rest
            if not best[full] < old * (1 - 1e-9):
                continue
            for u in inner:
                del kids[u]

            def build(S, node=None):
                nonlocal next_id
                if S & (S - 1) == 0:
                    return front[S.bit_length() - 1]
                A = split[S]
                a, b = build(A), build(S ^ A)
                if node is None:
                    node = next_id
                    next_id += 1
                kids[node] = (a, b)
                lab[node] = ls[S]
                return node

            build(full, v)
            improved = True
        if not improved:
            break

    # back to SSA order (post-order from the root)
    out, ids = [], {i: i for i in range(n)}
    stack = [(root, False)] if len(tree) else []
    while stack:
        v, done = stack.pop()
        if v < n:
            continue
        if done:
            a, b = kids[v]
            out.append((ids[a], ids[b]))
            ids[v] = n + len(out) - 1
        else:
            stack.append((v, True))
            a, b = kids[v]
            stack.append((b, False))
            stack.append((a, False))
    return np.array(out, dtype=np.int32).reshape(-1, 2)


def plan_network(net, n_sliced, trials=16, seed=0, width_cap=None, reconfigure=0, window=8, mem_weight=0.0):
    """Best of ``trials`` noisy greedy trees, each sliced by tree trimming.

    Trial 0 is the plain greedy (alpha=1, no noise).  A tree is ranked by
    (sliced width above ``width_cap``, total sliced flops).  With ``reconfigure`` = r > 0 the
    best r trials are then refined by alternating local sub-tree re-ordering and re-slicing
    (two rounds) and ranked again; with ``mem_weight`` > 0 each is refined under both the flop and
    the roofline cost of ``contraction_cost`` and all are ranked by the roofline cost.  Returns
    (tree, sliced_labels, stats).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ranked = []
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
        st["trial"] = t
        ranked.append(((over, st["total_flops"]), t, tree, sliced, st, tseed))
    ranked.sort(key=lambda r: (r[0], r[1]))
    best = ranked[0]
    if reconfigure and mem_weight > 0:
        # rank on the same cost the refinement minimises
        k0 = best[0][0], tree_cost(net, best[2], best[3], mem_weight) * 2 ** len(best[3])
        best = (k0,) + best[1:]
    # the local search lands in different optima under the two costs, so with a roofline cost
    # both refinements are tried and ranked by the roofline cost
    weights = (0.0, mem_weight) if mem_weight > 0 else (0.0,)
    for key, t, tree0, sliced0, st, tseed in ranked[:reconfigure]:
        for mw in weights:
            tree, sliced = tree0, sliced0
            for r in range(2):
                tree = local_reconfigure(net, tree, sliced, window=window, mem_weight=mw)
                sliced = tree_trimming(net, tree, n_sliced, seed=tseed + 2 + r) if n_sliced else []
            tree = local_reconfigure(net, tree, sliced, window=window, mem_weight=mw)
            st = tree_stats(net, tree, sliced)
            over = max(0, st["width"] - width_cap) if width_cap is not None else 0
            st["trial"] = t
            st["reconfigured"] = True
            total = (st["total_flops"] if mem_weight <= 0
                     else tree_cost(net, tree, sliced, mem_weight) * 2 ** len(sliced))
            if ((over, total), t) < (best[0], best[1]):
                best = ((over, total), t, tree, sliced, st, tseed)
    return best[2], best[3], best[4]
