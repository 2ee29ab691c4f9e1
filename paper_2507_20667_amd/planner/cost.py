"""Cost model of Section 3, in exact Python integers.

A contraction tree is given in SSA form: with |V| leaves numbered 0..|V|-1,
internal node |V|+j contracts the pair tree[j]; the last pair is the root.

Readings where the paper leaves room:
  * path(v, u) includes both end points, so the leaf-to-root paths of the
    critical path (eq. con_par) drop only the leaf and keep the root, and the
    paths of eq. con_dist drop root(B_k) and keep root(B);
  * 2^vc(v) is taken as the exact product of the edge dimensions of E(v);
  * comm(c) is 0, as in the paper's experiments; con inside con_dist is
    con_serial unless asked otherwise.
"""
from __future__ import annotations

from math import prod


def node_legs(leaf_legs, tree):
    """legs(v) for every tree vertex (Section 2.3): a leaf's edges, and for an
    internal vertex the symmetric difference of its children's legs."""
    legs = [frozenset(l) for l in leaf_legs]
    for a, b in tree:
        legs.append(legs[a] ^ legs[b])
    return legs


def node_weights(leaf_legs, dims, tree):
    """2^vc(v) = product of n(e) over E(v), the union of the children's legs,
    for every internal vertex, in SSA order."""
    legs = node_legs(leaf_legs, tree)
    return [prod(dims[e] for e in (legs[a] | legs[b])) for a, b in tree]


def size_of(legset, dims) -> int:
    return prod(dims[e] for e in legset)


def con_serial(leaf_legs, dims, tree) -> int:
    """Eq. con_serial: sum of 2^vc over internal vertices."""
    return sum(node_weights(leaf_legs, dims, tree))


def _parents(nv, tree):
    par = [-1] * (nv + len(tree))
    for j, (a, b) in enumerate(tree):
        par[a] = nv + j
        par[b] = nv + j
    return par


def con_par(leaf_legs, dims, tree) -> int:
    """Eq. con_par: the largest sum of 2^vc along a leaf-to-root path, the leaf
    itself excluded."""
    nv = len(leaf_legs)
    w = node_weights(leaf_legs, dims, tree)
    # best[v] = heaviest path from any leaf below v up to v (v included)
    best = [0] * (nv + len(tree))
    for j, (a, b) in enumerate(tree):
        best[nv + j] = w[j] + max(best[a], best[b])
    return best[-1] if tree else 0


def leaf_sets(nv, tree):
    sets = [frozenset([i]) for i in range(nv)]
    for a, b in tree:
        sets.append(sets[a] | sets[b])
    return sets


def partition_roots(nv, tree, partition_of, num_partitions):
    """For each partition k the tree vertex whose leaf set equals k (the
    acceptance condition of Section 2.4), or None if the tree does not accept
    the partitioning."""
    sets = leaf_sets(nv, tree)
    want = {}
    for v, k in enumerate(partition_of):
        want.setdefault(k, set()).add(v)
    index = {s: i for i, s in enumerate(sets)}
    roots = []
    for k in range(num_partitions):
        s = frozenset(want.get(k, ()))
        if not s or s not in index:
            return None
        roots.append(index[s])
    return roots


def subtree_weight(nv, tree, w, root) -> int:
    """Sum of 2^vc over the internal vertices of the subtree rooted at `root`."""
    if root < nv:
        return 0
    total = 0
    stack = [root]
    while stack:
        v = stack.pop()
        if v < nv:
            continue
        j = v - nv
        total += w[j]
        stack.extend(tree[j])
    return total


def subtree_par(nv, tree, w, root) -> int:
    if root < nv:
        return 0
    best = {}
    order = []
    stack = [root]
    while stack:
        v = stack.pop()
        if v >= nv:
            order.append(v)
            stack.extend(tree[v - nv])
    for v in reversed(order):
        a, b = tree[v - nv]
        best[v] = w[v - nv] + max(best.get(a, 0), best.get(b, 0))
    return best[root]


def con_dist(leaf_legs, dims, tree, partition_of, num_partitions, con="serial") -> int:
    """Eq. con_dist with comm = 0: the largest, over partitions k, of con(B_k)
    plus the 2^vc of every vertex above root(B_k) on the way to root(B)."""
    nv = len(leaf_legs)
    w = node_weights(leaf_legs, dims, tree)
    roots = partition_roots(nv, tree, partition_of, num_partitions)
    if roots is None:
        raise ValueError("tree does not accept the partitioning")
    par = _parents(nv, tree)
    best = 0
    for r in roots:
        c = subtree_weight(nv, tree, w, r) if con == "serial" else subtree_par(nv, tree, w, r)
        v = par[r]
        while v != -1:
            c += w[v - nv]
            v = par[v]
        best = max(best, c)
    return best


def mem(leaf_legs, dims, tree) -> int:
    """Eq. mem: the largest |v| + |c1| + |c2| over internal vertices, in
    elements."""
    legs = node_legs(leaf_legs, tree)
    nv = len(leaf_legs)
    out = 0
    for j, (a, b) in enumerate(tree):
        out = max(out, size_of(legs[nv + j], dims) + size_of(legs[a], dims) + size_of(legs[b], dims))
    return out


def largest_intermediate(leaf_legs, dims, tree) -> int:
    legs = node_legs(leaf_legs, tree)
    nv = len(leaf_legs)
    return max((size_of(legs[nv + j], dims) for j in range(len(tree))), default=0)


def all_costs(leaf_legs, dims, tree, partition_of, num_partitions) -> dict:
    return dict(
        con_serial=con_serial(leaf_legs, dims, tree),
        con_par=con_par(leaf_legs, dims, tree),
        con_dist=con_dist(leaf_legs, dims, tree, partition_of, num_partitions),
        mem=mem(leaf_legs, dims, tree),
        largest_intermediate=largest_intermediate(leaf_legs, dims, tree),
    )
