"""Plans: a partitioning K plus a contraction tree (B, b) that accepts it.

A plan is built the way Section 4.4 describes: a Greedy tree inside every
partition, then a RandomGreedy reduction path over the partition results; its
score is eq. con_dist with con = con_serial and comm = 0 (Section 5.2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import json
from math import prod

from .greedy import greedy_pairs, random_greedy_pairs


@dataclass
class PartTree:
    """Greedy tree of one partition, in local SSA ids (leaves 0..m-1)."""
    members: list
    pairs: list
    legs: list        # legs of every local vertex
    leafsets: list    # global tensor ids under every local vertex
    weight: int       # con_serial(B_k)

    @property
    def root(self) -> int:
        return len(self.legs) - 1

    @property
    def root_legs(self) -> frozenset:
        return self.legs[-1]


def build_part(members, leaf_legs, dims) -> PartTree:
    members = sorted(members)
    items = [frozenset(leaf_legs[t]) for t in members]
    pairs = greedy_pairs(items, dims)
    legs = list(items)
    leafsets = [frozenset([t]) for t in members]
    weight = 0
    for a, b in pairs:
        weight += prod(dims[e] for e in (legs[a] | legs[b]))
        legs.append(legs[a] ^ legs[b])
        leafsets.append(leafsets[a] | leafsets[b])
    return PartTree(members, pairs, legs, leafsets, weight)


def reduction_value(bases, red_pairs, root_legs, dims) -> int:
    """con_dist given the partition costs `bases` and a reduction path over
    the partition results: a leaf carries con(B_k), an internal vertex adds its
    2^vc to the larger of its children."""
    k = len(bases)
    val = list(bases)
    legs = list(root_legs)
    for a, b in red_pairs:
        w = prod(dims[e] for e in (legs[a] | legs[b]))
        legs.append(legs[a] ^ legs[b])
        val.append(w + max(val[a], val[b]))
    return val[-1] if red_pairs else (val[0] if k else 0)


def plan_reduction(parts, dims, rng=None, samples=64, temperature=0.1):
    roots = [p.root_legs for p in parts]
    bases = [p.weight for p in parts]
    if len(parts) == 1:
        return [], bases[0]
    if rng is None:
        pairs = greedy_pairs(roots, dims)
        return pairs, reduction_value(bases, pairs, roots, dims)
    return random_greedy_pairs(roots, dims,
                               lambda pr: reduction_value(bases, pr, roots, dims),
                               rng, samples, temperature)


def assemble_tree(num_tensors, parts, red_pairs):
    """Global SSA tree: partition trees in partition order, then the reduction
    path.  Returns (tree, partition root ids)."""
    tree = []
    nxt = num_tensors
    roots = []
    for p in parts:
        idmap = list(p.members)
        for a, b in p.pairs:
            tree.append((idmap[a], idmap[b]))
            idmap.append(nxt)
            nxt += 1
        roots.append(idmap[-1])
    idmap = list(roots)
    for a, b in red_pairs:
        tree.append((idmap[a], idmap[b]))
        idmap.append(nxt)
        nxt += 1
    return tree, roots


@dataclass
class Plan:
    partition_of: list
    num_partitions: int
    tree: list
    meta: dict = field(default_factory=dict)

    def to_json(self) -> str:
        return json.dumps(dict(partition_of=list(map(int, self.partition_of)),
                               num_partitions=int(self.num_partitions),
                               tree=[[int(a), int(b)] for a, b in self.tree],
                               meta=self.meta))

    @staticmethod
    def from_json(s: str) -> "Plan":
        d = json.loads(s)
        return Plan(d["partition_of"], d["num_partitions"], [tuple(p) for p in d["tree"]],
                    d.get("meta", {}))


def contiguous_partition(num_tensors: int, k: int) -> list:
    """Tensors in generation order split into k contiguous, near-equal parts
    (the stand-in for the paper's unspecified naive partitioning)."""
    return [i * k // num_tensors for i in range(num_tensors)]


def tree_partition(leaf_legs, dims, k: int) -> list:
    """Initial K-way partitioning cut from a whole-network Greedy tree: start
    from the root and repeatedly replace the subtree with the largest
    con_serial (ties: more leaves, then lower id) by its two children, until
    there are k subtrees.  The tree accepts the result by construction.  This
    stands in for the hypergraph min-cut partitioner the paper starts from
    (Section 4.2), which is not available here."""
    nv = len(leaf_legs)
    items = [frozenset(l) for l in leaf_legs]
    pairs = greedy_pairs(items, dims)
    legs = list(items)
    weight = [0] * nv
    nleaves = [1] * nv
    for a, b in pairs:
        w = prod(dims[e] for e in (legs[a] | legs[b]))
        legs.append(legs[a] ^ legs[b])
        weight.append(w + weight[a] + weight[b])
        nleaves.append(nleaves[a] + nleaves[b])
    parts = [len(legs) - 1]
    while len(parts) < min(k, nv):
        splittable = [v for v in parts if v >= nv]
        v = max(splittable, key=lambda x: (weight[x], nleaves[x], -x))
        parts.remove(v)
        parts.extend(pairs[v - nv])
    owner = [0] * nv

    def leaves_of(v):
        out, stack = [], [v]
        while stack:
            u = stack.pop()
            if u < nv:
                out.append(u)
            else:
                stack.extend(pairs[u - nv])
        return out

    groups = sorted((sorted(leaves_of(v)) for v in parts), key=lambda g: g[0])
    for idx, g in enumerate(groups):
        for t in g:
            owner[t] = idx
    return owner


def plan_from_partition(leaf_legs, dims, partition_of, num_partitions, rng=None,
                        samples=64, temperature=0.1) -> Plan:
    parts = []
    for k in range(num_partitions):
        members = [t for t, p in enumerate(partition_of) if p == k]
        if not members:
            raise ValueError(f"partition {k} is empty")
        parts.append(build_part(members, leaf_legs, dims))
    red, cost = plan_reduction(parts, dims, rng, samples, temperature)
    tree, _ = assemble_tree(len(leaf_legs), parts, red)
    return Plan(list(partition_of), num_partitions, tree, dict(con_dist=str(cost)))
