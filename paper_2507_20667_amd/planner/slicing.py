"""Slicing on top of partitioning: fix some legs so that every intermediate
fits, contract once per assignment of the fixed legs, and add the results.

A contraction is a sum over every bound index (Section 2.2), so restricting a
leg to one value and summing over its values gives the same result; the tree
and the partition stay as they are.  Here a sliced leg keeps its label with
dimension 1, and slice number s overrides every tensor that carries a sliced
leg with its sub-tensor at that leg's value: all slices share one plan (the
network with the sliced dimensions) and run as one batch of queries through
the library; the slice results are added in FP64 on the device (tn_plan_slice).
"""
from __future__ import annotations

import itertools

import numpy as np

from .cost import node_legs, size_of


def largest_after(leaf_legs, dims, tree, sliced) -> int:
    """Largest intermediate (entries) of the tree with the legs in `sliced`
    at dimension 1."""
    d = dict(dims)
    for l in sliced:
        d[l] = 1
    legs = node_legs(leaf_legs, tree)
    nv = len(leaf_legs)
    return max((size_of(legs[v], d) for v in range(nv, len(legs))), default=1)


def choose_slices(leaf_legs, dims, tree, target_elems: int, max_legs: int = 16) -> list:
    """Bound legs to fix until the largest intermediate of `tree` holds at most
    `target_elems` entries: greedily the leg whose fixing shrinks the current
    largest intermediate most (ties: the leg on most intermediates of that
    size, then the lower label).  Open legs are never sliced."""
    count = {}
    for l in leaf_legs:
        for e in l:
            count[e] = count.get(e, 0) + 1
    bound = sorted(e for e, c in count.items() if c == 2 and dims[e] > 1)
    legs = node_legs(leaf_legs, tree)
    nv = len(leaf_legs)
    sliced = []
    while len(sliced) < max_legs:
        d = dict(dims)
        for l in sliced:
            d[l] = 1
        sizes = [size_of(legs[v], d) for v in range(nv, len(legs))]
        top = max(sizes, default=1)
        if top <= target_elems:
            break
        best, best_key = None, None
        for e in bound:
            if e in sliced:
                continue
            on_top = sum(1 for v, s in zip(range(nv, len(legs)), sizes) if s == top and e in legs[v])
            if on_top == 0:
                continue
            after = largest_after(leaf_legs, dims, tree, sliced + [e])
            key = (after, -on_top, e)
            if best_key is None or key < best_key:
                best, best_key = e, key
        if best is None:
            break
        sliced.append(best)
    return sliced


def sliced_problem(leaf_legs, dims, tensors, sliced):
    """(dims with the sliced legs at 1, slice 0's tensors, one override dict
    per slice).  Slice s fixes sliced[k] to digit k of s in the mixed radix of
    the sliced dimensions (last leg fastest); the overrides replace every
    tensor that carries a sliced leg."""
    d = dict(dims)
    for l in sliced:
        d[l] = 1
    touched = [t for t, l in enumerate(leaf_legs) if any(e in sliced for e in l)]

    def sub(t, values):
        a = np.asarray(tensors[t])
        idx = tuple(slice(values[e], values[e] + 1) if e in values else slice(None) for e in leaf_legs[t])
        return a[idx]

    ranges = [range(dims[l]) for l in sliced]
    overrides = []
    for vals in itertools.product(*ranges):
        values = dict(zip(sliced, vals))
        overrides.append({t: sub(t, values) for t in touched})
    base = list(tensors)
    for t in touched:
        base[t] = overrides[0][t]
    return d, base, overrides


def contract_sliced(lib, ctx, leaf_legs, dims, tensors, partition_of, num_partitions, tree,
                    sliced, output_legs=None, flags=0, result_shape=(), extra_overrides=None):
    """Contract the network with the legs in `sliced` fixed slice by slice: the
    library's sliced plan (tn_plan_slice) runs every slice as one query of one
    batch and adds the slice results on the device in FP64.  Returns the
    result (complex128, `result_shape`)."""
    p = ctx.plan_load(leaf_legs, dims, tensors, partition_of, num_partitions, tree, output_legs, flags)
    try:
        s = ctx.slice_plan(p, list(sliced))
        try:
            out, _ = lib.tn_contract(s, extra_overrides or {}, result_shape=tuple(result_shape))
            return np.asarray(out, dtype=np.complex128)
        finally:
            ctx.free_plan(s)
    finally:
        ctx.free_plan(p)
