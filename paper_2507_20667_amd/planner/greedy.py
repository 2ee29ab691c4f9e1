"""Greedy and RandomGreedy contraction paths (Sections 2.3 and 4.4).

Greedy repeatedly contracts the connected pair with the largest memory
reduction |A| + |B| - |A (.) B| (eq. greedy_mem_reduction); ties go to the
lowest (smaller id, larger id).  Components that share no edge are joined at
the end by outer products, two smallest first.

RandomGreedy samples several such paths with Gumbel noise on a log-scaled
version of the same score and keeps the best under a caller-supplied cost;
sample 0 is the noiseless Greedy path, so RandomGreedy never does worse than
Greedy under that cost.
"""
from __future__ import annotations

import heapq
import math
from math import prod


def _size(legs, dims):
    return prod(dims[e] for e in legs)


def greedy_pairs(items, dims, rng=None, temperature: float = 0.0):
    """Contraction path over `items` (a list of leg sets).

    Returns the SSA pair list over local ids: leaves 0..m-1, internal vertex
    m+j is pair j.  With m == 1 the list is empty."""
    m = len(items)
    legs = {i: frozenset(items[i]) for i in range(m)}
    size = {i: _size(legs[i], dims) for i in range(m)}
    holders = {}
    for i in range(m):
        for e in legs[i]:
            holders.setdefault(e, set()).add(i)
    noisy = rng is not None and temperature > 0.0
    heap = []

    def push(a, b):
        lo, hi = (a, b) if a < b else (b, a)
        c = legs[a] ^ legs[b]
        score = size[a] + size[b] - _size(c, dims)
        if noisy:
            s = math.copysign(math.log2(1.0 + abs(score)), score)
            g = -math.log(-math.log(max(rng.random(), 1e-300)))
            key = -(s + temperature * g)
        else:
            key = -score
        heapq.heappush(heap, (key, lo, hi))

    # edges in label order, so that the order of the pushes (and of the noise
    # draws) does not depend on how a set happens to iterate
    seen = set()
    for e in sorted(holders):
        hs = sorted(holders[e])
        for x in range(len(hs)):
            for y in range(x + 1, len(hs)):
                p = (hs[x], hs[y])
                if p not in seen:
                    seen.add(p)
                    push(*p)
    alive = set(range(m))
    pairs = []
    nxt = m
    while heap:
        _, a, b = heapq.heappop(heap)
        if a not in alive or b not in alive:
            continue
        c = nxt
        nxt += 1
        pairs.append((a, b))
        legs[c] = legs[a] ^ legs[b]
        size[c] = _size(legs[c], dims)
        alive.discard(a)
        alive.discard(b)
        for e in legs[a] | legs[b]:
            hs = holders.get(e)
            if hs is not None:
                hs.discard(a)
                hs.discard(b)
        nbrs = set()
        for e in legs[c]:
            hs = holders.setdefault(e, set())
            nbrs.update(hs)
            hs.add(c)
        alive.add(c)
        for nb in sorted(nbrs):
            if nb in alive and nb != c:
                push(nb, c)
    while len(alive) > 1:
        a, b = sorted(alive, key=lambda i: (size[i], i))[:2]
        lo, hi = min(a, b), max(a, b)
        c = nxt
        nxt += 1
        pairs.append((lo, hi))
        legs[c] = legs[a] ^ legs[b]
        size[c] = _size(legs[c], dims)
        alive.discard(a)
        alive.discard(b)
        alive.add(c)
    return pairs


def random_greedy_pairs(items, dims, cost_fn, rng, samples: int = 64, temperature: float = 0.1):
    """Best of `samples` noised Greedy paths under cost_fn(pairs) (lower is
    better; ties keep the earliest sample).  Returns (pairs, cost)."""
    best = None
    best_cost = None
    for s in range(samples):
        pairs = greedy_pairs(items, dims, rng if s > 0 else None, temperature if s > 0 else 0.0)
        c = cost_fn(pairs)
        if best_cost is None or c < best_cost:
            best, best_cost = pairs, c
    return best, best_cost
