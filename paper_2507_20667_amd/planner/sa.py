"""Simulated-annealing refinement of a partitioning (Section 4.3, Algorithms 1
and 2).

State: a partitioning K with a Greedy tree per partition and a RandomGreedy
reduction path; its cost is eq. con_dist (con = con_serial, comm = 0).

Neighbour (Algorithm 2, Rebalance): pick a source partition with at least two
tensors, pick a vertex of its tree other than its root (so the source is never
emptied), move the tensors under that vertex to a destination partition chosen
at random (SelectTargetNaive) or as the partition whose root tensor gives the
largest memory reduction when contracted with the moved subtree's tensor
(SelectTargetDirected, eq. greedy_mem_reduction), then re-plan the two changed
partitions and the reduction path.  The pseudo-code's move set reads
b^-1(leaves(B_{k_src})); the text and figure move the subtree at the chosen
vertex, which is what is done here.

Acceptance uses the log-ratio form P = exp(-log(c_new/c)/T) and the cooling
schedule T(t) = T0 * (Tf/T0)^t.  Each temperature iteration runs ceil(N/p)
steps on each of p workers from the same state and keeps the cheapest result
(division algorithm); the best state so far is tracked and the search restarts
from it after RestartThreshold iterations without improvement.

The paper leaves T0, Tf, N, p, the threshold and the time limit to the user;
the defaults below are this implementation's choices.  With `iterations`
given, t = i / iterations replaces elapsed / time_limit so that a run is
reproducible from (seed, iterations).
"""
from __future__ import annotations

from dataclasses import dataclass
import math
import time

import numpy as np

from .plan import PartTree, Plan, assemble_tree, build_part, plan_reduction


@dataclass
class SAState:
    partition_of: list
    parts: list
    red_pairs: list
    cost: int


@dataclass
class SAConfig:
    t0: float = 1.0
    tf: float = 0.05
    n_steps: int = 64
    workers: int = 4
    restart_threshold: int = 20
    iterations: int | None = 30
    time_limit: float | None = None
    directed: bool = True
    rg_samples: int = 16
    rg_temperature: float = 0.1
    seed: int = 0


def objective(legs_a, legs_b, dims) -> int:
    """|A| + |B| - |A (.) B| for two leg sets."""
    def sz(s):
        return math.prod(dims[e] for e in s)
    return sz(legs_a) + sz(legs_b) - sz(legs_a ^ legs_b)


class Annealer:
    def __init__(self, leaf_legs, dims, num_partitions, cfg: SAConfig):
        self.leaf_legs = [frozenset(l) for l in leaf_legs]
        self.dims = dims
        self.k = num_partitions
        self.cfg = cfg
        self.evaluations = 0

    def make_state(self, partition_of, rng) -> SAState:
        parts = [build_part([t for t, p in enumerate(partition_of) if p == k], self.leaf_legs,
                            self.dims) for k in range(self.k)]
        red, cost = plan_reduction(parts, self.dims, rng, self.cfg.rg_samples,
                                   self.cfg.rg_temperature)
        self.evaluations += 1
        return SAState(list(partition_of), parts, red, cost)

    def neighbour(self, s: SAState, rng) -> SAState:
        sources = [k for k in range(self.k) if len(s.parts[k].members) >= 2]
        if not sources or self.k < 2:
            return s
        ksrc = sources[int(rng.integers(0, len(sources)))]
        src: PartTree = s.parts[ksrc]
        v = int(rng.integers(0, src.root))       # any vertex of B_src but its root
        moved = src.leafsets[v]
        if self.cfg.directed:
            best_k, best_obj = None, None
            for k in range(self.k):
                if k == ksrc:
                    continue
                o = objective(src.legs[v], s.parts[k].root_legs, self.dims)
                if best_obj is None or o > best_obj:
                    best_k, best_obj = k, o
            kdst = best_k
        else:
            r = int(rng.integers(0, self.k - 1))
            kdst = r if r < ksrc else r + 1
        pof = list(s.partition_of)
        for t in moved:
            pof[t] = kdst
        parts = list(s.parts)
        for k in (ksrc, kdst):
            parts[k] = build_part([t for t, p in enumerate(pof) if p == k], self.leaf_legs,
                                  self.dims)
        red, cost = plan_reduction(parts, self.dims, rng, self.cfg.rg_samples,
                                   self.cfg.rg_temperature)
        self.evaluations += 1
        return SAState(pof, parts, red, cost)

    def do_steps(self, n, s: SAState, temp, rng) -> SAState:
        for _ in range(n):
            new = self.neighbour(s, rng)
            if s.cost == 0:
                accept = new.cost <= s.cost
            elif new.cost <= s.cost:
                accept = True
            else:
                p = math.exp(-(math.log(new.cost) - math.log(s.cost)) / temp)
                accept = p >= rng.random()
            if accept:
                s = new
        return s

    def run(self, initial_partition_of) -> tuple:
        cfg = self.cfg
        rngs = [np.random.default_rng([cfg.seed, w]) for w in range(cfg.workers)]
        cur = self.make_state(initial_partition_of, rngs[0])
        best = cur
        i_best = i = -1
        alpha = cfg.tf / cfg.t0
        n_p = -(-cfg.n_steps // cfg.workers)
        start = time.monotonic()
        history = []
        while True:
            if cfg.iterations is not None:
                if i + 1 >= cfg.iterations:
                    break
                t = (i + 1) / cfg.iterations
            else:
                elapsed = time.monotonic() - start
                if elapsed >= cfg.time_limit:
                    break
                t = elapsed / cfg.time_limit
            i += 1
            temp = cfg.t0 * alpha ** t
            results = [self.do_steps(n_p, cur, temp, rngs[w]) for w in range(cfg.workers)]
            cur = min(enumerate(results), key=lambda x: (x[1].cost, x[0]))[1]
            if cur.cost < best.cost:
                i_best, best = i, cur
            elif i - i_best >= cfg.restart_threshold:
                i_best, cur = i, best
            history.append((i, temp, cur.cost, best.cost))
        return best, history


def simulated_annealing(leaf_legs, dims, initial_partition_of, num_partitions,
                        cfg: SAConfig | None = None) -> Plan:
    cfg = cfg or SAConfig()
    ann = Annealer(leaf_legs, dims, num_partitions, cfg)
    init = ann.make_state(initial_partition_of, np.random.default_rng([cfg.seed, 0]))
    best, history = ann.run(initial_partition_of)
    tree, roots = assemble_tree(len(leaf_legs), best.parts, best.red_pairs)
    meta = dict(method="sa-directed" if cfg.directed else "sa-naive", seed=cfg.seed,
                t0=cfg.t0, tf=cfg.tf, n_steps=cfg.n_steps, workers=cfg.workers,
                restart_threshold=cfg.restart_threshold, iterations=cfg.iterations,
                rg_samples=cfg.rg_samples, rg_temperature=cfg.rg_temperature,
                initial_con_dist=str(init.cost), con_dist=str(best.cost),
                evaluations=ann.evaluations)
    return Plan(best.partition_of, num_partitions, tree, meta)
