"""Simulated-annealing refinement of a partitioning (Section 4.3, Algorithms 1
and 2).  The search loop is built from a cooling schedule, an acceptance
predicate, a best-state tracker with restarts and a progress clock.

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
    # run the p workers' chains in forked processes (same result as in turn)
    parallel: bool = False


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
        """n Metropolis steps at temperature `temp` from state s."""
        for _ in range(n):
            new = self.neighbour(s, rng)
            if accept(s.cost, new.cost, temp, rng):
                s = new
        return s

    def run(self, initial_partition_of, pool=None) -> tuple:
        """Search from the initial partitioning; returns (best state, history
        of (iteration, temperature, current cost, best cost)).  `pool`: an
        executor whose map runs the workers' step chains side by side (the
        same result as one after another: each worker has its own random
        stream)."""
        cfg = self.cfg
        rngs = [np.random.default_rng([cfg.seed, w]) for w in range(cfg.workers)]
        cur = self.make_state(initial_partition_of, rngs[0])
        track = BestTracker(cur, cfg.restart_threshold)
        clock = Progress(cfg.iterations, cfg.time_limit)
        steps = -(-cfg.n_steps // cfg.workers)     # each worker's share of N
        history = []
        while True:
            t = clock.next()
            if t is None:
                break
            temp = cooling(t, cfg.t0, cfg.tf)
            if pool is None:
                ends = [self.do_steps(steps, cur, temp, r) for r in rngs]
            else:
                out = list(pool.map(_worker_chain, [(self, steps, cur, temp, r) for r in rngs]))
                ends = [e for e, _ in out]
                rngs = [r for _, r in out]
                self.evaluations += steps * len(rngs)
            # the cheapest worker's end state (lowest worker index on ties)
            cur = min(enumerate(ends), key=lambda x: (x[1].cost, x[0]))[1]
            cur = track.update(clock.i, cur)
            history.append((clock.i, temp, cur.cost, track.best.cost))
        return track.best, history


def cooling(t: float, t0: float, tf: float) -> float:
    """Exponential cooling from t0 at progress t = 0 to tf at t = 1."""
    return t0 * (tf / t0) ** t


def accept(c_cur: int, c_new: int, temp: float, rng) -> bool:
    """Metropolis rule on the log of the cost ratio: downhill or equal moves
    always, an uphill move with probability exp(-log(c_new / c_cur) / temp),
    i.e. (c_cur / c_new)^(1 / temp).  A draw is made only for uphill moves."""
    if c_new <= c_cur:
        return True
    if c_cur == 0:
        return False
    return math.exp(-(math.log(c_new) - math.log(c_cur)) / temp) >= rng.random()


class BestTracker:
    """The cheapest state seen and the iteration that found it; after
    `threshold` iterations without improvement the search restarts from it."""

    def __init__(self, start: SAState, threshold: int):
        self.best = start
        self.found = -1
        self.threshold = threshold

    def update(self, i: int, cur: SAState) -> SAState:
        if cur.cost < self.best.cost:
            self.best, self.found = cur, i
            return cur
        if i - self.found >= self.threshold:
            self.found = i
            return self.best
        return cur


class Progress:
    """Search progress t in [0, 1): iteration / budget when a budget is
    given (reproducible), else elapsed / time limit.  next() returns None once
    the search is over."""

    def __init__(self, iterations, time_limit):
        self.iterations, self.time_limit = iterations, time_limit
        self.i = -1
        self.start = time.monotonic()

    def next(self):
        if self.iterations is not None:
            if self.i + 1 >= self.iterations:
                return None
            t = (self.i + 1) / self.iterations
        else:
            elapsed = time.monotonic() - self.start
            if elapsed >= self.time_limit:
                return None
            t = elapsed / self.time_limit
        self.i += 1
        return t


def _worker_chain(args):
    ann, steps, state, temp, rng = args
    end = ann.do_steps(steps, state, temp, rng)
    return end, rng


def simulated_annealing(leaf_legs, dims, initial_partition_of, num_partitions,
                        cfg: SAConfig | None = None) -> Plan:
    cfg = cfg or SAConfig()
    ann = Annealer(leaf_legs, dims, num_partitions, cfg)
    init = ann.make_state(initial_partition_of, np.random.default_rng([cfg.seed, 0]))
    if cfg.parallel and cfg.workers > 1:
        # the workers' step chains in processes of their own (forked: no
        # program is started, the planner's state is copied)
        import multiprocessing
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(cfg.workers, mp_context=multiprocessing.get_context("fork")) as pool:
            best, history = ann.run(initial_partition_of, pool)
    else:
        best, history = ann.run(initial_partition_of)
    tree, roots = assemble_tree(len(leaf_legs), best.parts, best.red_pairs)
    meta = dict(method="sa-directed" if cfg.directed else "sa-naive", seed=cfg.seed,
                t0=cfg.t0, tf=cfg.tf, n_steps=cfg.n_steps, workers=cfg.workers,
                restart_threshold=cfg.restart_threshold, iterations=cfg.iterations,
                rg_samples=cfg.rg_samples, rg_temperature=cfg.rg_temperature,
                initial_con_dist=str(init.cost), con_dist=str(best.cost),
                evaluations=ann.evaluations)
    return Plan(best.partition_of, num_partitions, tree, meta)
