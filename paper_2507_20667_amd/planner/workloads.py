"""The seeded workloads the benchmark and the tests share: circuit, network
and simulated-annealing plan, built the same way everywhere.

  * brickwork20: 20-qubit brickwork circuit of depth 14 (seed 0), closed
    single-amplitude networks, 4 partitions refined by SA from the tree split;
  * random30: 30-qubit random circuit of depth 20 (seed 0, 7 CX pairs per
    layer, 70 % nearest-neighbour), closed single-amplitude networks, 8
    partitions refined by SA (largest intermediate 2^27 complex64);
  * uneven_mix: 64 random-family circuits of 12-26 qubits and depth 8-20
    (floor(n/4) CX pairs per layer), 4 SA partitions each, and 512 queries
    whose circuit follows a truncated Zipf(1.2) law (bitstrings uniform).

Plans are deterministic in (seed, iteration budget).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from ..inputs import amplitude_network, brickwork_circuit, circuit_mix, random_circuit, zipf_indices
from .cost import largest_intermediate
from .plan import Plan, tree_partition
from .sa import SAConfig, simulated_annealing

RANDOM30 = {"family": "random_circuit", "n": 30, "depth": 20, "seed": 0, "cx_per_layer": 7, "p_nn": 0.7}


@dataclass
class Workload:
    name: str
    circ: object
    net: object
    plan: Plan
    num_partitions: int
    planning_s: float


def brickwork20() -> Workload:
    circ = brickwork_circuit(20, 14, 0)
    net = amplitude_network(circ, 0)
    t0 = time.perf_counter()
    plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 4), 4,
                               SAConfig(iterations=20, n_steps=32, workers=4, rg_samples=8, seed=0))
    return Workload("brickwork 20 qubits depth 14 seed 0, single-amplitude networks, 4 SA partitions",
                    circ, net, plan, 4, time.perf_counter() - t0)


def random30() -> Workload:
    c = RANDOM30
    circ = random_circuit(c["n"], c["depth"], c["seed"], cx_per_layer=c["cx_per_layer"], p_nn=c["p_nn"])
    net = amplitude_network(circ, 0)
    t0 = time.perf_counter()
    plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 8), 8,
                               SAConfig(iterations=8, seed=0))
    return Workload(f"random circuit {c['n']} qubits depth {c['depth']} seed {c['seed']}, "
                    f"{c['cx_per_layer']} CX pairs per layer (p_nn {c['p_nn']}), single-amplitude "
                    "networks, 8 SA partitions", circ, net, plan, 8, time.perf_counter() - t0)


def uneven_mix(queries=512):
    """(circuits [(circ, net, plan)], query circuit indices, bitstrings,
    planning seconds).  A seed is skipped when the planned largest
    intermediate leaves [2^4, 2^24]."""
    t0 = time.perf_counter()
    circs, seed = [], 0
    while len(circs) < 64:
        (s, circ), = circuit_mix(1, seed)
        seed += 1
        net = amplitude_network(circ, 0)
        plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 4), 4,
                                   SAConfig(iterations=4, n_steps=16, workers=2, rg_samples=4, seed=s))
        li = largest_intermediate(net.legs, net.dims, plan.tree)
        if li > 1 << 24 or li < 1 << 4:
            continue
        circs.append((circ, net, plan))
    idx = zipf_indices(len(circs), queries, 1.2, 7)
    rng = np.random.default_rng(8)
    bits = [int(rng.integers(0, 1 << circs[i][0].n)) for i in idx]
    return circs, idx, bits, time.perf_counter() - t0
