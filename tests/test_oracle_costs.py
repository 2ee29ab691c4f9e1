"""Pins of the cost recomputation (oracle_costs, 128-bit integers).

  * hand-worked values of eq. con_serial, con_par, con_dist and mem on the
    networks in tests/golden/cost_worked_examples.json;
  * invariants that follow from the definitions: con_par <= con_dist <=
    con_serial; one partition gives con_dist = con_serial; all-singleton
    partitions give con_dist = con_par; mem <= 3 * largest tensor;
  * rejection of a tree that does not accept the partitioning (Section 2.4)
    and of an integer overflow past 128 bits;
  * bit-exact agreement with the planner's Python-integer cost model on plans
    of every circuit family (two independent implementations).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2507_20667_amd.inputs import (amplitude_network, brickwork_circuit, phase_poly_circuit,
                                         random_circuit, zz_network)
from paper_2507_20667_amd.planner import cost, contiguous_partition, plan_from_partition
from paper_2507_20667_amd.planner.plan import tree_partition

GOLD = os.path.join(os.path.dirname(__file__), "golden", "cost_worked_examples.json")


def _example(ex):
    names = sorted(ex["dims"])
    lab = {n: i for i, n in enumerate(names)}
    legs = [[lab[x] for x in l] for l in ex["legs"]]
    dims = {lab[k]: v for k, v in ex["dims"].items()}
    return legs, dims, [tuple(p) for p in ex["tree"]]


@pytest.mark.parametrize("idx", [0, 1])
def test_worked_examples(idx):
    ex = json.load(open(GOLD))["examples"][idx]
    legs, dims, tree = _example(ex)
    for case in ex["con_dist"]:
        got = oracle.costs(legs, dims, tree, case["partition_of"], case["k"])
        assert got["con_serial"] == ex["con_serial"]
        assert got["con_par"] == ex["con_par"]
        assert got["mem"] == ex["mem"]
        assert got["largest_intermediate"] == ex["largest_intermediate"]
        assert got["con_dist"] == case["value"], case["why"]
        # the planner's model, written separately, gives the same integers
        py = cost.all_costs(legs, dims, tree, case["partition_of"], case["k"])
        assert py["con_dist"] == case["value"]
        assert py["con_serial"] == ex["con_serial"] and py["con_par"] == ex["con_par"]
        assert py["mem"] == ex["mem"]


def test_tree_must_accept_partitioning():
    ex = json.load(open(GOLD))["examples"][0]
    legs, dims, tree = _example(ex)
    with pytest.raises(RuntimeError):
        oracle.costs(legs, dims, tree, [0, 1, 0, 1], 2)   # {v0,v2} is no subtree
    with pytest.raises(RuntimeError):
        oracle.costs(legs, dims, tree, [0, 0, 0, 0], 2)   # partition 1 empty


def test_overflow_is_reported():
    # 40 legs of dimension 2^4 on one bound pair: 2^160 > 2^128
    legs = [list(range(40)), list(range(40))]
    dims = {i: 16 for i in range(40)}
    with pytest.raises(RuntimeError):
        oracle.costs(legs, dims, [(0, 1)], [0, 0], 1)


def _networks():
    yield amplitude_network(phase_poly_circuit(10, 10, 0), 0), 2
    yield amplitude_network(brickwork_circuit(12, 8, 1), 0), 4
    yield amplitude_network(random_circuit(14, 10, 2), 0), 4
    yield zz_network(random_circuit(12, 8, 3), 2, 9), 3


def test_planner_and_oracle_agree_bit_exact():
    for net, k in _networks():
        for part in (contiguous_partition(net.num_tensors, k), tree_partition(net.legs, net.dims, k)):
            plan = plan_from_partition(net.legs, net.dims, part, k)
            a = oracle.costs(net.legs, net.dims, plan.tree, plan.partition_of, k)
            b = cost.all_costs(net.legs, net.dims, plan.tree, plan.partition_of, k)
            assert a == b
            assert b["con_par"] <= b["con_dist"] <= b["con_serial"]
            assert b["mem"] <= 3 * max(b["largest_intermediate"], 16)
            one = oracle.costs(net.legs, net.dims, plan.tree, [0] * net.num_tensors, 1)
            assert one["con_dist"] == one["con_serial"]


def test_singletons_recover_con_par_and_par_variant():
    net = amplitude_network(random_circuit(10, 6, 5), 0)
    plan = plan_from_partition(net.legs, net.dims, [0] * net.num_tensors, 1)
    nv = net.num_tensors
    got = oracle.costs(net.legs, net.dims, plan.tree, list(range(nv)), nv)
    assert got["con_dist"] == got["con_par"]
    # with con = con_par inside con_dist, any accepted partitioning gives con_par
    # (stated after eq. con_dist for comm = 0)
    k = 4
    part = tree_partition(net.legs, net.dims, k)
    p2 = plan_from_partition(net.legs, net.dims, part, k)
    assert cost.con_dist(net.legs, net.dims, p2.tree, p2.partition_of, k, con="par") == \
        cost.con_par(net.legs, net.dims, p2.tree)
