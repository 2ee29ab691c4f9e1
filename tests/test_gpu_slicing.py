"""Slicing through the library: the network with some legs fixed runs as one
batch (one query per slice) and the slices are added in FP64; the sum equals
the unsliced contraction (library and oracle), for a closed network and one
with open legs."""
import numpy as np
import pytest

import oracle
from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import amplitude_network, random_circuit
from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
from paper_2507_20667_amd.planner.cost import largest_intermediate
from paper_2507_20667_amd.planner.plan import tree_partition
from paper_2507_20667_amd.planner.slicing import choose_slices, contract_sliced, largest_after

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(4 << 30)
    yield c
    c.close()


@pytest.mark.parametrize("n,d,open_qubits", [(18, 10, ()), (14, 8, (0, 5))])
def test_sliced_equals_unsliced(ctx, n, d, open_qubits):
    circ = random_circuit(n, d, 7)
    net = amplitude_network(circ, 3, open_qubits=open_qubits)
    plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 4), 4,
                               SAConfig(iterations=3, n_steps=16, workers=2, rg_samples=4, seed=1))
    top = largest_intermediate(net.legs, net.dims, plan.tree)
    sl = choose_slices(net.legs, net.dims, plan.tree, max(top // 16, 2))
    assert sl and largest_after(net.legs, net.dims, plan.tree, sl) < top
    shape = (2,) * len(open_qubits)
    outs = net.output_legs or None
    p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 4, plan.tree, outs)
    full, _ = lib.tn_contract(p, result_shape=shape)
    ctx.free_plan(p)
    got = contract_sliced(lib, ctx, net.legs, net.dims, net.tensors, plan.partition_of, 4, plan.tree,
                          sl, output_legs=outs, result_shape=shape)
    ref = oracle.contract_tree(net.legs, net.dims, net.tensors, plan.tree, net.output_legs or ())
    scale = max(float(np.max(np.abs(ref))), 2.0 ** (-n / 2))
    assert np.max(np.abs(got - ref)) / scale < 1e-5
    assert np.max(np.abs(got - full)) / scale < 1e-5
