"""Slicing through the library: the network with some legs fixed runs as one
batch (one query per slice) and the slices are added in FP64; the sum equals
the unsliced contraction (library and oracle), for a closed network and one
with open legs; the library's own choice of legs; overrides of tensors that
carry a sliced leg; an arena too small for the unsliced plan, in direct calls
and in serving."""
import ctypes
import time

import numpy as np
import pytest

import oracle
from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import (amplitude_network, amplitude_overrides, output_tensor_ids,
                                         random_bitstrings, random_circuit)
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


def _net20():
    circ = random_circuit(20, 20, 11)
    net = amplitude_network(circ, 0)
    plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 4), 4,
                               SAConfig(iterations=3, n_steps=16, workers=2, rg_samples=4, seed=1))
    return circ, net, plan


@pytest.fixture(scope="module")
def net20():
    circ, net, plan = _net20()
    return circ, net, plan, oracle.statevector(circ)


def test_keep_scale_and_auto_choice(ctx, net20):
    """The library's own choice of legs (max_intermediate) and the mantissa /
    scale form of the sliced result: mantissa * 2^scale is the plain result
    bit for bit (the scale is folded in by an exact power-of-two product)."""
    circ, net, plan, psi = net20
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    top = lib.tn_plan_costs_get(p)["largest_intermediate"]
    s = ctx.slice_plan(p, (), top // 16)
    assert lib.tn_plan_costs_get(s)["largest_intermediate"] <= top // 16
    plain, l0 = lib.tn_contract(s)
    mant, l2 = lib.tn_contract(s, flags=lib.TN_FLAG_KEEP_SCALE)
    assert l0 == 0.0
    assert complex(plain) == complex(mant) * 2.0 ** l2
    assert abs(complex(plain) - psi[0]) <= 1e-5 * max(abs(psi[0]), 2.0 ** -10)
    ctx.free_plan(s)
    ctx.free_plan(p)


def test_overrides_of_sliced_tensors(ctx, net20):
    """Overrides of tensors that carry a sliced leg (an output tensor's leg is
    sliced on purpose) are cut per slice on the host: every bitstring's
    amplitude matches the state vector."""
    circ, net, plan, psi = net20
    top = largest_intermediate(net.legs, net.dims, plan.tree)
    sl = choose_slices(net.legs, net.dims, plan.tree, top // 8)
    out_leg = net.legs[output_tensor_ids(net)[3]][0]
    if out_leg not in sl:
        sl = sl + [out_leg]
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    s = ctx.slice_plan(p, sl)
    for x in random_bitstrings(20, 6, 5):
        got, _ = lib.tn_contract(s, amplitude_overrides(net, circ, x))
        assert abs(complex(got) - psi[x]) <= 1e-5 * max(abs(psi[x]), 2.0 ** -10), x
    # device data for a tensor that carries a sliced leg is refused
    import torch
    dev = torch.zeros(2, dtype=torch.complex64, device="cuda")
    arr = (lib.tn_leaf * 1)(lib.tn_leaf(output_tensor_ids(net)[3], dev.data_ptr(), lib.TN_C64_DEVICE))
    out = np.zeros(1, dtype=np.complex128)
    st = lib.load().tn_contract(ctypes.c_void_p(s), 1, ctypes.cast(arr, ctypes.c_void_p),
                                out.ctypes.data, lib.TN_C128, None, 0)
    assert st == lib.TN_E_INVALID_ARG
    ctx.free_plan(s)
    ctx.free_plan(p)


def test_small_arena_needs_slices(net20):
    """An arena smaller than one query's workspace: the plain plan fails with
    TN_E_NOMEM, the sliced plan runs (its slices in chunks that fit) and
    serving slices such a request by itself; all results match the state
    vector."""
    circ, net, plan, psi = net20
    xs = random_bitstrings(20, 4, 9)
    with lib.Context(4 << 20) as c:
        p = c.load_network(net, plan.partition_of, 4, plan.tree)
        costs = lib.tn_plan_costs_get(p)
        assert costs["live_peak_bytes"] > 4 << 20
        with pytest.raises(lib.TnError) as e:
            lib.tn_contract(p)
        assert e.value.status == lib.TN_E_NOMEM
        s = c.slice_plan(p, (), costs["largest_intermediate"] // 16)
        for x in xs[:2]:
            got, _ = lib.tn_contract(s, amplitude_overrides(net, circ, x))
            assert abs(complex(got) - psi[x]) <= 1e-5 * max(abs(psi[x]), 2.0 ** -10), x
        c.free_plan(s)
        tickets = [lib.tn_serve_submit(c.handle, p, amplitude_overrides(net, circ, x)) for x in xs]
        for t, x in zip(tickets, xs):
            t0 = time.time()
            while True:
                st, out, _, _ = lib.tn_serve_poll(c.handle, t)
                if st != lib.TN_PENDING:
                    break
                assert time.time() - t0 < 60
                time.sleep(0.001)
            assert st == lib.TN_OK
            assert abs(complex(out) - psi[x]) <= 1e-5 * max(abs(psi[x]), 2.0 ** -10), x
        c.free_plan(p)
