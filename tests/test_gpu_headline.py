"""The benchmark's 20-qubit launch shape itself, checked result by result.

The brickwork workload (20 qubits, depth 14, 4 SA partitions) runs 4096
amplitude queries in one tn_contract_strided call, the way the benchmark
times it: the output basis vectors read in place from one device buffer,
four queries per workgroup of the batch subtree kernel, spilled
intermediates at per-query offsets across the whole workspace, and the
complex128 results written by the kernel straight into pinned host memory.
Every one of the 4096 results is compared with the oracle's state vector
(a 2^20 complex128 vector, the independent gate-by-gate algorithm), and 16
of them also with the loop-nest contraction of the same network and tree.

The graph-state variant (H on every qubit, then the brickwork's CZ bricks)
runs the same shape against the exact closed form 2^(-n/2) (-1)^(sum over
edges of x_i x_j), which pins the CZ convention end to end.

Amplitude error |a - a_ref| / max(|a_ref|, 2^(-n/2)), bound 1e-5 (FP32).
"""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import (amplitude_network, amplitude_overrides, brick_edges,
                                         graph_state_circuit, output_tensor_ids, random_bitstrings)
from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
from paper_2507_20667_amd.planner.plan import tree_partition
from paper_2507_20667_amd.planner.workloads import brickwork20

pytestmark = pytest.mark.gpu
TOL = 1e-5
Q = 4096


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(16 << 30)
    yield c
    c.close()


def _device_basis(torch, n, xs):
    """(Q, n, 2) complex64 basis vectors on the device, qubit q of query i at
    [i, q]."""
    bits = np.array([[(x >> q) & 1 for q in range(n)] for x in xs], dtype=np.int64)
    host = np.zeros((len(xs), n, 2), dtype=np.complex64)
    host[np.arange(len(xs))[:, None], np.arange(n)[None, :], bits] = 1.0
    return torch.from_numpy(host).to("cuda")


def _strided_pinned(torch, plan_handle, net, n, dev):
    """One tn_contract_strided call over the device basis vectors, results
    into a pinned complex128 array (the kernel writes them itself)."""
    ids = output_tensor_ids(net)
    base = dev.data_ptr()
    ovr = [(t, base + i * 16, n * 16, lib.TN_C64_DEVICE) for i, t in enumerate(ids)]
    out_t = torch.zeros((dev.shape[0], 2), dtype=torch.float64, pin_memory=True)
    out = out_t.numpy().view(np.complex128).reshape(dev.shape[0])
    res, _ = lib.tn_contract_strided(plan_handle, dev.shape[0], ovr, out=out, scales=False)
    torch.cuda.synchronize()
    return np.array(res), out_t


def _err(got, ref, n):
    return np.abs(got - ref) / np.maximum(np.abs(ref), 2.0 ** (-n / 2))


def test_headline_shape_every_result(ctx):
    import torch
    w = brickwork20()
    circ, net, plan, n = w.circ, w.net, w.plan, w.circ.n
    p = ctx.load_network(net, plan.partition_of, w.num_partitions, plan.tree)
    xs = random_bitstrings(n, Q, 1000)          # the benchmark's first step
    print(f"headline shape: {Q} queries, plan con_serial {lib.tn_plan_costs_get(p)['con_serial']}",
          flush=True)
    dev = _device_basis(torch, n, xs)
    got, keep = _strided_pinned(torch, p, net, n, dev)
    psi = oracle.statevector(circ)
    ref = psi[np.array(xs, dtype=np.int64)]
    e = _err(got, ref, n)
    print(f"max error over {Q} results {e.max():.2e} (worst query {int(e.argmax())})")
    assert e.max() < TOL, (int(e.argmax()), got[e.argmax()], ref[e.argmax()])
    # the loop-nest contraction of the same network and tree on a sample,
    # spread over the whole launch (first, last and evenly between)
    for qi in sorted(set([0, Q - 1] + list(range(0, Q, Q // 14)))):
        ovr = amplitude_overrides(net, circ, xs[qi])
        r = complex(oracle.contract_tree(net.legs, net.dims, net.copy_with(ovr).tensors, plan.tree))
        assert abs(r - ref[qi]) < 1e-12
        assert _err(got[qi], r, n) < TOL
    # a second call on the same buffers returns the same values (nothing
    # left over from the first call changes them)
    got2, _ = _strided_pinned(torch, p, net, n, dev)
    assert np.array_equal(got, got2)
    ctx.free_plan(p)


def test_headline_shape_graph_state_closed_form(ctx):
    """H layer + the brickwork's 7 CZ layers on 20 qubits: every one of 4096
    amplitudes is the exact closed form."""
    import torch
    n = 20
    circ = graph_state_circuit(n, brick_edges(n, 7))
    net = amplitude_network(circ, 0)
    plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 4), 4,
                               SAConfig(iterations=6, n_steps=16, workers=2, rg_samples=4, seed=0))
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    xs = random_bitstrings(n, Q, 77)
    dev = _device_basis(torch, n, xs)
    got, keep = _strided_pinned(torch, p, net, n, dev)
    ref = np.array([cf.graph_state_amplitude(circ, x) for x in xs])
    e = _err(got, ref, n)
    print(f"graph state: max error over {Q} results {e.max():.2e}")
    assert e.max() < TOL
    # both signs occur among the queries
    assert (ref > 0).any() and (ref < 0).any()
    ctx.free_plan(p)


def test_headline_shape_batch_descriptors(ctx):
    """The same 4096 queries through tn_contract_batch (one descriptor per
    query and leaf, device-resident overrides) agree with the strided call."""
    import torch
    w = brickwork20()
    circ, net, plan, n = w.circ, w.net, w.plan, w.circ.n
    p = ctx.load_network(net, plan.partition_of, w.num_partitions, plan.tree)
    xs = random_bitstrings(n, Q, 1001)
    dev = _device_basis(torch, n, xs)
    got, keep = _strided_pinned(torch, p, net, n, dev)
    ids = output_tensor_ids(net)
    base = dev.data_ptr()
    qarr = (lib.tn_query * Q)()
    leaves = []
    for qi in range(Q):
        arr = (lib.tn_leaf * n)()
        for i, t in enumerate(ids):
            arr[i] = lib.tn_leaf(t, base + (qi * n + i) * 16, lib.TN_C64_DEVICE)
        leaves.append(arr)
        qarr[qi] = lib.tn_query(p, n, ctypes.cast(arr, ctypes.c_void_p).value)
    outs = np.zeros(Q, dtype=np.complex128)
    optrs = (ctypes.c_void_p * Q)(*[outs.ctypes.data + 16 * i for i in range(Q)])
    st = np.zeros(Q, dtype=np.int32)
    rc = lib.load().tn_contract_batch(ctypes.c_void_p(ctx.handle), Q, ctypes.cast(qarr, ctypes.c_void_p),
                                      ctypes.cast(optrs, ctypes.c_void_p), lib.TN_C128, None,
                                      st.ctypes.data_as(ctypes.c_void_p), 0)
    assert rc == 0, lib.tn_last_error()
    assert np.all(st == 0)
    psi = oracle.statevector(circ)
    ref = psi[np.array(xs, dtype=np.int64)]
    assert _err(outs, ref, n).max() < TOL
    assert np.max(np.abs(outs - got)) <= 1e-6 * 2.0 ** (-n / 2)
    ctx.free_plan(p)


def test_gate_chains_bit_identical(ctx, monkeypatch):
    """The batch kernel runs the brickwork's 31-gate chain as one kind 5 step
    (the running tensor in registers, X terms exchanged between lanes); with
    TN_TREE_CHAIN=0 it runs the same gates as separate kind 4 steps through
    LDS.  Both give the same 4096 results bit for bit, and the state vector's
    within the FP32 bound."""
    import torch
    w = brickwork20()
    circ, net, plan, n = w.circ, w.net, w.plan, w.circ.n
    xs = random_bitstrings(n, Q, 1002)
    dev = _device_basis(torch, n, xs)
    p = ctx.load_network(net, plan.partition_of, w.num_partitions, plan.tree)
    chained, _ = _strided_pinned(torch, p, net, n, dev)
    ctx.free_plan(p)
    monkeypatch.setenv("TN_TREE_CHAIN", "0")
    p = ctx.load_network(net, plan.partition_of, w.num_partitions, plan.tree)
    plain, _ = _strided_pinned(torch, p, net, n, dev)
    ctx.free_plan(p)
    assert np.array_equal(chained, plain)
    psi = oracle.statevector(circ)
    ref = psi[np.array(xs, dtype=np.int64)]
    assert _err(chained, ref, n).max() < TOL


@pytest.mark.parametrize("qw", [None, "8"])
def test_kind3_pair_bit_identical(ctx, monkeypatch, qw):
    """The batch kernel fuses the brickwork's kind 3 pair (a 1024-entry
    intermediate written to the query's device workspace and read back by the
    step that contracts it with a two-leg operand) into one kind 6 step that
    keeps the intermediate in registers; with TN_TREE_PAIR=0 the two steps run
    apart.  Both give the same 4096 results bit for bit, and the state
    vector's within the FP32 bound.  With eight queries per workgroup (two per
    wave) the kind 6 step runs as its two kind 3 steps."""
    import torch
    if qw:
        monkeypatch.setenv("TN_TREE_QW", qw)
    w = brickwork20()
    circ, net, plan, n = w.circ, w.net, w.plan, w.circ.n
    xs = random_bitstrings(n, Q, 1003)
    dev = _device_basis(torch, n, xs)
    p = ctx.load_network(net, plan.partition_of, w.num_partitions, plan.tree)
    paired, _ = _strided_pinned(torch, p, net, n, dev)
    ctx.free_plan(p)
    monkeypatch.setenv("TN_TREE_PAIR", "0")
    p = ctx.load_network(net, plan.partition_of, w.num_partitions, plan.tree)
    plain, _ = _strided_pinned(torch, p, net, n, dev)
    ctx.free_plan(p)
    assert np.array_equal(paired, plain)
    psi = oracle.statevector(circ)
    ref = psi[np.array(xs, dtype=np.int64)]
    assert _err(paired, ref, n).max() < TOL
