"""GPU parity of the batched path (tn_contract_batch): the subtree kernel that
runs whole small subtrees in one workgroup, shared subtrees computed once,
partial and device-resident overrides.  Each result is compared with the
oracle (amplitude error as in test_gpu_parity, bound 1e-5 for FP32) and with
the same query run alone through tn_contract."""
import numpy as np
import pytest

import oracle
from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import (amplitude_network, amplitude_overrides, basis_vec,
                                         brickwork_circuit, output_tensor_ids, phase_poly_circuit,
                                         random_bitstrings, random_circuit)
from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
from paper_2507_20667_amd.planner.plan import tree_partition

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(8 << 30)
    yield c
    c.close()


def _c(x):
    return complex(np.asarray(x).reshape(-1)[0])


def err(a, ref, n):
    return abs(_c(a) - _c(ref)) / max(abs(_c(ref)), 2.0 ** (-n / 2))


def _plan(net, k, iters=4):
    return simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, k), k,
                               SAConfig(iterations=iters, n_steps=16, workers=2, rg_samples=8))


def _ref(net, plan, ovr):
    return oracle.contract_tree(net.legs, net.dims, net.copy_with(ovr).tensors, plan.tree)


@pytest.mark.parametrize("family", ["brick20", "phase12", "rand16"])
def test_batch_against_oracle(ctx, family):
    if family == "brick20":
        circ = brickwork_circuit(20, 14, 0)
    elif family == "phase12":
        circ = phase_poly_circuit(12, 8, 2)
    else:
        circ = random_circuit(16, 10, 4)
    net = amplitude_network(circ, 0)
    plan = _plan(net, 4)
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    xs = random_bitstrings(circ.n, 48, 3)
    queries = [(p, amplitude_overrides(net, circ, x)) for x in xs]
    outs, _, st = lib.tn_contract_batch(ctx.handle, queries, [()] * len(xs))
    assert np.all(st == 0)
    worst = 0.0
    for x, o in zip(xs, outs):
        ovr = amplitude_overrides(net, circ, x)
        e = err(o, _ref(net, plan, ovr), circ.n)
        worst = max(worst, e)
        assert e < TOL, (x, o)
        alone, _ = lib.tn_contract(p, ovr)
        assert abs(_c(o) - _c(alone)) <= 2e-6 * max(abs(_c(alone)), 2.0 ** (-circ.n / 2))
    print(family, "max err", worst)
    ctx.free_plan(p)


def test_batch_partial_and_mixed_overrides(ctx):
    """Queries override different subsets of the output leaves; a leaf a query
    does not override keeps the plan's data."""
    circ = random_circuit(12, 8, 6)
    net = amplitude_network(circ, 0b101)        # built for bitstring 5
    plan = _plan(net, 3)
    p = ctx.load_network(net, plan.partition_of, 3, plan.tree)
    ids = output_tensor_ids(net)
    rng = np.random.default_rng(1)
    queries, refs = [], []
    for i in range(20):
        ovr = {}
        for q, t in enumerate(ids):
            if rng.random() < 0.4:
                ovr[t] = basis_vec(int(rng.integers(0, 2)))
        queries.append((p, ovr))
        refs.append(_ref(net, plan, ovr))
    outs, _, st = lib.tn_contract_batch(ctx.handle, queries, [()] * len(queries))
    assert np.all(st == 0)
    for o, r in zip(outs, refs):
        assert err(o, r, 12) < TOL
    ctx.free_plan(p)


@pytest.mark.parametrize("scattered", [False, True])
def test_batch_device_overrides(ctx, scattered):
    import torch
    circ = brickwork_circuit(14, 10, 5)
    net = amplitude_network(circ, 0)
    plan = _plan(net, 4)
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    ids = output_tensor_ids(net)
    n = circ.n
    xs = random_bitstrings(n, 32, 8)
    host = np.zeros((len(xs), n, 2), dtype=np.complex64)
    for qi, x in enumerate(xs):
        for q in range(n):
            host[qi, q, (x >> q) & 1] = 1
    dev = torch.from_numpy(host).to("cuda")
    order = list(range(len(xs)))
    if scattered:
        order = [int(i) for i in np.random.default_rng(0).permutation(len(xs))]
    base = dev.data_ptr()
    qarr = (lib.tn_query * len(xs))()
    keep = []
    for i, qi in enumerate(order):
        arr = (lib.tn_leaf * n)()
        for q, t in enumerate(ids):
            arr[q] = lib.tn_leaf(t, base + (qi * n + q) * 16, lib.TN_C64_DEVICE)
        keep.append(arr)
        import ctypes
        qarr[i] = lib.tn_query(p, n, ctypes.cast(arr, ctypes.c_void_p).value)
    import ctypes
    outs = np.zeros((len(xs), 2), dtype=np.float64)
    optrs = (ctypes.c_void_p * len(xs))(*[outs.ctypes.data + 16 * i for i in range(len(xs))])
    st = np.zeros(len(xs), dtype=np.int32)
    torch.cuda.synchronize()
    rc = lib.load().tn_contract_batch(ctypes.c_void_p(ctx.handle), len(xs),
                                      ctypes.cast(qarr, ctypes.c_void_p),
                                      ctypes.cast(optrs, ctypes.c_void_p), lib.TN_C128, None,
                                      st.ctypes.data_as(ctypes.c_void_p), 0)
    assert rc == 0, lib.tn_last_error()
    for i, qi in enumerate(order):
        ref = _ref(net, plan, amplitude_overrides(net, circ, xs[qi]))
        assert err(complex(outs[i, 0], outs[i, 1]), ref, n) < TOL
    ctx.free_plan(p)


def test_profile_counts_subtree_kernel(ctx):
    circ = brickwork_circuit(12, 8, 1)
    net = amplitude_network(circ, 0)
    plan = _plan(net, 2)
    p = ctx.load_network(net, plan.partition_of, 2, plan.tree)
    xs = random_bitstrings(12, 16, 2)
    lib.tn_profile_enable(ctx.handle, True)
    lib.tn_profile_read(ctx.handle, reset=True)
    lib.tn_contract_batch(ctx.handle, [(p, amplitude_overrides(net, circ, x)) for x in xs],
                          [()] * len(xs))
    stats = lib.tn_profile_read(ctx.handle, reset=True)
    lib.tn_profile_enable(ctx.handle, False)
    assert stats["tree"]["launches"] >= 1 and stats["tree"]["seconds"] > 0
    ctx.free_plan(p)
