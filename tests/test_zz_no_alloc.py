"""tn_contract_strided_noalloc: the strided call with its workspace in the
static scratch array and its results written to device memory, checked
against tn_contract_strided on the same queries (the same kernels: equal
values) on two calls in a row, the second with fewer queries, for a plan
whose closed root runs in the subtree kernel (20-qubit brickwork) and one
whose closed root is a separate FP64 inner product (a 26-qubit circuit with
GEMM vertices); also against the state vector.  Sizes beyond the scratch
and host overrides are refused with clear errors."""
import numpy as np
import pytest

import oracle
from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import (amplitude_network, output_tensor_ids, random_bitstrings,
                                         random_circuit)
from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
from paper_2507_20667_amd.planner.plan import tree_partition
from paper_2507_20667_amd.planner.workloads import brickwork20

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(8 << 30)
    yield c
    c.close()


def _basis(torch, n, xs):
    bits = np.array([[(x >> q) & 1 for q in range(n)] for x in xs], dtype=np.int64)
    host = np.zeros((len(xs), n, 2), dtype=np.complex64)
    host[np.arange(len(xs))[:, None], np.arange(n)[None, :], bits] = 1.0
    return torch.from_numpy(host).to("cuda")


def _ovr(net, n, dev):
    ids = output_tensor_ids(net)
    return [(t, dev.data_ptr() + i * 16, n * 16) for i, t in enumerate(ids)]


def _strided(p, net, n, dev):
    ovr = [(t, a, s, lib.TN_C64_DEVICE) for t, a, s in _ovr(net, n, dev)]
    got, _ = lib.tn_contract_strided(p, dev.shape[0], ovr, scales=False)
    return np.array(got)


def _noalloc(torch, p, net, n, dev, out_stride=1):
    Q = dev.shape[0]
    out = torch.full((Q * out_stride,), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    lib.tn_contract_strided_noalloc(p, Q, _ovr(net, n, dev), out.data_ptr(), out_stride)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    if out_stride > 1:
        # the elements between results are left alone
        assert np.all(np.isnan(host.reshape(Q, out_stride)[:, 1:].real))
    return host[::out_stride]


def test_noalloc_matches_strided_subtree_root(ctx):
    import torch
    w = brickwork20()
    circ, net, plan, n = w.circ, w.net, w.plan, w.circ.n
    p = ctx.load_network(net, plan.partition_of, w.num_partitions, plan.tree)
    psi = oracle.statevector(circ)
    for Q, seed, ostride in ((512, 5, 1), (100, 6, 3)):   # the second call smaller
        xs = random_bitstrings(n, Q, seed)
        dev = _basis(torch, n, xs)
        ref = _strided(p, net, n, dev)
        got = _noalloc(torch, p, net, n, dev, ostride)
        assert np.array_equal(got, ref), np.max(np.abs(got - ref))
        exact = psi[np.array(xs, dtype=np.int64)]
        assert np.max(np.abs(got - exact) / np.maximum(np.abs(exact), 2.0 ** -10)) < 1e-5
    ctx.free_plan(p)


def test_noalloc_matches_strided_dot_root(ctx):
    import torch
    circ = random_circuit(26, 16, 3, cx_per_layer=6)
    net = amplitude_network(circ, 0)
    plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 4), 4,
                               SAConfig(iterations=4, n_steps=16, workers=2, rg_samples=8, seed=0))
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    n = circ.n
    for Q, seed in ((2, 1), (1, 2)):   # about 22 MB of workspace per query
        xs = random_bitstrings(n, Q, seed)
        dev = _basis(torch, n, xs)
        ref = _strided(p, net, n, dev)
        got = _noalloc(torch, p, net, n, dev)
        assert np.array_equal(got, ref), np.max(np.abs(got - ref))
    ctx.free_plan(p)


def test_noalloc_refusals(ctx):
    import torch
    w = brickwork20()
    net, plan, n = w.net, w.plan, w.circ.n
    p = ctx.load_network(net, plan.partition_of, w.num_partitions, plan.tree)
    dev = _basis(torch, n, random_bitstrings(n, 8, 1))
    out = torch.zeros(200000, dtype=torch.complex128, device="cuda")
    # the subtree programs are not on the device before a first strided call
    with pytest.raises(lib.TnError) as e:
        lib.tn_contract_strided_noalloc(p, 8, _ovr(net, n, dev), out.data_ptr())
    assert e.value.status == lib.TN_E_INVALID_ARG and "tn_contract_strided once" in str(e.value)
    _strided(p, net, n, dev)
    # more queries than the 64 MiB scratch holds
    big = _basis(torch, n, random_bitstrings(n, 200000, 2))
    with pytest.raises(lib.TnError) as e:
        lib.tn_contract_strided_noalloc(p, 200000, _ovr(net, n, big), out.data_ptr())
    assert e.value.status == lib.TN_E_NOMEM and "static scratch" in str(e.value)
    # host override data cannot be read in place
    arr = (lib.tn_leaf * n)()
    strides = (lib.ctypes.c_int64 * n)()
    host = np.zeros((8, n, 2), dtype=np.complex64)
    for i, t in enumerate(output_tensor_ids(net)):
        arr[i] = lib.tn_leaf(t, host.ctypes.data + i * 16, lib.TN_C64)
        strides[i] = n * 16
    rc = lib.load().tn_contract_strided_noalloc(lib.ctypes.c_void_p(p), 8, n,
                                                lib.ctypes.cast(arr, lib.ctypes.c_void_p),
                                                lib.ctypes.cast(strides, lib.ctypes.c_void_p),
                                                lib.ctypes.c_void_p(out.data_ptr()),
                                                lib.ctypes.c_int64(1), 0)
    assert rc == lib.TN_E_INVALID_ARG and "TN_C64_DEVICE" in lib.tn_last_error()
    ctx.free_plan(p)
