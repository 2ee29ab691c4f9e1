"""TN_FLAG_CONCURRENT (the partitions' subtrees side by side, one stream each,
then the cross-partition tree): every vertex computes the same values as in
the serial order, so results must be bit-identical to the plain path, and
within the FP32 amplitude bound of the oracle."""
import numpy as np
import pytest

import oracle
from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import (amplitude_network, amplitude_overrides, brickwork_circuit,
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


def _plan(net, k):
    return simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, k), k,
                               SAConfig(iterations=3, n_steps=16, workers=2, rg_samples=8, seed=1))


@pytest.mark.parametrize("family,k,open_q", [("brick16", 4, ()), ("rand14", 3, ()), ("rand18", 6, ()),
                                              ("rand12", 3, (0, 5)), ("brick12", 1, ())])
def test_concurrent_matches_serial(ctx, family, k, open_q):
    n = int(family[-2:])
    circ = brickwork_circuit(n, 10, 3) if family.startswith("brick") else random_circuit(n, 10, 5)
    net = amplitude_network(circ, 0, open_qubits=open_q)
    plan = _plan(net, k)
    p = ctx.load_network(net, plan.partition_of, k, plan.tree)
    shape = (2,) * len(open_q)
    for x in random_bitstrings(n, 4, 9):
        ovr = amplitude_overrides(net, circ, x, open_qubits=open_q)
        a, la = lib.tn_contract(p, ovr, shape)
        b, lb = lib.tn_contract(p, ovr, shape, flags=lib.TN_FLAG_CONCURRENT)
        assert np.array_equal(a, b) and la == lb, (family, x)
        # mantissa and scale kept apart: the same bits as well
        am, al2 = lib.tn_contract(p, ovr, shape, flags=lib.TN_FLAG_KEEP_SCALE)
        bm, bl2 = lib.tn_contract(p, ovr, shape, flags=lib.TN_FLAG_KEEP_SCALE | lib.TN_FLAG_CONCURRENT)
        assert np.array_equal(am, bm) and al2 == bl2
        ref = np.asarray(oracle.contract_tree(net.legs, net.dims, net.copy_with(ovr).tensors, plan.tree,
                                              output_legs=net.output_legs or ())).reshape(shape)
        floor = 2.0 ** (-n / 2)
        assert np.max(np.abs(b - ref)) / max(np.max(np.abs(ref)), floor) < TOL
    ctx.free_plan(p)


def test_concurrent_between_batches(ctx):
    """Concurrent single calls interleaved with batched calls on the same
    context and plan: the partition streams start after the context's stream
    and every result stays exact."""
    circ = random_circuit(14, 10, 7)
    net = amplitude_network(circ, 0)
    plan = _plan(net, 4)
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    xs = random_bitstrings(14, 12, 3)
    serial = [lib.tn_contract(p, amplitude_overrides(net, circ, x))[0] for x in xs]
    for rep in range(2):
        outs, _, st = lib.tn_contract_batch(ctx.handle, [(p, amplitude_overrides(net, circ, x)) for x in xs],
                                            [()] * len(xs))
        assert np.all(st == 0)
        for x, s_ in zip(xs, serial):
            c, _ = lib.tn_contract(p, amplitude_overrides(net, circ, x), flags=lib.TN_FLAG_CONCURRENT)
            assert np.array_equal(c, s_)
        for o, s_ in zip(outs, serial):
            assert abs(complex(np.asarray(o).reshape(-1)[0]) - complex(s_.reshape(-1)[0])) <= \
                2e-6 * max(abs(complex(s_.reshape(-1)[0])), 2.0 ** -7)
    ctx.free_plan(p)
