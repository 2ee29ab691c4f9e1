"""30-qubit random circuit (depth 20, 7 CX pairs per layer, 70 % nearest-
neighbour), 8 partitions refined by simulated annealing, largest intermediate
2^27 complex64: amplitudes of the all-zero and 8 seeded bitstrings against the
oracle's state-vector values stored in tests/golden/config3_amplitudes.json
(written by tests/golden/make_config3_reference.py, which calls only the
oracle).  Bounds: 1e-5 (FP32), 1e-3 (three-term split BF16), on the amplitude
error |a - a_ref| / max(|a_ref|, 2^-15)."""
import json
import os
import time

import numpy as np
import pytest

from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import amplitude_network, amplitude_overrides, random_circuit
from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
from paper_2507_20667_amd.planner.plan import tree_partition

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "config3_amplitudes.json")


@pytest.fixture(scope="module")
def setup():
    gold = json.load(open(GOLD))
    c = gold["circuit"]
    circ = random_circuit(c["n"], c["depth"], c["seed"], cx_per_layer=c["cx_per_layer"],
                          p_nn=c["p_nn"])
    net = amplitude_network(circ, 0)
    plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 8), 8,
                               SAConfig(iterations=8, seed=0))
    ctx = lib.Context(16 << 30)
    yield gold, circ, net, plan, ctx
    ctx.close()


@pytest.mark.parametrize("flags,tol", [(lib.TN_PREC_FP32, 1e-5),
                                       (lib.TN_PREC_BF16X3 | lib.TN_FORM_4M, 1e-3),
                                       (lib.TN_PREC_BF16X3 | lib.TN_FORM_3M, 1e-3)])
def test_config3_amplitudes(setup, flags, tol):
    gold, circ, net, plan, ctx = setup
    p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 8, plan.tree, None, flags)
    costs = lib.tn_plan_costs_get(p)
    assert costs["largest_intermediate"] >= 1 << 26
    worst = 0.0
    t0 = time.time()
    for x in gold["bitstrings"]:
        got, _ = lib.tn_contract(p, amplitude_overrides(net, circ, x))
        ref = complex(*gold["amplitudes"][str(x)])
        e = abs(complex(np.asarray(got).reshape(-1)[0]) - ref) / max(abs(ref), 2.0 ** -15)
        worst = max(worst, e)
        assert e < tol, (x, got, ref, e)
    print(f"flags {flags}: {len(gold['bitstrings'])} amplitudes in {time.time() - t0:.2f} s, "
          f"max err {worst:.2e}, largest intermediate {costs['largest_intermediate']}, "
          f"con_serial {costs['con_serial']}")
    ctx.free_plan(p)


@pytest.mark.parametrize("flags,tol", [(lib.TN_PREC_FP32, 1e-5), (lib.TN_PREC_FP32 | lib.TN_FORM_3M, 1e-5),
                                       (lib.TN_PREC_BF16X3 | lib.TN_FORM_4M, 1e-3),
                                       (lib.TN_PREC_BF16X3 | lib.TN_FORM_3M, 1e-3)])
def test_fused_gemm_epilogue_bit_identical(setup, flags, tol, monkeypatch):
    """The plane GEMMs (FP32; BF16x3, whose producers write the four or six
    split bf16 planes) that write their parent's operand planes in their epilogue
    (the parent then reads them as they are and scales its result by the
    power of two instead) give the same bits as the permuted operands."""
    gold, circ, net, plan, ctx = setup
    perms, amps, batch = {}, {}, {}
    for fuse in ("0", "1"):
        monkeypatch.setenv("TN_GEMM_FUSE", fuse)
        p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 8, plan.tree, None, flags)
        perms[fuse] = lib.tn_plan_costs_get(p)["num_permutations"]
        amps[fuse] = np.array([np.asarray(lib.tn_contract(p, amplitude_overrides(net, circ, x))[0]).reshape(-1)[0]
                               for x in gold["bitstrings"]], dtype=np.complex128)
        if fuse == "1":
            # the fused plan with the partitions side by side (one stream
            # each): the same bits
            conc = np.array([np.asarray(lib.tn_contract(p, amplitude_overrides(net, circ, x),
                                                        flags=lib.TN_FLAG_CONCURRENT)[0]).reshape(-1)[0]
                             for x in gold["bitstrings"]], dtype=np.complex128)
            assert np.array_equal(conc.view(np.uint64), amps[fuse].view(np.uint64))
        # all the bitstrings as one batch (its small vertices in the subtree
        # kernel, the GEMMs batched over the queries)
        res, _, st = lib.tn_contract_batch(ctx.handle, [(p, amplitude_overrides(net, circ, x))
                                                        for x in gold["bitstrings"]],
                                           [()] * len(gold["bitstrings"]))
        assert all(v == 0 for v in st)
        batch[fuse] = np.array([complex(np.asarray(r).reshape(-1)[0]) for r in res], dtype=np.complex128)
        ctx.free_plan(p)
    assert perms["1"] < perms["0"], perms
    assert np.array_equal(amps["1"].view(np.uint64), amps["0"].view(np.uint64)), (amps["0"], amps["1"])
    assert np.array_equal(batch["1"].view(np.uint64), batch["0"].view(np.uint64)), (batch["0"], batch["1"])
    for i, x in enumerate(gold["bitstrings"]):
        ref = complex(*gold["amplitudes"][str(x)])
        assert abs(amps["1"][i] - ref) / max(abs(ref), 2.0 ** -15) < tol
        assert abs(batch["1"][i] - ref) / max(abs(ref), 2.0 ** -15) < tol
