"""Three-term split-BF16 plans (4M and 3M) on every batched and served path.

A 26-qubit random circuit (depth 16, 6 CX pairs per layer, 4 SA partitions,
largest intermediate 2^20, nine GEMM vertices) runs through
tn_contract_batch, tn_contract_strided (pageable and pinned output),
TN_FLAG_GRAPH (capture, then replays with eager work in between, each replay
equal to the eager result) and serve (mixed with FP32 requests on another
plan).  Every result is held to the BF16x3 bound 1e-3 against the complex128
oracle (loop-nest contraction of the same network and tree) and to the same
bound against the same query run alone through tn_contract.  The 30-qubit
plan (largest intermediate 2^27) runs two queries through the batched and
strided calls against the stored state-vector amplitudes.

Amplitude error |a - a_ref| / max(|a_ref|, 2^(-n/2)).
"""
import json
import os
import time

import numpy as np
import pytest

import oracle
from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import (amplitude_network, amplitude_overrides, output_tensor_ids,
                                         random_bitstrings, random_circuit)
from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
from paper_2507_20667_amd.planner.plan import tree_partition
from paper_2507_20667_amd.planner.workloads import random30

pytestmark = pytest.mark.gpu
TOL = 1e-3
FORMS = {"4m": lib.TN_PREC_BF16X3 | lib.TN_FORM_4M, "3m": lib.TN_PREC_BF16X3 | lib.TN_FORM_3M}
GOLD = os.path.join(os.path.dirname(__file__), "golden", "config3_amplitudes.json")


def _c(x):
    return complex(np.asarray(x).reshape(-1)[0])


def err(a, ref, n):
    return abs(_c(a) - _c(ref)) / max(abs(_c(ref)), 2.0 ** (-n / 2))


@pytest.fixture(scope="module")
def setup():
    circ = random_circuit(26, 16, 3, cx_per_layer=6)
    net = amplitude_network(circ, 0)
    plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 4), 4,
                               SAConfig(iterations=4, n_steps=16, workers=2, rg_samples=8, seed=0))
    xs = random_bitstrings(circ.n, 6, 31)
    refs = [complex(oracle.contract_tree(net.legs, net.dims,
                                         net.copy_with(amplitude_overrides(net, circ, x)).tensors,
                                         plan.tree)) for x in xs]
    ctx = lib.Context(8 << 30)
    yield circ, net, plan, xs, refs, ctx
    ctx.close()


def _load(setup, form):
    circ, net, plan, xs, refs, ctx = setup
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree, FORMS[form])
    c = lib.tn_plan_costs_get(p)
    assert c["num_gemm_nodes"] >= 4 and c["largest_intermediate"] >= 1 << 20
    return p


def _alone(p, net, circ, x):
    return _c(lib.tn_contract(p, amplitude_overrides(net, circ, x))[0])


@pytest.mark.parametrize("form", ["4m", "3m"])
def test_bf16x3_batch(setup, form):
    circ, net, plan, xs, refs, ctx = setup
    p = _load(setup, form)
    outs, _, st = lib.tn_contract_batch(ctx.handle, [(p, amplitude_overrides(net, circ, x)) for x in xs],
                                        [()] * len(xs))
    assert np.all(st == 0)
    worst = 0.0
    for x, o, r in zip(xs, outs, refs):
        e = err(o, r, circ.n)
        worst = max(worst, e)
        assert e < TOL, (x, o, r)
        assert err(o, _alone(p, net, circ, x), circ.n) < TOL
    print(form, "batch max err", worst)
    ctx.free_plan(p)


@pytest.mark.parametrize("form", ["4m", "3m"])
@pytest.mark.parametrize("pinned", [False, True])
def test_bf16x3_strided(setup, form, pinned):
    import torch
    circ, net, plan, xs, refs, ctx = setup
    p = _load(setup, form)
    ids = output_tensor_ids(net)
    vec = {t: np.stack([amplitude_overrides(net, circ, x)[t] for x in xs]) for t in ids}
    ovr = [(t, vec[t].astype(np.complex128), 16 * vec[t].shape[1], lib.TN_C128) for t in ids]
    out = None
    if pinned:
        out = torch.zeros(len(xs), dtype=torch.complex128, pin_memory=True).numpy()
    got, _ = lib.tn_contract_strided(p, len(xs), ovr, out=out)
    batch, _, _ = lib.tn_contract_batch(ctx.handle, [(p, amplitude_overrides(net, circ, x)) for x in xs],
                                        [()] * len(xs))
    for i, r in enumerate(refs):
        assert err(got[i], r, circ.n) < TOL
        # the strided and the descriptor form run the same kernels
        assert abs(complex(got[i]) - _c(batch[i])) <= 1e-6 * max(abs(r), 2.0 ** (-circ.n / 2))
    ctx.free_plan(p)


@pytest.mark.parametrize("form", ["4m", "3m"])
def test_bf16x3_graph_replays(setup, form):
    """TN_FLAG_GRAPH: the first call captures; three replays, with eager
    calls on another plan in between, each give the eager result."""
    circ, net, plan, xs, refs, ctx = setup
    p = _load(setup, form)
    other = random_circuit(14, 8, 4)
    onet = amplitude_network(other, 0)
    opl = simulated_annealing(onet.legs, onet.dims, tree_partition(onet.legs, onet.dims, 2), 2,
                              SAConfig(iterations=2, n_steps=8, workers=2, rg_samples=4))
    op = ctx.load_network(onet, opl.partition_of, 2, opl.tree)
    qs = [(p, amplitude_overrides(net, circ, x)) for x in xs]
    eager, _, st = lib.tn_contract_batch(ctx.handle, qs, [()] * len(xs))
    assert np.all(st == 0)
    for rep in range(4):
        g, _, st = lib.tn_contract_batch(ctx.handle, qs, [()] * len(xs), flags=lib.TN_FLAG_GRAPH)
        assert np.all(st == 0)
        for i in range(len(xs)):
            assert _c(g[i]) == _c(eager[i]), (rep, i)
        lib.tn_contract_batch(ctx.handle, [(op, amplitude_overrides(onet, other, 5))], [()])
    for i, r in enumerate(refs):
        assert err(eager[i], r, circ.n) < TOL
    ctx.free_plan(op)
    ctx.free_plan(p)


def _wait(ctx, ticket, timeout=60.0):
    t0 = time.time()
    while True:
        st, out, l2, lat = lib.tn_serve_poll(ctx.handle, ticket)
        if st != lib.TN_PENDING:
            return st, out
        if time.time() - t0 > timeout:
            raise TimeoutError(f"ticket {ticket} still pending")
        time.sleep(0.0005)


def test_bf16x3_serve_mix(setup):
    """BF16x3 4M and 3M requests served in a mix with FP32 requests on another
    plan: each within 1e-3 of the oracle and of the query run alone."""
    circ, net, plan, xs, refs, ctx = setup
    p4, p3 = _load(setup, "4m"), _load(setup, "3m")
    other = random_circuit(16, 10, 8)
    onet = amplitude_network(other, 0)
    opl = simulated_annealing(onet.legs, onet.dims, tree_partition(onet.legs, onet.dims, 3), 3,
                              SAConfig(iterations=2, n_steps=8, workers=2, rg_samples=4))
    op = ctx.load_network(onet, opl.partition_of, 3, opl.tree)
    oxs = random_bitstrings(other.n, 8, 2)
    reqs = []
    for i in range(3):
        for k, x in enumerate(xs):
            reqs.append(("4m", p4, k, x))
            reqs.append(("3m", p3, k, x))
        for x in oxs:
            reqs.append(("fp32", op, None, x))
    order = np.random.default_rng(4).permutation(len(reqs))
    tickets = []
    for i in order:
        kind, p, k, x = reqs[i]
        n_, c_ = (net, circ) if kind != "fp32" else (onet, other)
        tickets.append((i, lib.tn_serve_submit(ctx.handle, p, amplitude_overrides(n_, c_, x))))
    for i, t in tickets:
        kind, p, k, x = reqs[i]
        st, out = _wait(ctx, t)
        assert st == lib.TN_OK
        if kind == "fp32":
            ref = complex(oracle.contract_tree(onet.legs, onet.dims,
                                               onet.copy_with(amplitude_overrides(onet, other, x)).tensors,
                                               opl.tree))
            assert err(out, ref, other.n) < 1e-5
        else:
            assert err(out, refs[k], circ.n) < TOL
            assert err(out, _alone(p, net, circ, x), circ.n) < TOL
    for q in (op, p4, p3):
        ctx.free_plan(q)


@pytest.fixture(scope="module")
def big():
    gold = json.load(open(GOLD))
    w = random30()
    assert gold["circuit"]["n"] == w.circ.n
    ctx = lib.Context(24 << 30)
    yield gold, w, ctx
    ctx.close()


@pytest.mark.parametrize("flags,tol", [(lib.TN_PREC_FP32, 1e-5), (FORMS["4m"], TOL), (FORMS["3m"], TOL)])
def test_random30_batched_two_queries(big, flags, tol):
    gold, w, ctx = big
    circ, net, plan = w.circ, w.net, w.plan
    p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 8, plan.tree, None, flags)
    xs = gold["bitstrings"][1:3]
    refs = [complex(*gold["amplitudes"][str(x)]) for x in xs]
    outs, _, st = lib.tn_contract_batch(ctx.handle, [(p, amplitude_overrides(net, circ, x)) for x in xs],
                                        [()] * len(xs))
    assert np.all(st == 0)
    ids = output_tensor_ids(net)
    vec = {t: np.stack([amplitude_overrides(net, circ, x)[t] for x in xs]) for t in ids}
    got, _ = lib.tn_contract_strided(p, len(xs), [(t, vec[t], 32, lib.TN_C128) for t in ids])
    for i, r in enumerate(refs):
        assert err(outs[i], r, circ.n) < tol, (xs[i], outs[i], r)
        assert err(got[i], r, circ.n) < tol
    ctx.free_plan(p)
