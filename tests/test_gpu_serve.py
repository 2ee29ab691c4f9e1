"""Serving (tn_serve_submit / tn_serve_poll): continuous batching on the GPU.

  * every result equals the same query run alone (tn_contract) within the
    FP32 bound, whether it ran in a mix of requests on several plans or not,
    and matches the oracle;
  * requests submitted from several threads while others run all complete;
  * a ticket is consumed by the poll that returns its result; unknown tickets
    are reported; a plan with pending requests cannot be freed;
  * a request whose workspace cannot fit the arena fails alone with
    TN_E_NOMEM.
"""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import (amplitude_network, amplitude_overrides, brickwork_circuit,
                                         random_bitstrings, random_circuit, zz_network)
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


def _plan(net, k):
    return simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, k), k,
                               SAConfig(iterations=3, n_steps=8, workers=2, rg_samples=4))


def _wait(ctx, ticket, timeout=60.0):
    t0 = time.time()
    while True:
        st, out, l2, lat = lib.tn_serve_poll(ctx.handle, ticket)
        if st != lib.TN_PENDING:
            return st, out, lat
        if time.time() - t0 > timeout:
            raise TimeoutError(f"ticket {ticket} still pending")
        time.sleep(0.0005)


def test_serve_mix_equals_alone(ctx):
    circs = [random_circuit(12, 8, 1), brickwork_circuit(14, 10, 2), random_circuit(16, 8, 3)]
    plans, nets = [], []
    for c in circs:
        net = amplitude_network(c, 0)
        pl = _plan(net, 3)
        plans.append((ctx.load_network(net, pl.partition_of, 3, pl.tree), pl))
        nets.append(net)
    zc = random_circuit(12, 6, 9)
    znet = zz_network(zc, 2, 7)
    zpl = _plan(znet, 2)
    zp = ctx.load_network(znet, zpl.partition_of, 2, zpl.tree)
    rng = np.random.default_rng(0)
    reqs = []
    for i in range(96):
        k = int(rng.integers(0, 4))
        if k == 3:
            reqs.append((zp, {}, None, None))
        else:
            x = int(rng.integers(0, 1 << circs[k].n))
            reqs.append((plans[k][0], amplitude_overrides(nets[k], circs[k], x), k, x))
    tickets = []
    for p, ovr, _, _ in reqs:
        tickets.append(lib.tn_serve_submit(ctx.handle, p, ovr))
        if rng.random() < 0.3:
            time.sleep(0.0002)          # arrivals spread over time
    lats = []
    for t, (p, ovr, k, x) in zip(tickets, reqs):
        st, out, lat = _wait(ctx, t)
        assert st == lib.TN_OK
        lats.append(lat)
        alone, _ = lib.tn_contract(p, ovr)
        n = circs[k].n if k is not None else 12
        assert abs(_c(out) - _c(alone)) <= TOL * max(abs(_c(alone)), 2.0 ** (-n / 2))
        if k is None:
            ref = oracle.contract_tree(znet.legs, znet.dims, znet.tensors, zpl.tree)
            assert abs(_c(out) - complex(ref)) < 1e-5
        elif t % 8 == 0:
            ref = oracle.contract_tree(nets[k].legs, nets[k].dims,
                                       nets[k].copy_with(ovr).tensors, plans[k][1].tree)
            assert abs(_c(out) - complex(ref)) <= TOL * max(abs(complex(ref)), 2.0 ** (-n / 2))
    assert all(l > 0 for l in lats)
    print("latency p50 %.3f ms p99 %.3f ms" % (1e3 * np.percentile(lats, 50),
                                               1e3 * np.percentile(lats, 99)))
    for p, _ in plans:
        ctx.free_plan(p)
    ctx.free_plan(zp)


def test_serve_threads_and_tickets(ctx):
    circ = random_circuit(14, 8, 5)
    net = amplitude_network(circ, 0)
    pl = _plan(net, 2)
    p = ctx.load_network(net, pl.partition_of, 2, pl.tree)
    xs = random_bitstrings(14, 64, 4)
    tickets = [None] * len(xs)

    def submit(lo, hi):
        for i in range(lo, hi):
            tickets[i] = lib.tn_serve_submit(ctx.handle, p, amplitude_overrides(net, circ, xs[i]))

    th = [threading.Thread(target=submit, args=(i * 16, i * 16 + 16)) for i in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert len(set(tickets)) == len(xs)
    # a plan with pending requests cannot be freed (or every request finished already)
    try:
        lib.tn_plan_free(p)
        freed = True
    except lib.TnError as e:
        assert e.status == lib.TN_E_INVALID_ARG
        freed = False
    for i, t in enumerate(tickets):
        st, out, _ = _wait(ctx, t)
        assert st == lib.TN_OK
        alone, _ = lib.tn_contract(p, amplitude_overrides(net, circ, xs[i])) if not freed else (out, 0)
        assert abs(_c(out) - _c(alone)) <= TOL * max(abs(_c(alone)), 2.0 ** -7)
    with pytest.raises(lib.TnError) as e:
        lib.tn_serve_poll(ctx.handle, tickets[0])
    assert e.value.status == lib.TN_E_UNKNOWN_TICKET
    with pytest.raises(lib.TnError):
        lib.tn_serve_poll(ctx.handle, 10 ** 12)
    if not freed:
        ctx.free_plan(p)
    else:
        ctx.plans.remove(p)


def test_serve_request_too_big_fails_alone():
    """An arena that holds the small plan's requests but not one request of the
    big plan: the big one ends TN_E_NOMEM, the small ones succeed."""
    with lib.Context(24 << 20) as c:
        small = random_circuit(10, 6, 2)
        snet = amplitude_network(small, 0)
        spl = _plan(snet, 2)
        sp = c.load_network(snet, spl.partition_of, 2, spl.tree)
        # a two-tensor network whose one result needs 64 MiB
        A = np.ones((2048, 16), dtype=np.complex128)
        B = np.ones((16, 2048), dtype=np.complex128)
        bp = c.plan_load([[1, 2], [2, 3]], {1: 2048, 2: 16, 3: 2048}, [A, B], [0, 1], 2, [(0, 1)],
                         [1, 3])
        tb = lib.tn_serve_submit(c.handle, bp, {})
        ts = [lib.tn_serve_submit(c.handle, sp, amplitude_overrides(snet, small, x))
              for x in random_bitstrings(10, 8, 3)]
        with pytest.raises(lib.TnError) as e:
            t0 = time.time()
            while True:
                st, _, _, _ = lib.tn_serve_poll(c.handle, tb, (2048, 2048))
                if st != lib.TN_PENDING:
                    break
                assert time.time() - t0 < 30
                time.sleep(0.001)
        assert e.value.status == lib.TN_E_NOMEM
        for t in ts:
            st, out, _ = _wait(c, t)
            assert st == lib.TN_OK


def test_serve_queue_bound(monkeypatch):
    """TN_SERVE_QUEUE bounds the requests waiting for admission: with one
    worker busy on a long request (a closed 8192^3 complex GEMM network), the
    bound's worth of requests is accepted and the next submit returns
    TN_E_AGAIN; every accepted request completes, and once the queue has
    drained submits are accepted again."""
    monkeypatch.setenv("TN_SERVE_WORKERS", "1")
    monkeypatch.setenv("TN_SERVE_QUEUE", "4")
    L = 8192
    with lib.Context(8 << 30) as c:
        ones = np.full((L, L), 1.0 / L, dtype=np.complex64)
        big = c.plan_load([[1, 2], [2, 3], [1, 3]], {1: L, 2: L, 3: L}, [ones, ones, ones], [0, 0, 1], 2,
                          [(0, 1), (3, 2)], None, 0, lib.TN_C64)
        small = random_circuit(10, 6, 2)
        snet = amplitude_network(small, 0)
        spl = _plan(snet, 2)
        sp = c.load_network(snet, spl.partition_of, 2, spl.tree)
        lib.tn_contract(big)                      # plan warm (first-call set-up outside the window)
        tb = lib.tn_serve_submit(c.handle, big, {})
        time.sleep(0.005)                         # the worker takes it
        accepted = []
        with pytest.raises(lib.TnError) as e:
            for x in random_bitstrings(10, 16, 4):
                accepted.append((x, lib.tn_serve_submit(c.handle, sp, amplitude_overrides(snet, small, x))))
        assert e.value.status == lib.TN_E_AGAIN
        assert len(accepted) == 4
        st, out, _ = _wait(c, tb)
        assert st == lib.TN_OK and abs(_c(out) - 1.0) < 1e-4     # sum over i, j of (1/L)^3 * L
        for x, t in accepted:
            st, out, _ = _wait(c, t)
            assert st == lib.TN_OK
            alone, _ = lib.tn_contract(sp, amplitude_overrides(snet, small, x))
            assert abs(_c(out) - _c(alone)) <= TOL * max(abs(_c(alone)), 2.0 ** -5)
        t = lib.tn_serve_submit(c.handle, sp, {})
        assert _wait(c, t)[0] == lib.TN_OK
