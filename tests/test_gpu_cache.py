"""The device cache of shared parts: the vertices no override reaches are
computed by the first batched call of a layout and read from the arena by
later calls (exact: they depend only on the plan's own leaves, Section 2.3).

  * a second call skips the shared subtree launch (profiler) and gives the
    same values, bit for bit, as the first and as a context with the cache
    off (TN_CACHE_BYTES=0), and the oracle's within the FP32 bound;
  * with a budget that holds one plan's entry only, calls alternating over
    two plans evict each other and stay right;
  * serve requests on a plan read the entry batched calls filled.
"""
import numpy as np
import pytest

import oracle
from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import (amplitude_network, amplitude_overrides, brickwork_circuit,
                                         output_tensor_ids, random_bitstrings)
from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
from paper_2507_20667_amd.planner.plan import tree_partition
from paper_2507_20667_amd.planner.workloads import brickwork20

pytestmark = pytest.mark.gpu


def _plan(net, k):
    return simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, k), k,
                               SAConfig(iterations=4, n_steps=16, workers=2, rg_samples=8, seed=0))


def _strided(p, net, circ, xs):
    ids = output_tensor_ids(net)
    vec = {t: np.stack([amplitude_overrides(net, circ, x)[t] for x in xs]) for t in ids}
    got, _ = lib.tn_contract_strided(p, len(xs), [(t, vec[t], 32, lib.TN_C128) for t in ids],
                                     scales=False)
    return np.array(got)


def test_cache_hit_skips_shared_and_matches(monkeypatch):
    w = brickwork20()
    circ, net, plan, n = w.circ, w.net, w.plan, w.circ.n
    xs = random_bitstrings(n, 256, 3)
    psi = oracle.statevector(circ)
    exact = psi[np.array(xs, dtype=np.int64)]
    with lib.Context(4 << 30) as ctx:
        p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
        lib.tn_profile_enable(ctx.handle, True)
        lib.tn_profile_read(ctx.handle, reset=True)
        first = _strided(p, net, circ, xs)
        s1 = lib.tn_profile_read(ctx.handle, reset=True)
        second = _strided(p, net, circ, xs)
        s2 = lib.tn_profile_read(ctx.handle, reset=True)
        lib.tn_profile_enable(ctx.handle, False)
        # the shared subtrees ran once, in the first call only
        assert s1["tree"]["launches"] >= 1 and s2["tree"]["launches"] == 0
        assert s2["tree_batch"]["launches"] == s1["tree_batch"]["launches"]
        assert np.array_equal(first, second)
        third = _strided(p, net, circ, xs[:17])
        assert np.array_equal(third, first[:17])
    monkeypatch.setenv("TN_CACHE_BYTES", "0")
    with lib.Context(4 << 30) as ctx0:
        p0 = ctx0.load_network(net, plan.partition_of, 4, plan.tree)
        lib.tn_profile_enable(ctx0.handle, True)
        _strided(p0, net, circ, xs)
        off = _strided(p0, net, circ, xs)
        s = lib.tn_profile_read(ctx0.handle, reset=True)
        assert s["tree"]["launches"] == 2          # no cache: every call runs them
        assert np.array_equal(off, first)
    assert np.max(np.abs(first - exact) / np.maximum(np.abs(exact), 2.0 ** (-n / 2))) < 1e-5


def _entry_bytes(capfd, monkeypatch, nets):
    """Bytes of each plan's cache entry: its shared part (from the layout line
    under TN_DEBUG) plus one 16-byte scale record per tensor id, each rounded
    to 256 bytes."""
    import re
    rnd = lambda b: (b + 255) // 256 * 256
    sizes = []
    monkeypatch.setenv("TN_DEBUG", "1")
    with lib.Context(1 << 30) as ctx:
        for c, net, pl in nets:
            p = ctx.load_network(net, pl.partition_of, 4, pl.tree)
            capfd.readouterr()
            _strided(p, net, c, random_bitstrings(c.n, 4, 1))
            err = capfd.readouterr().err
            shared = int(re.search(r"shared part (\d+) bytes", err).group(1))
            sizes.append(rnd(shared) + rnd((2 * net.num_tensors - 1) * 16))
    monkeypatch.delenv("TN_DEBUG")
    return sizes


def test_cache_eviction_between_plans(capfd, monkeypatch):
    nets = []
    for c in (brickwork_circuit(16, 10, 3), brickwork_circuit(14, 12, 5)):
        net = amplitude_network(c, 0)
        nets.append((c, net, _plan(net, 4)))
    sizes = _entry_bytes(capfd, monkeypatch, nets)
    # room for either entry, not both: the two plans keep evicting each other
    monkeypatch.setenv("TN_CACHE_BYTES", str(max(sizes) + 256))
    assert max(sizes) + 256 < sum(sizes)
    with lib.Context(4 << 30) as ctx:
        ps = [ctx.load_network(net, pl.partition_of, 4, pl.tree) for c, net, pl in nets]
        ref = []
        for (c, net, pl), p in zip(nets, ps):
            xs = random_bitstrings(c.n, 12, 7)
            ref.append((xs, _strided(p, net, c, xs)))
        lib.tn_profile_enable(ctx.handle, True)
        lib.tn_profile_read(ctx.handle, reset=True)
        for rep in range(3):
            for k, ((c, net, pl), p) in enumerate(zip(nets, ps)):
                xs, r = ref[k]
                assert np.array_equal(_strided(p, net, c, xs), r), (rep, k)
        s = lib.tn_profile_read(ctx.handle, reset=True)
        lib.tn_profile_enable(ctx.handle, False)
        # every call found its entry evicted by the other plan's and refilled it
        assert s["tree"]["launches"] >= 6
        # a single plan, called again, hits its entry
        xs, r = ref[1]
        lib.tn_profile_enable(ctx.handle, True)
        assert np.array_equal(_strided(ps[1], nets[1][1], nets[1][0], xs), r)
        s = lib.tn_profile_read(ctx.handle, reset=True)
        lib.tn_profile_enable(ctx.handle, False)
        assert s["tree"]["launches"] == 0
        for k, (c, net, pl) in enumerate(nets):
            xs, r = ref[k]
            for i in (0, 11):
                o = complex(oracle.contract_tree(net.legs, net.dims,
                                                 net.copy_with(amplitude_overrides(net, c, xs[i])).tensors,
                                                 pl.tree))
                assert abs(r[i] - o) / max(abs(o), 2.0 ** (-c.n / 2)) < 1e-5


def test_serve_reads_the_cache():
    c = brickwork_circuit(16, 10, 4)
    net = amplitude_network(c, 0)
    pl = _plan(net, 4)
    with lib.Context(4 << 30) as ctx:
        p = ctx.load_network(net, pl.partition_of, 4, pl.tree)
        xs = random_bitstrings(c.n, 20, 9)
        ref = _strided(p, net, c, xs)          # fills the entry
        tickets = [lib.tn_serve_submit(ctx.handle, p, amplitude_overrides(net, c, x)) for x in xs]
        import time
        for i, t in enumerate(tickets):
            t0 = time.time()
            while True:
                st, out, _, _ = lib.tn_serve_poll(ctx.handle, t)
                if st != lib.TN_PENDING:
                    break
                assert time.time() - t0 < 60
                time.sleep(0.0005)
            assert st == lib.TN_OK
            assert abs(complex(out.reshape(-1)[0]) - ref[i]) <= 1e-6 * max(abs(ref[i]), 2.0 ** -8)
