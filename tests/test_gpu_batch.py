"""GPU parity of the batched path (tn_contract_batch): the subtree kernel that
runs whole small subtrees in one workgroup, shared subtrees computed once,
partial and device-resident overrides.  Each result is compared with the
oracle (amplitude error as in test_gpu_parity, bound 1e-5 for FP32) and with
the same query run alone through tn_contract."""
import math

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
    # one launch for the shared subtrees, one for the batch of 16 queries
    assert stats["tree"]["launches"] >= 1 and stats["tree"]["seconds"] > 0
    assert stats["tree_batch"]["launches"] >= 1 and stats["tree_batch"]["seconds"] > 0
    ctx.free_plan(p)


def _gate_net(rng, dims_choice, n_state, n_gates):
    """A rank-n_state tensor with gate-like tensors (one or two of its legs in,
    as many out) applied one after the other, then closed by rank-1 boundary
    tensors: small operands along the fibers of a large one, with legs of the
    given dimensions."""
    lab = 0
    cur, dims = [], {}
    for _ in range(n_state):
        dims[lab] = int(rng.choice(dims_choice))
        cur.append(lab)
        lab += 1
    legs = [list(cur)]
    for _ in range(n_gates):
        k = int(rng.integers(1, 3))
        pos = [int(x) for x in rng.choice(n_state, k, replace=False)]
        new = []
        for p_ in pos:
            dims[lab] = dims[cur[p_]]
            new.append(lab)
            lab += 1
        legs.append([cur[p_] for p_ in pos] + new)
        for p_, l in zip(pos, new):
            cur[p_] = l
    for l in cur:
        legs.append([l])
    ts = [rng.standard_normal(tuple(dims[x] for x in l)) + 1j * rng.standard_normal(tuple(dims[x] for x in l))
          for l in legs]
    return legs, dims, ts


@pytest.mark.parametrize("seed,dims_choice", [(0, (2,)), (1, (2, 3)), (2, (3, 4)), (3, (1, 2, 5)), (4, (2, 4))])
def test_batch_general_dims(ctx, seed, dims_choice):
    """Subtrees over legs of any dimension (the gate-along-fibers form and the
    general form, power-of-two and mixed-radix index maps), each of 24
    queries overriding the first boundary tensor, against the oracle."""
    from paper_2507_20667_amd.planner import plan_from_partition
    rng = np.random.default_rng(seed)
    legs, dims, ts = _gate_net(rng, dims_choice, 7, 12)
    nv = len(legs)
    plan = plan_from_partition(legs, dims, tree_partition(legs, dims, 2), 2)
    p = ctx.plan_load(legs, dims, ts, plan.partition_of, 2, plan.tree)
    first = nv - 7
    queries, refs = [], []
    for _ in range(24):
        v = rng.standard_normal(ts[first].shape) + 1j * rng.standard_normal(ts[first].shape)
        queries.append((p, {first: v}))
        refs.append(complex(oracle.contract_tree(legs, dims, ts[:first] + [v] + ts[first + 1:], plan.tree)))
    outs, l2, st = lib.tn_contract_batch(ctx.handle, queries, [()] * len(queries))
    assert np.all(st == 0)
    scale = max(abs(r) for r in refs) or 1.0
    tol = 64 * 2.0 ** -24 * math.sqrt(max(lib.tn_plan_costs_get(p)["con_serial"], 1))
    for o, r in zip(outs, refs):
        assert abs(_c(o) - r) / scale < tol, (o, r)
    ctx.free_plan(p)


@pytest.mark.parametrize("where", ["host", "device", "device_unaligned"])
def test_strided_matches_batch(ctx, where):
    """tn_contract_strided (one descriptor and one stride per overridden leaf)
    gives the same results as tn_contract_batch on the same queries, with the
    overrides in host memory (staged), on the device read in place, and on the
    device at a stride the kernels cannot step (copied per query); and agrees
    with the oracle."""
    import torch
    circ = random_circuit(14, 8, 21)
    net = amplitude_network(circ, 0)
    plan = _plan(net, 4)
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    xs = random_bitstrings(circ.n, 40, 9)
    ids = output_tensor_ids(net)
    # one array per overridden leaf: (queries, 2) basis vectors, in query order
    vec = {t: np.stack([amplitude_overrides(net, circ, x)[t] for x in xs]) for t in ids}
    ref, _, st = lib.tn_contract_batch(ctx.handle, [(p, amplitude_overrides(net, circ, x)) for x in xs],
                                       [()] * len(xs))
    assert np.all(st == 0)
    keep = []
    ovr = []
    for t in ids:
        if where == "host":
            ovr.append((t, vec[t].astype(np.complex128), 16 * vec[t].shape[1], lib.TN_C128))
        else:
            # floats per query: 4 (the two complex64 entries, a 16-byte stride) or 5
            # (a 20-byte stride the kernels cannot step)
            cols = 5 if where == "device_unaligned" else 4
            d = torch.zeros((len(xs), cols), dtype=torch.float32, device="cuda")
            v = torch.from_numpy(vec[t].astype(np.complex64).view(np.float32)).to("cuda")
            d[:, :4] = v.reshape(len(xs), 4)
            keep.append(d)
            stride = d.shape[1] * 4
            ovr.append((t, d.data_ptr(), stride, lib.TN_C64_DEVICE))
    torch.cuda.synchronize()
    got, l2 = lib.tn_contract_strided(p, len(xs), ovr)
    for i, x in enumerate(xs):
        assert abs(complex(got[i]) - _c(ref[i])) <= 1e-6 * max(abs(_c(ref[i])), 2.0 ** -7)
    for i in (0, 17, 39):
        r = _ref(net, plan, amplitude_overrides(net, circ, xs[i]))
        assert err(got[i], r, circ.n) < TOL
    ctx.free_plan(p)


@pytest.mark.parametrize("stride", [1, 3])
def test_strided_pinned_output(ctx, capfd, monkeypatch, stride):
    """Complex128 results into pinned host memory: the subtree kernel writes each
    closed root's value there itself (the call says so under TN_DEBUG), bit for
    bit what the host writes into pageable memory from the result records, the
    results `stride` elements apart (the elements between left alone), with and
    without the scales asked for; and the values agree with the oracle."""
    import torch
    circ = brickwork_circuit(16, 10, 3)
    net = amplitude_network(circ, 0)
    plan = _plan(net, 4)
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    xs = random_bitstrings(circ.n, 48, 12)
    ids = output_tensor_ids(net)
    vec = {t: np.stack([amplitude_overrides(net, circ, x)[t] for x in xs]) for t in ids}
    ovr = [(t, vec[t].astype(np.complex128), 16 * vec[t].shape[1], lib.TN_C128) for t in ids]
    ref, _ = lib.tn_contract_strided(p, len(xs), ovr)  # pageable: converted on the host
    pinned = torch.zeros((len(xs), stride), dtype=torch.complex128, pin_memory=True)
    out = pinned.numpy()
    out[:] = np.nan
    monkeypatch.setenv("TN_DEBUG", "1")
    got, l2 = lib.tn_contract_strided(p, len(xs), ovr, out=out, out_stride=stride)
    monkeypatch.delenv("TN_DEBUG")
    assert "results written by the kernel" in capfd.readouterr().err
    assert np.array_equal(got[:, 0], ref)
    assert np.all(l2 == 0.0)
    assert np.all(np.isnan(got[:, 1:]))
    out[:, 0] = np.nan
    got2, none = lib.tn_contract_strided(p, len(xs), ovr, out=out, out_stride=stride, scales=False)
    assert none is None and np.array_equal(got2[:, 0], ref)
    for i in (0, 23, 47):
        r = _ref(net, plan, amplitude_overrides(net, circ, xs[i]))
        assert err(got[i, 0], r, circ.n) < TOL
    ctx.free_plan(p)


def test_packed_gate_steps_match_unpacked(ctx, monkeypatch):
    """Small gate vertices packed into lane-record steps (the default) give the
    same amplitudes, bit for bit, as the same programs with packing off
    (TN_TREE_PACK=0, read when a plan's layouts are built) and with vertices
    of up to 256 entries packed (TN_TREE_PACK_NC=256: one vertex over several
    steps): on a batch (the batch kernel) and on single queries (the level
    kernel); and they agree with the oracle."""
    circ = brickwork_circuit(16, 10, 7)
    net = amplitude_network(circ, 0)
    plan = _plan(net, 4)
    xs = random_bitstrings(circ.n, 40, 77)
    ids = output_tensor_ids(net)
    vec = {t: np.stack([amplitude_overrides(net, circ, x)[t] for x in xs]) for t in ids}
    ovr = [(t, vec[t].astype(np.complex128), 16 * vec[t].shape[1], lib.TN_C128) for t in ids]

    def run():
        p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
        batch, _ = lib.tn_contract_strided(p, len(xs), ovr)
        singles = [lib.tn_contract(p, amplitude_overrides(net, circ, xs[i]))[0] for i in (0, 5)]
        ctx.free_plan(p)
        return batch, singles

    monkeypatch.setenv("TN_TREE_PACK", "0")
    b0, s0 = run()
    monkeypatch.delenv("TN_TREE_PACK")
    # vertices up to 256 entries packed too (one vertex spanning several steps)
    monkeypatch.setenv("TN_TREE_PACK_NC", "256")
    b2, s2 = run()
    monkeypatch.delenv("TN_TREE_PACK_NC")
    b1, s1 = run()
    assert np.array_equal(b0, b1) and np.array_equal(b0, b2)
    for a, b, c in zip(s0, s1, s2):
        assert _c(a) == _c(b) == _c(c)
    for i in (0, 5, 39):
        r = _ref(net, plan, amplitude_overrides(net, circ, xs[i]))
        assert err(b1[i], r, circ.n) < TOL
    for i, sq in zip((0, 5), s1):  # single queries (level kernel) against the batch
        assert abs(_c(sq) - _c(b1[i])) <= 1e-6 * max(abs(_c(b1[i])), 2.0 ** -8)


def test_graph_replay_matches_eager(ctx):
    """TN_FLAG_GRAPH: the first call captures the plan group's launch sequence,
    later calls with the same group replay it.  Every replay (new bitstrings
    staged into the same workspace, with eager calls and synchronizations in
    between) equals the eager batch; in-place device overrides replay while
    their buffer stays the same and are captured again when it changes; a
    different query count replaces the graph."""
    import torch
    circ = random_circuit(16, 10, 31)
    net = amplitude_network(circ, 0)
    plan = _plan(net, 4)
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    ids = output_tensor_ids(net)
    for rep in range(4):
        xs = random_bitstrings(circ.n, 32, 100 + rep)
        qs = [(p, amplitude_overrides(net, circ, x)) for x in xs]
        ref, _, st = lib.tn_contract_batch(ctx.handle, qs, [()] * len(xs))
        assert np.all(st == 0)
        got, _, st = lib.tn_contract_batch(ctx.handle, qs, [()] * len(xs), flags=lib.TN_FLAG_GRAPH)
        assert np.all(st == 0)
        for a, b in zip(got, ref):
            assert _c(a) == _c(b)
        single, _ = lib.tn_contract(*qs[3])  # eager work between replays
        assert abs(_c(single) - _c(ref[3])) <= 1e-6 * max(abs(_c(ref[3])), 2.0 ** -8)
        torch.cuda.synchronize()
    # device overrides read in place: one buffer (replay), then another (capture)
    for rep in range(3):
        xs = random_bitstrings(circ.n, 24, 200 + rep)
        vec = {t: np.stack([amplitude_overrides(net, circ, x)[t] for x in xs]) for t in ids}
        if rep < 2:
            if rep == 0:
                bufs = {t: torch.zeros((len(xs), 4), dtype=torch.float32, device="cuda") for t in ids}
            for t in ids:
                bufs[t].copy_(torch.from_numpy(vec[t].astype(np.complex64).view(np.float32)).reshape(len(xs), 4))
        else:
            bufs = {t: torch.from_numpy(vec[t].astype(np.complex64).view(np.float32)).reshape(len(xs), 4).cuda()
                    for t in ids}
        torch.cuda.synchronize()
        ovr = [(t, bufs[t].data_ptr(), 16, lib.TN_C64_DEVICE) for t in ids]
        eager, _ = lib.tn_contract_strided(p, len(xs), ovr)
        graph, _ = lib.tn_contract_strided(p, len(xs), ovr, flags=lib.TN_FLAG_GRAPH)
        assert np.array_equal(eager, graph)
        refs = [_ref(net, plan, amplitude_overrides(net, circ, xs[i])) for i in (0, 11)]
        for i, r in zip((0, 11), refs):
            assert err(graph[i], r, circ.n) < TOL
    ctx.free_plan(p)


def test_multi_plan_batch_concurrent(ctx):
    """Queries of several plans in one call (their groups run concurrently on
    separate streams) equal the same queries one at a time, interleaved in
    any order, and match the oracle."""
    circs = [random_circuit(12, 8, 41), random_circuit(14, 10, 42), brickwork_circuit(12, 8, 43),
             phase_poly_circuit(10, 6, 44), random_circuit(16, 6, 45)]
    loaded = []
    for c in circs:
        net = amplitude_network(c, 0)
        plan = _plan(net, 2)
        loaded.append((c, net, plan, ctx.load_network(net, plan.partition_of, 2, plan.tree)))
    rng = np.random.default_rng(7)
    qs, meta = [], []
    for _ in range(60):
        k = int(rng.integers(0, len(loaded)))
        c, net, plan, p = loaded[k]
        x = int(rng.integers(0, 1 << c.n))
        qs.append((p, amplitude_overrides(net, c, x)))
        meta.append((k, x))
    outs, _, st = lib.tn_contract_batch(ctx.handle, qs, [()] * len(qs))
    assert np.all(st == 0)
    for (k, x), q, o in zip(meta, qs, outs):
        single, _ = lib.tn_contract(*q)
        assert abs(_c(o) - _c(single)) <= 1e-6 * max(abs(_c(single)), 2.0 ** -8)
    for j in (0, 13, 59):
        k, x = meta[j]
        c, net, plan, p = loaded[k]
        assert err(outs[j], _ref(net, plan, qs[j][1]), c.n) < TOL
    for c, net, plan, p in loaded:
        ctx.free_plan(p)


def test_batch_open_legs_each_query(ctx):
    """Open legs in a batch: every query's result (several entries, permuted
    into output-leg order) is its own, equal to the query run alone and to the
    oracle."""
    circ = random_circuit(13, 8, 51)
    net = amplitude_network(circ, 0, open_qubits=(2, 7, 11))
    plan = _plan(net, 3)
    p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 3, plan.tree,
                      net.output_legs)
    xs = random_bitstrings(circ.n, 21, 52)
    qs = [(p, amplitude_overrides(net, circ, x, open_qubits=(2, 7, 11))) for x in xs]
    outs, _, st = lib.tn_contract_batch(ctx.handle, qs, [(2, 2, 2)] * len(qs))
    assert np.all(st == 0)
    for q, o in zip(qs, outs):
        single, _ = lib.tn_contract(q[0], q[1], result_shape=(2, 2, 2))
        scale = max(float(np.max(np.abs(single))), 2.0 ** -7)
        assert np.max(np.abs(o - single)) <= 1e-6 * scale
    for i in (0, 10, 20):
        r = oracle.contract_tree(net.legs, net.dims, net.copy_with(qs[i][1]).tensors, plan.tree,
                                 net.output_legs)
        assert np.max(np.abs(outs[i] - r)) / max(float(np.max(np.abs(r))), 2.0 ** -7) < TOL
    ctx.free_plan(p)


@pytest.mark.parametrize("qw", [None, "8", "6"])
def test_batch_sizes_and_query_grouping(ctx, qw, monkeypatch):
    """Batches of 1 to 13 queries: workgroups with fewer queries than waves,
    a last workgroup partly filled, and (through the queries-per-workgroup
    override, read when a plan's layout is built) waves that take two queries
    each; every amplitude against the oracle."""
    if qw is None:
        monkeypatch.delenv("TN_TREE_QW", raising=False)
    else:
        monkeypatch.setenv("TN_TREE_QW", qw)
    circ = brickwork_circuit(14, 8, 5)
    net = amplitude_network(circ, 0)
    plan = _plan(net, 3)
    p = ctx.load_network(net, plan.partition_of, 3, plan.tree)
    xs_all = random_bitstrings(circ.n, 31, 7)
    off = 0
    for q in (1, 2, 3, 5, 7, 13):
        xs = xs_all[off:off + q]
        off += q
        queries = [(p, amplitude_overrides(net, circ, x)) for x in xs]
        outs, _, st = lib.tn_contract_batch(ctx.handle, queries, [()] * len(xs))
        assert np.all(st == 0)
        for x, o in zip(xs, outs):
            e = err(o, _ref(net, plan, amplitude_overrides(net, circ, x)), circ.n)
            assert e < TOL, (qw, q, x, o)
    ctx.free_plan(p)
