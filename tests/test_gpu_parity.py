"""GPU parity: libtn through its C ABI against the CPU oracle.

Amplitude error is |a - a_ref| / max(|a_ref|, 2^(-n/2)) (the RMS amplitude of
an n-qubit state is 2^(-n/2), so near-zero amplitudes are judged on that
scale); the bound for the FP32 path is 1e-5.  Networks that are not circuits
(random tensors, general dimensions) are judged relative to the largest
reference entry, with a bound of 64 * 2^-24 times the square root of the
contraction length, which covers FP32 rounding of the inputs plus FP32
accumulation.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from paper_2507_20667_amd import lib
from paper_2507_20667_amd.inputs import (amplitude_network, amplitude_overrides, brickwork_circuit,
                                         phase_poly_circuit, random_bitstrings, random_circuit)
from paper_2507_20667_amd.planner import (SAConfig, contiguous_partition, plan_from_partition,
                                          simulated_annealing)
from paper_2507_20667_amd.planner.plan import tree_partition

pytestmark = pytest.mark.gpu
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(8 << 30)
    yield c
    c.close()


def _c(x):
    return complex(np.asarray(x).reshape(-1)[0])


def amp_err(a, ref, n):
    return abs(_c(a) - _c(ref)) / max(abs(_c(ref)), 2.0 ** (-n / 2))


def test_config1_phase_polynomial_amplitudes(ctx):
    """10 qubits, depth 10, two contiguous partitions; 0^n plus 16 random
    bitstrings per seed, against the oracle and the exact closed form."""
    worst = 0.0
    for seed in range(4):
        circ = phase_poly_circuit(10, 10, seed)
        net = amplitude_network(circ, 0)
        plan = plan_from_partition(net.legs, net.dims, contiguous_partition(net.num_tensors, 2), 2)
        p = ctx.load_network(net, plan.partition_of, 2, plan.tree)
        for x in [0] + random_bitstrings(10, 16, seed):
            ovr = amplitude_overrides(net, circ, x)
            got, l2 = lib.tn_contract(p, ovr)
            exact = cf.phase_poly_amplitude(circ, x)
            ref = oracle.contract_tree(net.legs, net.dims,
                                       net.copy_with(ovr).tensors, plan.tree)
            assert abs(complex(ref) - exact) < 1e-13
            e = amp_err(got, exact, 10)
            worst = max(worst, e)
            assert e < FP32_TOL, (seed, x, got, exact)
        ctx.free_plan(p)
    print(f"config1 max err {worst:.3e}")


def _plan_sa(net, k, seed=0, iters=6):
    init = tree_partition(net.legs, net.dims, k)
    return simulated_annealing(net.legs, net.dims, init, k,
                               SAConfig(iterations=iters, n_steps=16, workers=2, rg_samples=8,
                                        seed=seed))


def test_config2_brickwork_sampled(ctx):
    circ = brickwork_circuit(20, 14, 0)
    net = amplitude_network(circ, 0)
    plan = _plan_sa(net, 4)
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    worst = 0.0
    for x in [0] + random_bitstrings(20, 5, 1):
        ovr = amplitude_overrides(net, circ, x)
        got, _ = lib.tn_contract(p, ovr)
        ref = oracle.contract_tree(net.legs, net.dims, net.copy_with(ovr).tensors, plan.tree)
        e = amp_err(got, ref, 20)
        worst = max(worst, e)
        assert e < FP32_TOL, (x, got, ref)
    ctx.free_plan(p)
    print(f"config2 max err {worst:.3e}")


@pytest.mark.parametrize("form", [lib.TN_FORM_4M, lib.TN_FORM_3M])
def test_gemm_heavy_circuit(ctx, form):
    """A circuit whose plan has GEMM vertices (both operands > 64 entries)."""
    circ = random_circuit(18, 12, 7)
    net = amplitude_network(circ, 0)
    plan = _plan_sa(net, 4, iters=3)
    p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 4, plan.tree, None, form)
    costs = lib.tn_plan_costs_get(p)
    print("gemm nodes", costs["num_gemm_nodes"], "perms", costs["num_permutations"],
          "largest", costs["largest_intermediate"])
    psi = None
    for x in [0] + random_bitstrings(18, 3, 2):
        ovr = amplitude_overrides(net, circ, x)
        got, _ = lib.tn_contract(p, ovr)
        ref = oracle.contract_tree(net.legs, net.dims, net.copy_with(ovr).tensors, plan.tree)
        assert amp_err(got, ref, 18) < FP32_TOL, (x, got, ref)
    ctx.free_plan(p)


def _random_net(rng, nv, dims_choice, n_open):
    legs = [[] for _ in range(nv)]
    dims = {}
    lab = 0
    for e in range(nv - 1):
        legs[e].append(lab)
        legs[e + 1].append(lab)
        dims[lab] = int(rng.choice(dims_choice))
        lab += 1
    for _ in range(nv):
        u, v = rng.choice(nv, 2, replace=False)
        legs[int(u)].append(lab)
        legs[int(v)].append(lab)
        dims[lab] = int(rng.choice(dims_choice))
        lab += 1
    opens = []
    for _ in range(n_open):
        u = int(rng.integers(0, nv))
        legs[u].append(lab)
        dims[lab] = int(rng.choice(dims_choice))
        opens.append(lab)
        lab += 1
    for l in legs:
        rng.shuffle(l)
    ts = [(rng.standard_normal(tuple(dims[x] for x in l))
           + 1j * rng.standard_normal(tuple(dims[x] for x in l))) for l in legs]
    return legs, dims, ts, opens


@pytest.mark.parametrize("seed,dims_choice,n_open", [(0, (2,), 0), (1, (2, 3), 2), (2, (1, 2, 5), 1),
                                                      (3, (2, 4), 3), (4, (3,), 0), (5, (2,), 4)])
def test_random_networks_general_dims(ctx, seed, dims_choice, n_open):
    rng = np.random.default_rng(seed)
    nv = int(rng.integers(5, 9))
    legs, dims, ts, opens = _random_net(rng, nv, dims_choice, n_open)
    k = int(rng.integers(1, 4))
    part = tree_partition(legs, dims, k)
    plan = plan_from_partition(legs, dims, part, k)
    ref = oracle.contract_tree(legs, dims, ts, plan.tree, opens)
    p = ctx.plan_load(legs, dims, ts, plan.partition_of, k, plan.tree, opens or None)
    got, _ = lib.tn_contract(p, result_shape=ref.shape)
    scale = float(np.max(np.abs(ref))) or 1.0
    kmax = max(lib.tn_plan_costs_get(p)["con_serial"], 1)
    tol = 64 * 2.0 ** -24 * math.sqrt(kmax)
    assert np.max(np.abs(got - ref)) / scale < tol
    ctx.free_plan(p)


@pytest.mark.parametrize("shape,perm", [((2,) * 14, None), ((2,) * 20, None), ((4, 8, 2, 16, 2, 8), None),
                                        ((3, 5, 7, 2), None), ((2,) * 23, None)])
def test_permutation_is_bit_exact(ctx, shape, perm):
    """A single-tensor network returned in another leg order is one
    permutation kernel: the complex64 bits must equal numpy's transpose."""
    rng = np.random.default_rng(len(shape))
    r = len(shape)
    perm = perm or list(rng.permutation(r))
    t = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    labs = list(range(100, 100 + r))
    dims = {labs[i]: shape[i] for i in range(r)}
    out_labs = [labs[i] for i in perm]
    p = ctx.plan_load([labs], dims, [t], [0], 1, [], out_labs, 0, lib.TN_C64)
    got, l2 = lib.tn_contract(p, result_shape=tuple(shape[i] for i in perm), out_dtype=lib.TN_C64)
    assert np.array_equal(got, np.transpose(t, perm))
    ctx.free_plan(p)


@pytest.mark.parametrize("M,K,N,form", [(256, 64, 256, lib.TN_FORM_4M), (300, 37, 129, lib.TN_FORM_4M),
                                         (96, 1, 80, lib.TN_FORM_4M), (512, 256, 96, lib.TN_FORM_3M),
                                         (130, 70, 200, lib.TN_FORM_3M),
                                         # few output tiles, deep k: split into k chunks
                                         (64, 4100, 96, lib.TN_FORM_4M), (100, 8192, 70, lib.TN_FORM_3M),
                                         # k a multiple of 16: float planes, k-tiled, ragged M and N
                                         (130, 48, 300, lib.TN_FORM_4M), (200, 4096, 72, lib.TN_FORM_4M),
                                         (130, 48, 300, lib.TN_FORM_3M), (200, 4096, 72, lib.TN_FORM_3M),
                                         (1024, 512, 1024, lib.TN_FORM_3M)]
                         # 1, 3, 5, 7 and 11 stages of 16 k: every tail of the four-slot ring
                         + [(130, k, 200, f) for k in (16, 48, 80, 112, 176)
                            for f in (lib.TN_FORM_4M, lib.TN_FORM_3M)]
                         # 64 x 256 tiles (M <= 64) and 256 x 64 tiles (N <= 64), ragged
                         # and split into k chunks
                         + [(64, 512, 1000, f) for f in (lib.TN_FORM_4M, lib.TN_FORM_3M)]
                         + [(40, 48, 300, lib.TN_FORM_4M), (1000, 64, 48, lib.TN_FORM_3M),
                            (300, 176, 50, lib.TN_FORM_4M), (64, 4096, 600, lib.TN_FORM_3M),
                            (600, 4096, 33, lib.TN_FORM_4M)])
def test_gemm_vertex_against_fp64(ctx, M, K, N, form):
    """Two tensors A(m, k) and B(k, n) with an open output: one GEMM vertex.
    Error bound |dC| <= gamma * |A||B| with gamma = 4 * K * 2^-24 (FP32 inputs
    rounded once, FP32 accumulation)."""
    rng = np.random.default_rng(M + K + N)
    A = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    B = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    legs = [[1, 2], [2, 3]]
    dims = {1: M, 2: K, 3: N}
    p = ctx.plan_load(legs, dims, [A, B], [0, 1], 2, [(0, 1)], [1, 3], form)
    assert lib.tn_plan_costs_get(p)["num_gemm_nodes"] == 1
    got, _ = lib.tn_contract(p, result_shape=(M, N))
    A32 = A.astype(np.complex64).astype(np.complex128)
    B32 = B.astype(np.complex64).astype(np.complex128)
    ref = A32 @ B32
    bound = (np.abs(A32) @ np.abs(B32)) * (4 * K * 2.0 ** -24) * (2 if form == lib.TN_FORM_3M else 1)
    assert np.all(np.abs(got - ref) <= bound + 1e-30)
    ctx.free_plan(p)


def test_batch_matches_single(ctx):
    circ = random_circuit(14, 10, 11)
    net = amplitude_network(circ, 0)
    plan = _plan_sa(net, 4, iters=3)
    p = ctx.load_network(net, plan.partition_of, 4, plan.tree)
    xs = random_bitstrings(14, 24, 5)
    queries = [(p, amplitude_overrides(net, circ, x)) for x in xs]
    outs, l2, st = lib.tn_contract_batch(ctx.handle, queries, [()] * len(xs))
    assert np.all(st == 0)
    for x, o in zip(xs, outs):
        single, _ = lib.tn_contract(p, amplitude_overrides(net, circ, x))
        assert abs(_c(o) - _c(single)) <= 1e-6 * max(abs(_c(single)), 2 ** -7)
        ref = oracle.contract_tree(net.legs, net.dims,
                                   net.copy_with(amplitude_overrides(net, circ, x)).tensors,
                                   plan.tree)
        assert amp_err(o, ref, 14) < FP32_TOL
    ctx.free_plan(p)


def test_keep_scale_and_open_legs(ctx):
    circ = random_circuit(10, 6, 3)
    net = amplitude_network(circ, None)  # whole state
    plan = plan_from_partition(net.legs, net.dims, tree_partition(net.legs, net.dims, 2), 2)
    p = ctx.load_network(net, plan.partition_of, 2, plan.tree)
    psi = oracle.statevector(circ)
    got, l2 = lib.tn_contract(p, result_shape=(2,) * 10, flags=lib.TN_FLAG_KEEP_SCALE)
    full = got.reshape(-1) * 2.0 ** l2
    err = np.max(np.abs(full - psi)) / 2 ** -5
    assert err < FP32_TOL
    assert abs(np.sum(np.abs(full) ** 2) - 1) < 1e-5
    ctx.free_plan(p)


@pytest.mark.parametrize("M,K,N,form", [(256, 64, 256, lib.TN_FORM_4M), (300, 37, 129, lib.TN_FORM_4M),
                                         (512, 256, 96, lib.TN_FORM_3M), (130, 70, 200, lib.TN_FORM_3M),
                                         (1024, 512, 1024, lib.TN_FORM_4M),
                                         # split into k chunks (aligned, ragged and unaligned k)
                                         (64, 4096, 96, lib.TN_FORM_4M), (200, 3000, 130, lib.TN_FORM_3M),
                                         (64, 2050, 64, lib.TN_FORM_4M),
                                         # k a multiple of 16: k-tiled planes streamed into LDS
                                         (1024, 512, 1024, lib.TN_FORM_3M), (64, 4096, 96, lib.TN_FORM_3M),
                                         (300, 64, 129, lib.TN_FORM_3M)]
                         # 1 to 13 stages of 16 k: every tail of the two-slot (4M) and
                         # three-slot (3M) rings
                         + [(130, k, 200, f) for k in (16, 32, 48, 80, 96, 112, 176, 208)
                            for f in (lib.TN_FORM_4M, lib.TN_FORM_3M)]
                         # 4M on the two wave-group kernel: 256 x 128 tiles (M >= 256) and
                         # 128 x 256 (N >= 256), ragged in M and N, 1 to 7 stages (every
                         # tail of both groups' loops), and split into k chunks
                         + [(300, k, 260, lib.TN_FORM_4M) for k in (16, 32, 48, 64, 80, 96, 112)]
                         + [(140, 48, 520, lib.TN_FORM_4M), (140, 208, 300, lib.TN_FORM_4M),
                            (256, 8192, 256, lib.TN_FORM_4M), (520, 4096, 130, lib.TN_FORM_4M)])
def test_gemm_vertex_bf16x3_against_fp64(ctx, M, K, N, form):
    """Three-term split BF16: each real product a*b is carried as
    ha*hb + ha*lb + la*hb with h = bf16(a), l = bf16(a - h), so the dropped
    terms are below 2^-15 |a||b|; FP32 accumulation adds K * 2^-24.  Bound per
    entry: 4 (2^-15 + K 2^-24) (|A||B|) for 4M, twice that for 3M (whose
    products carry (Ar + Ai)(Br + Bi))."""
    rng = np.random.default_rng(M * 7 + K + N)
    A = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    B = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    legs = [[1, 2], [2, 3]]
    dims = {1: M, 2: K, 3: N}
    p = ctx.plan_load(legs, dims, [A, B], [0, 1], 2, [(0, 1)], [1, 3], lib.TN_PREC_BF16X3 | form)
    got, _ = lib.tn_contract(p, result_shape=(M, N))
    A32 = A.astype(np.complex64).astype(np.complex128)
    B32 = B.astype(np.complex64).astype(np.complex128)
    ref = A32 @ B32
    gamma = 4 * (2.0 ** -15 + K * 2.0 ** -24) * (2 if form == lib.TN_FORM_3M else 1)
    bound = (np.abs(A32) @ np.abs(B32)) * gamma
    assert np.all(np.abs(got - ref) <= bound)
    # and it is not FP32-exact: the split really ran (its error is well above
    # that of an FP32 product of the same operands, whatever K; a product
    # carries ~2^-17 relative error against FP32's 2^-24)
    ref32 = (A.astype(np.complex64) @ B.astype(np.complex64)).astype(np.complex128)
    assert np.max(np.abs(got - ref)) > 4 * np.max(np.abs(ref32 - ref))
    ctx.free_plan(p)


@pytest.mark.parametrize("form", [lib.TN_FORM_4M, lib.TN_FORM_3M])
def test_gemm_heavy_circuit_bf16x3(ctx, form):
    circ = random_circuit(18, 12, 7)
    net = amplitude_network(circ, 0)
    plan = _plan_sa(net, 4, iters=3)
    p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 4, plan.tree, None,
                      lib.TN_PREC_BF16X3 | form)
    worst = 0.0
    for x in [0] + random_bitstrings(18, 3, 2):
        ovr = amplitude_overrides(net, circ, x)
        got, _ = lib.tn_contract(p, ovr)
        ref = oracle.contract_tree(net.legs, net.dims, net.copy_with(ovr).tensors, plan.tree)
        e = amp_err(got, ref, 18)
        worst = max(worst, e)
        assert e < 1e-3, (x, got, ref)
    print("bf16x3 circuit max err", worst)
    ctx.free_plan(p)


@pytest.mark.parametrize("force", ["0,1", "1,1", "2,1", "0,4", "1,8", "2,2", "1,3"])
@pytest.mark.parametrize("form", [lib.TN_FORM_4M, lib.TN_FORM_3M])
def test_gemm_forced_tiles_and_chunks(ctx, monkeypatch, force, form):
    """Every FP32 plane tile shape and k-chunk count the tuner may choose
    (TN_GEMM_FORCE at plan load) on ragged shapes: within the FP32 bound of
    the FP64 product."""
    M, K, N = 150, 1024, 230
    rng = np.random.default_rng(sum(map(ord, force)) + form)
    A = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    B = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    monkeypatch.setenv("TN_GEMM_FORCE", force)
    p = ctx.plan_load([[1, 2], [2, 3]], {1: M, 2: K, 3: N}, [A, B], [0, 1], 2, [(0, 1)], [1, 3], form)
    monkeypatch.delenv("TN_GEMM_FORCE")
    got, _ = lib.tn_contract(p, result_shape=(M, N))
    A32 = A.astype(np.complex64).astype(np.complex128)
    B32 = B.astype(np.complex64).astype(np.complex128)
    ref = A32 @ B32
    bound = (np.abs(A32) @ np.abs(B32)) * (4 * K * 2.0 ** -24) * (2 if form == lib.TN_FORM_3M else 1)
    assert np.all(np.abs(got - ref) <= bound + 1e-30)
    ctx.free_plan(p)


@pytest.mark.parametrize("force", ["0,1", "1,1", "2,1", "1,4", "2,3"])
def test_gemm_forced_tiles_bf16x3(ctx, monkeypatch, force):
    """BF16x3 4M with every tile shape the tuner may choose (128 x 128 on two
    blocks per CU; 128 x 256 and 256 x 128 on the two wave-group kernel) and
    k chunks, on a shape smaller than the wide tiles in both directions (rows
    past M and N clamped): within the split-BF16 bound of the FP64 product."""
    M, K, N = 150, 1024, 230
    rng = np.random.default_rng(sum(map(ord, force)) + 17)
    A = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    B = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    monkeypatch.setenv("TN_GEMM_FORCE", force)
    p = ctx.plan_load([[1, 2], [2, 3]], {1: M, 2: K, 3: N}, [A, B], [0, 1], 2, [(0, 1)], [1, 3],
                      lib.TN_PREC_BF16X3 | lib.TN_FORM_4M)
    monkeypatch.delenv("TN_GEMM_FORCE")
    got, _ = lib.tn_contract(p, result_shape=(M, N))
    A32 = A.astype(np.complex64).astype(np.complex128)
    B32 = B.astype(np.complex64).astype(np.complex128)
    ref = A32 @ B32
    bound = (np.abs(A32) @ np.abs(B32)) * 4 * (2.0 ** -15 + K * 2.0 ** -24)
    assert np.all(np.abs(got - ref) <= bound)
    ctx.free_plan(p)
