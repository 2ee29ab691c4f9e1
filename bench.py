"""Throughput of partitioned tensor-network contraction on one MI355X.

Headline workload (the largest configuration): the 30-qubit random circuit of
depth 20 (seed 0, 7 CX pairs per layer, 70 % nearest-neighbour), one closed
network per output bitstring, 8 partitions refined by simulated annealing,
largest intermediate 2^27 complex64.  One step contracts `--queries`
amplitudes (seeded random bitstrings) through the whole path in one
tn_contract_strided call: leaf overrides (basis vectors read in place from
device memory), every partition's tree in turn (leg permutations, complex
GEMMs, the subtree kernels for the small vertices), the reduction path and
the FP64 closed root.  `value` is amplitudes/s of that path in the chosen
precision and form (default FP32 3M); beside it: the plain FP32 4M path
(tn_contract one query at a time, the denominator of the speed-up), effective
complex TFLOP/s (8 * con_serial per amplitude), the roofline position of the
dominant kernel (the GEMM, event-timed inside this run), the permutation
kernels' HBM GB/s, and the error of nine amplitudes against stored
state-vector values.  The CPU oracle is timed on a bounded sample.

Secondary legs (each can be skipped): the 20-qubit brickwork batch of 4096
queries per step, the GEMM phase of the 30-qubit plan in every precision and
form, the uneven 512-query batch over 64 circuits, and serving.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--queries 8]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "amplitudes/s + effective complex TFLOP/s vs plain FP32 path; serve p50/p99"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2516.6}
# FP32 vector rate without the packed FP32 instructions, which this build
# keeps off: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_VALU_ATTAINABLE_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def device_overrides(torch, net, n, bitstrings):
    """(queries, n, 2) complex64 basis vectors on the device, output qubit
    order; returns the tensor and per-query tn_leaf arrays pointing into it."""
    from paper_2507_20667_amd import lib
    from paper_2507_20667_amd.inputs import output_tensor_ids
    ids = output_tensor_ids(net)
    Q = len(bitstrings)
    bits = np.array([[(x >> q) & 1 for q in range(n)] for x in bitstrings], dtype=np.int64)
    host = np.zeros((Q, n, 2), dtype=np.complex64)
    host[np.arange(Q)[:, None], np.arange(n)[None, :], bits] = 1.0
    dev = torch.from_numpy(host).to("cuda")
    base = dev.data_ptr()
    leaves = []
    for qi in range(Q):
        arr = (lib.tn_leaf * n)()
        for i, t in enumerate(ids):
            arr[i] = lib.tn_leaf(t, base + ((qi * n + i) * 2) * 8, lib.TN_C64_DEVICE)
        leaves.append(arr)
    return dev, leaves


def strided_call(lib, plan, dev, net, n):
    """tn_contract_strided over the (queries, n, 2) device tensor: one leaf
    descriptor per output qubit with a stride of one query's block."""
    from paper_2507_20667_amd.inputs import output_tensor_ids
    ids = output_tensor_ids(net)
    Q = dev.shape[0]
    base = dev.data_ptr()
    arr = (lib.tn_leaf * n)()
    strides = (ctypes.c_int64 * n)()
    for i, t in enumerate(ids):
        arr[i] = lib.tn_leaf(t, base + i * 16, lib.TN_C64_DEVICE)
        strides[i] = n * 16
    # the results go to pinned host memory, which the subtree kernel writes itself
    import torch
    outs_t = torch.zeros((Q, 2), dtype=torch.float64, pin_memory=True)
    outs = outs_t.numpy()
    # the call's arguments, marshalled once
    fn = lib.load().tn_contract_strided
    args = (ctypes.c_void_p(plan), Q, n, ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(strides, ctypes.c_void_p),
            outs.ctypes.data_as(ctypes.c_void_p), 1, lib.TN_C128, None, 0)

    def call():
        rc = fn(*args)
        if rc != 0:
            raise lib.TnError(rc, lib.tn_last_error())
        return outs
    call.keep = (arr, strides, dev, outs_t)
    return call


def batch_call(lib, ctx, plan, leaves, n):
    Q = len(leaves)
    qarr = (lib.tn_query * Q)()
    for i, arr in enumerate(leaves):
        qarr[i] = lib.tn_query(plan, n, ctypes.cast(arr, ctypes.c_void_p).value)
    outs = np.zeros((Q, 2), dtype=np.float64)
    optrs = (ctypes.c_void_p * Q)(*[outs.ctypes.data + 16 * i for i in range(Q)])
    st = np.zeros(Q, dtype=np.int32)

    def call():
        rc = lib.load().tn_contract_batch(ctypes.c_void_p(ctx), Q, ctypes.cast(qarr, ctypes.c_void_p),
                                          ctypes.cast(optrs, ctypes.c_void_p), lib.TN_C128, None,
                                          st.ctypes.data_as(ctypes.c_void_p), 0)
        if rc != 0:
            raise lib.TnError(rc, lib.tn_last_error())
        return outs
    return call


SERVE_MAX_LARGEST = 1 << 32     # planned largest intermediate (entries)
SERVE_MAX_WORK = 1 << 36        # con_serial (complex multiply-adds) of one request


def _serve_circuit(args):
    """Circuit c of the serving pool and its three planned networks."""
    c, seed = args
    from paper_2507_20667_amd.inputs import amplitude_network, random_circuit, zz_network
    from paper_2507_20667_amd.planner import cost, plan_from_partition
    from paper_2507_20667_amd.planner.plan import tree_partition
    rng = np.random.default_rng([seed, c])
    for r in range(1000):
        # a draw out of bounds is replaced by a new draw of size, depth,
        # circuit and pairs
        n = int(rng.integers(12, 33))
        d = int(rng.integers(8, 25))
        pairs = [tuple(sorted(int(v) for v in rng.choice(n, 2, replace=False))) for _ in range(2)]
        circ = random_circuit(n, d, 7000 + 1000 * c + r)
        nets = [("amp", amplitude_network(circ, 0), None)] + \
               [("zz", zz_network(circ, i, j), (i, j)) for i, j in pairs]
        planned = []
        for kind, net, ij in nets:
            k = 4 if net.num_tensors >= 8 else 1
            pl = plan_from_partition(net.legs, net.dims, tree_partition(net.legs, net.dims, k), k)
            li = cost.largest_intermediate(net.legs, net.dims, pl.tree)
            cs = cost.con_serial(net.legs, net.dims, pl.tree)
            if li > SERVE_MAX_LARGEST or cs > SERVE_MAX_WORK:
                break
            planned.append((kind, net, ij, pl, k, cs, li))
        if len(planned) == len(nets):
            return circ, planned
    raise RuntimeError(f"no draw of circuit {c} fits the bounds")


def serve_pool(n_circuits=128, seed=2024, processes=8):
    """The serving pool: circuit c of the random family (n/4 CX pairs per
    layer, 70 % nearest-neighbour) with n ~ U{12..32} and depth ~ U{8..24}
    drawn from (seed, c), the circuit itself from seed 7000 + 1000 c + r, r
    counting the draws (size, depth, pairs and circuit drawn again until the
    networks are in bounds); per circuit its amplitude
    network and the light-cone-pruned networks of <Z_i Z_j> for two pairs
    i < j drawn uniformly.  Each network is planned with 4 partitions (the
    tree split, Greedy inside) and must keep its largest intermediate within
    2^32 entries and its con_serial within 2^36 multiply-adds.  The circuits
    are planned in forked processes (before this process touches the GPU)."""
    t0 = time.perf_counter()
    jobs = [(c, seed) for c in range(n_circuits)]
    if processes > 1:
        import multiprocessing
        with multiprocessing.get_context("fork").Pool(processes) as mp:
            pool = mp.map(_serve_circuit, jobs)
    else:
        pool = [_serve_circuit(j) for j in jobs]
    return pool, time.perf_counter() - t0


def serve_bench(lib, ctx, pool, flags, rate, warmup_s, seconds, seed=0, check=32):
    """Poisson arrivals (rate per second) of amplitude and <Z_i Z_j> requests:
    circuit ~ truncated Zipf(1.1) over the pool, amplitude (uniform bitstring)
    or one of the circuit's two <Z_i Z_j> networks with probability 1/2 each.
    Requests arrive for warmup_s + seconds; latencies (submit to ready) and
    the achieved rate are over the requests of the measured window.  Then
    `check` requests of the window are run again alone (tn_contract) and
    compared with what serving returned."""
    import threading
    from paper_2507_20667_amd.inputs import amplitude_overrides, zipf_indices
    rng = np.random.default_rng(seed)
    plans = []
    for circ, nets in pool:
        plans.append([(kind, net, ij, ctx.plan_load(net.legs, net.dims, net.tensors, pl.partition_of, k,
                                                     pl.tree, None, flags), cs)
                      for kind, net, ij, pl, k, cs, li in nets])
    nreq = max(1, int((warmup_s + seconds) * rate))
    which = zipf_indices(len(pool), nreq, 1.1, seed + 1)
    reqs = []
    for c in which:
        circ = pool[c][0]
        if rng.random() < 0.5:
            kind, net, ij, p, cs = plans[c][0]
            x = int(rng.integers(0, 1 << circ.n))
            reqs.append((c, 0, p, amplitude_overrides(net, circ, x), cs))
        else:
            z = 1 + int(rng.integers(0, 2))
            kind, net, ij, p, cs = plans[c][z]
            reqs.append((c, z, p, {}, cs))
    gaps = rng.exponential(1.0 / rate, size=nreq)
    tickets = [None] * nreq
    t_sub = [0.0] * nreq
    results = [None] * nreq
    lat = [None] * nreq
    done_at = [None] * nreq

    def submitter():
        t_next = time.perf_counter()
        for i, (c, z, p, ovr, cs) in enumerate(reqs):
            t_next += gaps[i]
            while time.perf_counter() < t_next:
                time.sleep(min(1e-3, max(0.0, t_next - time.perf_counter())))
            t_sub[i] = time.perf_counter()
            tickets[i] = lib.tn_serve_submit(ctx.handle, p, ovr)

    start = time.perf_counter()
    th = threading.Thread(target=submitter)
    th.start()
    remaining = nreq
    while remaining:
        progressed = False
        for i in range(nreq):
            t = tickets[i]
            if t is None or lat[i] is not None:
                continue
            st, out, _, l = lib.tn_serve_poll(ctx.handle, t)
            if st == lib.TN_PENDING:
                continue
            assert st == lib.TN_OK, (i, st)
            lat[i] = l
            done_at[i] = time.perf_counter()
            results[i] = complex(np.asarray(out).reshape(-1)[0])
            remaining -= 1
            progressed = True
        if not progressed:
            time.sleep(2e-4)
    th.join()
    w0 = start + warmup_s
    win = [i for i in range(nreq) if t_sub[i] >= w0]
    lw = np.array([lat[i] for i in win])
    achieved = len(win) / (max(done_at[i] for i in win) - w0)
    work = sum(reqs[i][4] for i in win)
    # alone against the mix, on requests spread over the window
    pick = [win[int(k)] for k in np.linspace(0, len(win) - 1, min(check, len(win)))]
    worst = 0.0
    for i in pick:
        c, z, p, ovr, cs = reqs[i]
        alone = complex(np.asarray(lib.tn_contract(p, ovr)[0]).reshape(-1)[0])
        n = pool[c][0].n
        floor = 2.0 ** (-n / 2) if z == 0 else 1.0
        worst = max(worst, abs(results[i] - alone) / max(abs(alone) if z == 0 else 0.0, floor))
    for row in plans:
        for kind, net, ij, p, cs in row:
            ctx.free_plan(p)
    return dict(offered_per_s=rate, requests_measured=len(win), warmup_s=warmup_s, measured_s=seconds,
                achieved_per_s=achieved, p50_ms=float(np.percentile(lw, 50) * 1e3),
                p99_ms=float(np.percentile(lw, 99) * 1e3), max_ms=float(lw.max() * 1e3),
                effective_tflops=8.0 * work / (max(done_at[i] for i in win) - w0) / 1e12,
                amplitude_share=float(np.mean([reqs[i][1] == 0 for i in win])),
                alone_vs_mix_checked=len(pick), alone_vs_mix_max_err=worst,
                error_metric="amplitudes: |a - a_alone| / max(|a_alone|, 2^(-n/2)); <ZZ>: absolute")


def gemm_phase_leg(lib, reps=3):
    """The largest configuration: 30-qubit random circuit (depth 20, 7 CX pairs
    per layer, 70 % nearest-neighbour), 8 SA partitions, largest intermediate
    2^27 complex64.  Per precision: event-timed GEMM phase (effective complex
    TFLOP/s and the fraction of the MFMA peak of the instruction it runs on),
    plain per-amplitude time, and the error of the sampled amplitudes against
    the oracle's state-vector values in tests/golden/config3_amplitudes.json."""
    from paper_2507_20667_amd.inputs import amplitude_network, amplitude_overrides, random_circuit
    from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
    from paper_2507_20667_amd.planner.plan import tree_partition
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "config3_amplitudes.json")))
    c = gold["circuit"]
    circ = random_circuit(c["n"], c["depth"], c["seed"], cx_per_layer=c["cx_per_layer"],
                          p_nn=c["p_nn"])
    net = amplitude_network(circ, 0)
    t0 = time.perf_counter()
    plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 8), 8,
                               SAConfig(iterations=8, seed=0))
    plan_s = time.perf_counter() - t0
    ctx = lib.Context(48 << 30)  # the concurrent layout holds every partition's peak at once
    # what the matrix cores sustain on this device with no memory traffic, on
    # operands that change from product to product (the GEMM's ceiling) and
    # on constant ones (the top clock)
    probe = {"fp32": lib.tn_probe_mfma(ctx.handle, lib.TN_PREC_FP32),
             "bf16x3": lib.tn_probe_mfma(ctx.handle, lib.TN_PREC_BF16X3)}
    probe_const = {"fp32": lib.tn_probe_mfma(ctx.handle, lib.TN_PREC_FP32 | lib.TN_PROBE_CONST_OPERANDS),
                   "bf16x3": lib.tn_probe_mfma(ctx.handle, lib.TN_PREC_BF16X3 | lib.TN_PROBE_CONST_OPERANDS)}
    out = {"workload": f"random circuit {c['n']} qubits depth {c['depth']} seed {c['seed']}, "
                       f"{c['cx_per_layer']} CX pairs per layer (p_nn {c['p_nn']}), single-amplitude "
                       "networks, 8 SA partitions", "planning_s": plan_s,
           "mfma_probe_tflops": probe, "mfma_probe_const_operands_tflops": probe_const}
    # bf16 MFMA operations per effective complex flop: 4M = 12 products of
    # 2 flops per 8 effective flops, 3M = 9 products
    for name, flags, peak, mul in [("fp32_4m", 0, MFMA_PEAK_TFLOPS["fp32"], 1.0),
                                   ("fp32_3m", lib.TN_FORM_3M, MFMA_PEAK_TFLOPS["fp32"], 0.75),
                                   ("bf16x3_4m", lib.TN_PREC_BF16X3, MFMA_PEAK_TFLOPS["bf16x3"], 3.0),
                                   ("bf16x3_3m", lib.TN_PREC_BF16X3 | lib.TN_FORM_3M,
                                    MFMA_PEAK_TFLOPS["bf16x3"], 2.25)]:
        p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 8, plan.tree, None, flags)
        costs = lib.tn_plan_costs_get(p)
        worst = 0.0
        for x in gold["bitstrings"]:
            got, _ = lib.tn_contract(p, amplitude_overrides(net, circ, x))
            ref = complex(*gold["amplitudes"][str(x)])
            worst = max(worst, abs(complex(np.asarray(got).reshape(-1)[0]) - ref)
                        / max(abs(ref), 2.0 ** (-c["n"] / 2)))
        ovr = amplitude_overrides(net, circ, 0)
        t1 = time.perf_counter()
        for _ in range(reps):
            lib.tn_contract(p, ovr)
        amp_ms = (time.perf_counter() - t1) / reps * 1e3
        # the same plain call with the partitions side by side (TN_FLAG_CONCURRENT)
        lib.tn_contract(p, ovr, flags=lib.TN_FLAG_CONCURRENT)
        t1 = time.perf_counter()
        for _ in range(reps):
            lib.tn_contract(p, ovr, flags=lib.TN_FLAG_CONCURRENT)
        camp_ms = (time.perf_counter() - t1) / reps * 1e3
        # the same amplitude through the batched path (one query): the small
        # vertices run in the subtree kernel instead of one launch each
        lib.tn_contract_batch(ctx.handle, [(p, ovr)], [()])
        t1 = time.perf_counter()
        for _ in range(reps):
            bo, _, _ = lib.tn_contract_batch(ctx.handle, [(p, ovr)], [()])
        bamp_ms = (time.perf_counter() - t1) / reps * 1e3
        lib.tn_profile_enable(ctx.handle, True)
        lib.tn_profile_read(ctx.handle, reset=True)
        for _ in range(reps):
            lib.tn_contract(p, ovr)
        lib.tn_profile_enable(ctx.handle, False)
        st = lib.tn_profile_read(ctx.handle, reset=True)
        g = st["gemm"]
        eff = g["algo_flops"] / g["seconds"] / 1e12
        ach = probe["fp32" if name.startswith("fp32") else "bf16x3"]
        out[name] = {"gemm_effective_tflops": eff, "mfma_peak_tflops": peak,
                     "mfma_util": eff * mul / peak, "mfma_frac_of_achievable": eff * mul / ach,
                     "gemm_ms_per_amplitude": g["seconds"] / reps * 1e3,
                     "gemm_launches_per_amplitude": g["launches"] // reps,
                     "gemm_small_ms_per_amplitude": st["gemm_small"]["seconds"] / reps * 1e3,
                     "plain_ms_per_amplitude": amp_ms,
                     "plain_concurrent_ms_per_amplitude": camp_ms,
                     "con_serial_over_con_par": float(costs["con_serial"]) / float(costs["con_par"]),
                     "batched_ms_per_amplitude": bamp_ms,
                     "permute_ms_per_amplitude": st["permute"]["seconds"] / reps * 1e3,
                     "permute_launches_per_amplitude": st["permute"]["launches"] // reps,
                     "permute_hbm_gbs": (st["permute"]["algo_bytes"] / st["permute"]["seconds"] / 1e9
                                         if st["permute"]["seconds"] else None),
                     "con_serial": costs["con_serial"],
                     "largest_intermediate": costs["largest_intermediate"],
                     "max_rel_err_vs_statevector": worst, "amplitudes_checked": len(gold["bitstrings"])}
        log(f"{name}: GEMM phase {eff:.1f} effective TFLOP/s ({out[name]['mfma_util']:.1%} of the "
            f"MFMA peak), {amp_ms:.2f} ms per amplitude ({camp_ms:.2f} concurrent partitions, "
            f"{bamp_ms:.2f} batched), max err {worst:.1e}")
        ctx.free_plan(p)
    ctx.close()
    return out


def batch_mix_leg(lib, queries=512, reps=3):
    """Uneven batch: 64 seeded circuits of the random family (n ~ U{12..26},
    depth ~ U{8..20}, floor(n/4) CX pairs per layer; a seed is skipped when
    the planned largest intermediate leaves [2^4, 2^24]), 4 SA partitions
    each, `queries` amplitude queries whose circuit follows a truncated
    Zipf(1.2) law over the 64 (bitstrings uniform).  Plain path (tn_contract
    per query) against one tn_contract_batch call over all of them; the
    executed flops of the batched call (shared parts once) come from the
    event-timed kernel classes."""
    import oracle
    from paper_2507_20667_amd.inputs import amplitude_overrides
    from paper_2507_20667_amd.planner.workloads import uneven_mix
    circs, idx, bits, plan_s = uneven_mix(queries)
    ctx = lib.Context(32 << 30)
    handles = [ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 4, plan.tree, None, 0)
               for _, net, plan in circs]
    costs = [lib.tn_plan_costs_get(h) for h in handles]
    cs = [c["con_serial"] for c in costs]
    qs = [(handles[i], amplitude_overrides(circs[i][1], circs[i][0], x)) for i, x in zip(idx, bits)]
    shapes = [()] * queries
    work = 8.0 * sum(cs[i] for i in idx)

    def amp(o, l2):
        return complex(o.reshape(-1)[0]) * 2.0 ** float(l2)

    outs, l2s, st = lib.tn_contract_batch(ctx.handle, qs, shapes)  # warm-up: layouts, programs
    assert all(int(x) == 0 for x in st), st
    t1 = time.perf_counter()
    for _ in range(reps):
        outs, l2s, st = lib.tn_contract_batch(ctx.handle, qs, shapes)
    bt = (time.perf_counter() - t1) / reps
    # the same batch with each plan group's launch sequence captured once as a
    # HIP graph and replayed (the first call captures)
    og, l2g, st = lib.tn_contract_batch(ctx.handle, qs, shapes, flags=lib.TN_FLAG_GRAPH)
    assert all(int(x) == 0 for x in st), st
    t1 = time.perf_counter()
    for _ in range(reps):
        og, l2g, st = lib.tn_contract_batch(ctx.handle, qs, shapes, flags=lib.TN_FLAG_GRAPH)
    btg = (time.perf_counter() - t1) / reps
    gdiff = max(abs(amp(og[k], l2g[k]) - amp(outs[k], l2s[k])) for k in range(queries))
    lib.tn_profile_enable(ctx.handle, True)
    lib.tn_profile_read(ctx.handle, reset=True)
    lib.tn_contract_batch(ctx.handle, qs, shapes)
    lib.tn_profile_enable(ctx.handle, False)
    prof = lib.tn_profile_read(ctx.handle, reset=True)
    exec_flops = sum(v["algo_flops"] for v in prof.values())
    kern_s = sum(v["seconds"] for v in prof.values())
    plain, per_q = [], []
    for q in qs[:8]:
        lib.tn_contract(*q)
    t2 = time.perf_counter()
    for q in qs:
        t3 = time.perf_counter()
        plain.append(lib.tn_contract(*q))
        per_q.append(time.perf_counter() - t3)
    pt = time.perf_counter() - t2
    # the same single calls with the partitions side by side (TN_FLAG_CONCURRENT)
    for q in qs[:8]:
        lib.tn_contract(*q, flags=lib.TN_FLAG_CONCURRENT)
    conc, per_qc = [], []
    t2 = time.perf_counter()
    for q in qs:
        t3 = time.perf_counter()
        conc.append(lib.tn_contract(*q, flags=lib.TN_FLAG_CONCURRENT))
        per_qc.append(time.perf_counter() - t3)
    ptc = time.perf_counter() - t2
    conc_diff = max(float(np.max(np.abs(np.asarray(a[0]) - np.asarray(b[0])))) for a, b in zip(conc, plain))
    # the paper's cost model against measured time: per circuit, mean plain
    # time per amplitude against con_serial (Pearson r, linear and log-log)
    by_c = {}
    for k, i in enumerate(idx):
        by_c.setdefault(i, []).append(per_q[k])
    xs_ = np.array([float(cs[i]) for i in by_c])
    ys_ = np.array([float(np.median(v)) for v in by_c.values()])
    r_lin = float(np.corrcoef(xs_, ys_)[0, 1]) if len(by_c) > 2 else None
    r_log = float(np.corrcoef(np.log(xs_), np.log(ys_))[0, 1]) if len(by_c) > 2 else None
    # concurrency (f4): per circuit, the serial-over-concurrent time ratio
    # against the cost model's bound con_serial / con_par
    by_cc = {}
    for k, i in enumerate(idx):
        by_cc.setdefault(i, []).append(per_qc[k])
    tc_ = np.array([float(np.median(by_cc[i])) for i in by_c])
    bound = np.array([float(costs[i]["con_serial"]) / float(costs[i]["con_par"]) for i in by_c])
    cpar = np.array([float(costs[i]["con_par"]) for i in by_c])
    speed = ys_ / tc_
    diff = max(abs(amp(outs[k], l2s[k]) - amp(*plain[k])) / max(abs(amp(*plain[k])), 2.0 ** (-circs[i][0].n / 2))
               for k, i in enumerate(idx))
    # the oracle on the queries of the smallest circuits
    errs = []
    for k, i in enumerate(idx):
        circ, net, plan = circs[i]
        if circ.n > 16 or len(errs) >= 8:
            continue
        ref = complex(oracle.contract_tree(net.legs, net.dims, net.copy_with(qs[k][1]).tensors, plan.tree))
        errs.append(abs(amp(outs[k], l2s[k]) - ref) / max(abs(ref), 2.0 ** (-circ.n / 2)))
    ctx.close()
    out = {"workload": f"{queries} amplitude queries over 64 random-family circuits (12-26 qubits, "
                       "depth 8-20, floor(n/4) CX per layer), circuit ~ truncated Zipf(1.2), 4 SA "
                       "partitions each",
           "planning_s": plan_s, "queries": queries,
           "distinct_circuits_queried": len(set(idx)),
           "batched_amplitudes_per_s": queries / bt, "plain_amplitudes_per_s": queries / pt,
           "batched_graph_amplitudes_per_s": queries / btg, "graph_max_abs_diff": gdiff,
           "speedup_vs_plain": pt / bt,
           "effective_tflops_batched": work / bt / 1e12,
           "effective_tflops_plain": work / pt / 1e12,
           "executed_tflops_batched": exec_flops / bt / 1e12,
           "kernel_seconds_batched": kern_s, "wall_seconds_batched": bt,
           "max_rel_diff_batched_vs_plain": diff,
           "max_rel_err_vs_oracle": max(errs) if errs else None, "oracle_checked": len(errs),
           "concurrent_partitions": {
               "plain_amplitudes_per_s": queries / pt, "concurrent_amplitudes_per_s": queries / ptc,
               "speedup": pt / ptc, "max_abs_diff_vs_serial": conc_diff,
               "per_circuit_speedup_median": float(np.median(speed)),
               "per_circuit_speedup_range": [float(speed.min()), float(speed.max())],
               "con_serial_over_con_par_median": float(np.median(bound)),
               "con_serial_over_con_par_range": [float(bound.min()), float(bound.max())],
               "pearson_r_log_con_par_vs_concurrent_time":
                   float(np.corrcoef(np.log(cpar), np.log(tc_))[0, 1]) if len(by_c) > 2 else None,
               "pearson_r_log_con_serial_vs_concurrent_time":
                   float(np.corrcoef(np.log(xs_), np.log(tc_))[0, 1]) if len(by_c) > 2 else None},
           "cost_points": [(f"uneven circuit {i} ({circs[i][0].n} qubits, {len(circs[i][0].gates)} gates)",
                            int(cs[i]), roofline_seconds(circs[i][1], circs[i][2]),
                            float(np.median(by_c[i]))) for i in by_c],
           "cost_model_vs_time": {"circuits": len(by_c), "pearson_r_con_serial_vs_plain_time": r_lin,
                                  "pearson_r_log": r_log,
                                  "con_serial_range": [float(xs_.min()), float(xs_.max())],
                                  "plain_seconds_range": [float(ys_.min()), float(ys_.max())]}}
    log(f"batch mix: {out['batched_amplitudes_per_s']:.0f} amplitudes/s batched "
        f"({out['batched_graph_amplitudes_per_s']:.0f} with graphs) vs "
        f"{out['plain_amplitudes_per_s']:.0f} plain (x{out['speedup_vs_plain']:.1f}), "
        f"max diff {diff:.1e}, oracle err {out['max_rel_err_vs_oracle']}")
    cp = out["concurrent_partitions"]
    log(f"concurrent partitions: {cp['concurrent_amplitudes_per_s']:.0f} amplitudes/s vs "
        f"{cp['plain_amplitudes_per_s']:.0f} serial (x{cp['speedup']:.2f}; per circuit median "
        f"x{cp['per_circuit_speedup_median']:.2f}, con_serial/con_par median "
        f"{cp['con_serial_over_con_par_median']:.2f}), max diff {cp['max_abs_diff_vs_serial']}")
    return out


# bf16 (or f32) MFMA flops executed per effective complex flop (8 per complex
# multiply-add): FP32 4M 8, FP32 3M 6; BF16x3 4M twelve bf16 products of 2
# flops, 3M nine
EXEC_PER_EFFECTIVE = {("fp32", "4m"): 1.0, ("fp32", "3m"): 0.75, ("bf16x3", "4m"): 3.0,
                      ("bf16x3", "3m"): 2.25}
GEMM_KERNEL = {("fp32", "4m"): "k_cgemm_f32_planes<0>", ("fp32", "3m"): "k_cgemm_f32_planes<1>",
               ("bf16x3", "4m"): "k_cgemm_bf16x3_dma<0>", ("bf16x3", "3m"): "k_cgemm_bf16x3_dma<1>"}
GEMM_SOURCE = {"fp32": "gemm_f32.hip", "bf16x3": "gemm_bf16.hip"}


def traffic_record(name):
    """HBM bytes per launch of kernel `name` from the committed counter record
    (profiles/traffic.json), if its source is unchanged since the counters
    were taken; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(name)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


def roofline_seconds(net, plan):
    """Sum over the plan's vertices of the roofline time max(8 * 2^vc / P,
    8 (|c1| + |c2| + |v|) / BW): P the FP32 matrix peak, BW the HBM peak
    (complex64 operands read once, the result written once)."""
    from paper_2507_20667_amd.planner.cost import node_legs, node_weights, size_of
    legs = node_legs(net.legs, plan.tree)
    w = node_weights(net.legs, net.dims, plan.tree)
    nv = len(net.legs)
    t = 0.0
    for j, (a, b) in enumerate(plan.tree):
        nbytes = 8.0 * (size_of(legs[a], net.dims) + size_of(legs[b], net.dims) + size_of(legs[nv + j], net.dims))
        t += max(8.0 * w[j] / (MFMA_PEAK_TFLOPS["fp32"] * 1e12), nbytes / (HBM_PEAK_GBS * 1e9))
    return t


def cost_model_fit(points):
    """Pearson r of measured plain time per amplitude against con_serial and
    against the summed per-vertex roofline time (linear and log-log), over
    (name, con_serial, roofline seconds, measured seconds) points."""
    cs = np.array([float(p[1]) for p in points])
    rt = np.array([p[2] for p in points])
    tm = np.array([p[3] for p in points])

    def r(x, y):
        return float(np.corrcoef(x, y)[0, 1]) if len(x) > 2 else None
    return {"plans": len(points), "pearson_r_con_serial": r(cs, tm), "pearson_r_log_con_serial": r(np.log(cs), np.log(tm)),
            "pearson_r_roofline_time": r(rt, tm), "pearson_r_log_roofline_time": r(np.log(rt), np.log(tm)),
            "measured_over_roofline_median": float(np.median(tm / rt)),
            "points": [{"plan": p[0], "con_serial": p[1], "roofline_s": p[2], "plain_s": p[3]} for p in points]}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_random30(w, seconds):
    """The oracle (complex128 loop-nest contraction of the same network and
    tree) on a bounded sample of one 30-qubit amplitude: bound legs fixed
    (sliced) so that a slice holds 1/16 of the work, timed on all host cores;
    a slice of 1/128 of the work timed on one core.  Amplitudes/s = the
    measured multiply-add rate / con_serial of the whole amplitude (the rate
    of a slice, whose intermediates are 16 times smaller, taken as the rate of
    the whole; a whole amplitude takes minutes on the host)."""
    import oracle
    from paper_2507_20667_amd.inputs import amplitude_overrides, random_bitstrings
    from paper_2507_20667_amd.planner import cost
    from paper_2507_20667_amd.planner.slicing import choose_slices, sliced_problem
    net, plan, circ = w.net, w.plan, w.circ
    full = cost.con_serial(net.legs, net.dims, plan.tree)
    x = random_bitstrings(circ.n, 1, 4242)[0]
    tensors = net.copy_with(amplitude_overrides(net, circ, x)).tensors

    def slice_rate(target, threads):
        sl = choose_slices(net.legs, net.dims, plan.tree, target)
        d, base, ovrs = sliced_problem(net.legs, net.dims, tensors, sl)
        work = cost.con_serial(net.legs, d, plan.tree)
        ts = [ovrs[0].get(i, t) for i, t in enumerate(base)]
        t0 = time.perf_counter()
        oracle.contract_tree(net.legs, d, ts, plan.tree, nthreads=threads)
        dt = time.perf_counter() - t0
        return work / dt, len(sl), work, dt

    threads = oracle.default_threads()
    rate, nsl, work, dt = slice_rate(1 << 23, threads)
    rate1, nsl1, work1, dt1 = slice_rate(1 << 20, 1)
    return dict(value=rate / full, unit="amplitudes/s", cores=threads, kind="oracle",
                sample=f"one 30-qubit amplitude (bitstring {x}) with {nsl} bound legs fixed: one slice of "
                       f"{work} multiply-adds of the amplitude's {full} ({dt:.1f} s on {threads} threads), "
                       "complex128 loop-nest contraction of the same network and tree; amplitudes/s = "
                       "multiply-adds per second / con_serial",
                gmac_per_s=rate / 1e9, cpu_model=cpu_model(),
                single_thread={"value": rate1 / full, "unit": "amplitudes/s", "gmac_per_s": rate1 / 1e9,
                               "sample": f"{nsl1} legs fixed, {work1} multiply-adds, {dt1:.1f} s on 1 thread"})


def headline_random30(lib, torch, args):
    """The 30-qubit amplitudes through tn_contract_strided, `args.queries` per
    step, in the requested precision and form; the plain FP32 4M path on the
    same plan; event-timed kernel classes; state-vector parity."""
    from paper_2507_20667_amd.inputs import amplitude_overrides, output_tensor_ids, random_bitstrings
    from paper_2507_20667_amd.planner.workloads import random30
    w = random30()
    circ, net, plan = w.circ, w.net, w.plan
    n = circ.n
    log(f"30-qubit plan in {w.planning_s:.1f} s")
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "config3_amplitudes.json")))
    assert gold["circuit"]["n"] == n and gold["circuit"]["seed"] == 0
    prec, form = args.prec, args.form
    flags = (lib.TN_PREC_BF16X3 if prec == "bf16x3" else 0) | (lib.TN_FORM_3M if form == "3m" else 0)
    ctx = lib.Context(args.arena_gib << 30)
    p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 8, plan.tree, None, flags)
    costs = lib.tn_plan_costs_get(p)
    con_serial = costs["con_serial"]
    # the same plan without fused GEMM epilogues (host-side plan, no device
    # work): the permutations the fused epilogues take away
    os.environ["TN_GEMM_FUSE"] = "0"
    try:
        pu = lib.tn_plan_load(None, net.legs, net.dims, net.tensors, plan.partition_of, 8, plan.tree, None, flags)
        perms_unfused = lib.tn_plan_costs_get(pu)["num_permutations"]
        lib.tn_plan_free(pu)
    finally:
        del os.environ["TN_GEMM_FUSE"]
    ids = output_tensor_ids(net)
    Q, K, W = args.queries, args.steps, args.warmup

    def basis(xs):
        bits = np.array([[(x >> q) & 1 for q in range(n)] for x in xs], dtype=np.int64)
        h = np.zeros((len(xs), n, 2), dtype=np.complex64)
        h[np.arange(len(xs))[:, None], np.arange(n)[None, :], bits] = 1.0
        return torch.from_numpy(h).pin_memory()

    def make_call(dev, nq):
        arr = (lib.tn_leaf * n)()
        strides = (ctypes.c_int64 * n)()
        for i, t in enumerate(ids):
            arr[i] = lib.tn_leaf(t, dev.data_ptr() + i * 16, lib.TN_C64_DEVICE)
            strides[i] = n * 16
        out_t = torch.zeros((nq, 2), dtype=torch.float64, pin_memory=True)
        fn = lib.load().tn_contract_strided
        a = (ctypes.c_void_p(p), nq, n, ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(strides, ctypes.c_void_p),
             ctypes.c_void_p(out_t.data_ptr()), 1, lib.TN_C128, None, 0)

        def call():
            rc = fn(*a)
            if rc != 0:
                raise lib.TnError(rc, lib.tn_last_error())
            return out_t.numpy()
        call.keep = (arr, strides, out_t)
        return call

    # parity: the nine stored state-vector amplitudes through the same call
    gx = gold["bitstrings"]
    gdev = basis(gx).to("cuda")
    res = make_call(gdev, len(gx))()
    errs = []
    for i, x in enumerate(gx):
        ref = complex(*gold["amplitudes"][str(x)])
        errs.append(abs(complex(res[i, 0], res[i, 1]) - ref) / max(abs(ref), 2.0 ** (-n / 2)))
    max_err = max(errs)
    tol = 1e-5 if prec == "fp32" else 1e-3
    log(f"30-qubit {prec} {form}: max error {max_err:.2e} over {len(gx)} stored amplitudes")
    # the timed steps: the basis vectors of each step go host -> device inside
    # the step (pinned host memory, the context's stream), then one call
    hosts = [basis(random_bitstrings(n, Q, 5000 + s)) for s in range(K + W)]
    devs = [torch.empty_like(h, device="cuda") for h in hosts]
    calls = [make_call(d, Q) for d in devs]
    for s in range(W):
        devs[s].copy_(hosts[s], non_blocking=True)
        calls[s]()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(W, W + K):
        devs[s].copy_(hosts[s], non_blocking=True)
        calls[s]()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    amps = Q * K / dt
    # the same steps on the plan loaded without the tuning table (the
    # built-in launch heuristics)
    os.environ["TN_TUNE_OFF"] = "1"
    try:
        p_tuned = p
        p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 8, plan.tree, None, flags)
    finally:
        del os.environ["TN_TUNE_OFF"]
    calls_off = [make_call(d, Q) for d in devs]
    for s in range(W):
        calls_off[s]()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(W, W + K):
        devs[s].copy_(hosts[s], non_blocking=True)
        calls_off[s]()
    torch.cuda.synchronize()
    amps_untuned = Q * K / (time.perf_counter() - t0)
    ctx.free_plan(p)
    p = p_tuned
    # the same steps with every kernel launch bracketed by events
    lib.tn_profile_enable(ctx.handle, True)
    lib.tn_profile_read(ctx.handle, reset=True)
    for s in range(W, W + K):
        calls[s]()
    lib.tn_profile_enable(ctx.handle, False)
    stats = lib.tn_profile_read(ctx.handle, reset=True)
    g = stats["gemm"]
    mul = EXEC_PER_EFFECTIVE[(prec, form)]
    peak = MFMA_PEAK_TFLOPS[prec]
    eff = g["algo_flops"] / g["seconds"] / 1e12
    achieved = eff * mul
    nl = max(g["launches"], 1)
    kname = GEMM_KERNEL[(prec, form)]
    traffic = traffic_record(kname)
    ach = lib.tn_probe_mfma(ctx.handle, lib.TN_PREC_FP32 if prec == "fp32" else lib.TN_PREC_BF16X3)
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic, "kernel": kname,
            "achievable_tflops": ach, "frac_of_achievable": achieved / ach,
            "launches": g["launches"], "avg_launch_us": g["seconds"] / nl * 1e6,
            "algo_flops_per_launch": g["algo_flops"] / nl * mul,
            "algo_bytes_per_launch": g["algo_bytes"] / nl,
            "effective_tflops": eff,
            "note": "achieved = MFMA flops of the form (8 M N K for 4M, 6 M N K for 3M, times 3 or 2.25 "
                    "bf16 products for BF16x3) per launch / event-timed average launch, the split-k "
                    "reduction of the one split vertex included; achievable_tflops = the rate the matrix "
                    "cores sustain on this device with no memory traffic on operands that change from "
                    "product to product (tn_probe_mfma)"}
    perm = stats["permute"]
    perm_gbs = perm["algo_bytes"] / perm["seconds"] / 1e9 if perm["seconds"] else None
    kern_s = sum(v["seconds"] for v in stats.values())
    # the plain FP32 4M path (tn_contract, one query at a time, one launch per
    # vertex) on the same network and plan
    pp = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 8, plan.tree, None, 0)
    ovr0 = amplitude_overrides(net, circ, gx[1])
    lib.tn_contract(pp, ovr0)
    t1 = time.perf_counter()
    for x in gx[1:4]:
        lib.tn_contract(pp, amplitude_overrides(net, circ, x))
    plain = 3 / (time.perf_counter() - t1)
    ctx.free_plan(pp)
    cost_point = (w.name, int(con_serial), roofline_seconds(net, plan), 1.0 / plain)
    ctx.close()
    from paper_2507_20667_amd.tune import DEFAULT_OUT
    rec = {"amplitudes_per_s": amps, "ms_per_step": dt / K * 1e3, "queries_per_step": Q,
           "untuned_amplitudes_per_s": amps_untuned, "tuning_table": os.path.exists(DEFAULT_OUT),
           "effective_tflops": 8.0 * con_serial * amps / 1e12,
           "executed_tflops": sum(v["algo_flops"] for v in stats.values()) * mul / K / (dt / K) / 1e12,
           "plain_fp32_amplitudes_per_s": plain, "speedup_vs_plain_fp32": amps / plain,
           "max_rel_err_vs_statevector": max_err, "tolerance": tol, "amplitudes_checked": len(gx),
           "roofline": roof,
           "permute": {"hbm_gbs": perm_gbs, "frac_of_hbm": perm_gbs / HBM_PEAK_GBS if perm_gbs else None,
                       "launches": perm["launches"], "ms_per_step": perm["seconds"] / K * 1e3,
                       "algo_bytes_per_step": perm["algo_bytes"] / K,
                       "note": "algorithmic bytes: 8 read + 8 written per complex entry for float "
                               "planes, 8 + 2 per bf16 plane; the operands of the three largest GEMMs "
                               "are written as planes by the GEMM before them (fused epilogues), so the "
                               "permutations left are of 2^20 to 2^25 entries (the permutation kernel's "
                               "rate on 2^27-entry operands: 4.1 TB/s, with TN_GEMM_FUSE=0)"},
           "kernel_seconds_per_step": kern_s / K,
           "kernel_classes": {k: v for k, v in stats.items() if v["launches"]},
           "con_serial": con_serial, "con_dist": costs["con_dist"],
           "largest_intermediate": costs["largest_intermediate"], "planning_s": w.planning_s,
           "permutations_per_amplitude": costs["num_permutations"],
           "permutations_per_amplitude_without_fused_epilogues": perms_unfused,
           "workload": w.name, "overrides": "host basis vectors copied to the device inside each step",
           "cost_point": cost_point}
    log(f"30-qubit {prec} {form}: {amps:.1f} amplitudes/s ({dt / K * 1e3:.1f} ms per step of {Q}), "
        f"plain FP32 {plain:.1f}/s, GEMM {achieved:.1f} TFLOP/s ({achieved / peak:.1%}), "
        f"permutations {perm_gbs or 0:.0f} GB/s")
    return w, rec


def brickwork_leg(lib, torch, args):
    """20-qubit brickwork, `args.bw_queries` amplitudes per step through
    tn_contract_strided (overrides resident in device memory before the timed
    region; the same with the host-to-device upload inside the step beside
    it), tn_contract_batch and the plain path; every result of the first step
    against the state vector; the batch subtree kernel's roofline position."""
    import oracle
    from paper_2507_20667_amd.inputs import random_bitstrings
    from paper_2507_20667_amd.planner.workloads import brickwork20
    w = brickwork20()
    circ, net, plan = w.circ, w.net, w.plan
    n = circ.n
    ctx = lib.Context(16 << 30)
    p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 4, plan.tree, None, 0)
    costs = lib.tn_plan_costs_get(p)
    Q, K, W = args.bw_queries, args.bw_steps, 3
    steps_bits = [random_bitstrings(n, Q, 1000 + s) for s in range(K + W)]
    devs, calls, bcalls = [], [], []
    for s in range(K + W):
        dev, leaves = device_overrides(torch, net, n, steps_bits[s])
        devs.append((dev, leaves))
        calls.append(strided_call(lib, p, dev, net, n))
        bcalls.append(batch_call(lib, ctx.handle, p, leaves, n))
    torch.cuda.synchronize()
    res = calls[0]()
    psi = oracle.statevector(circ)
    ref = psi[np.array(steps_bits[0], dtype=np.int64)]
    got = res[:, 0] + 1j * res[:, 1]
    max_err = float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 2.0 ** (-n / 2))))

    def timed(fns, pre=None):
        for s in range(W):
            fns[s]()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(W, W + K):
            if pre:
                pre(s)
            fns[s]()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    dt = timed(calls)
    hosts = [d[0].cpu().pin_memory() for d in devs]
    dtu = timed(calls, lambda s: devs[s][0].copy_(hosts[s], non_blocking=True))
    dtb = timed(bcalls)
    dev0, leaves0 = devs[W]
    P = min(args.plain_queries, Q)
    plain_out = np.zeros(2, dtype=np.float64)
    l2 = ctypes.c_double()
    L = lib.load()
    for qi in range(min(3, P)):
        L.tn_contract(ctypes.c_void_p(p), n, ctypes.cast(leaves0[qi], ctypes.c_void_p),
                      plain_out.ctypes.data_as(ctypes.c_void_p), lib.TN_C128, ctypes.byref(l2), 0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for qi in range(P):
        rc = L.tn_contract(ctypes.c_void_p(p), n, ctypes.cast(leaves0[qi], ctypes.c_void_p),
                           plain_out.ctypes.data_as(ctypes.c_void_p), lib.TN_C128, ctypes.byref(l2), 0)
        assert rc == 0, lib.tn_last_error()
    torch.cuda.synchronize()
    plain_amps = P / (time.perf_counter() - t1)
    lib.tn_profile_enable(ctx.handle, True)
    lib.tn_profile_read(ctx.handle, reset=True)
    for s in range(W, W + K):
        calls[s]()
    lib.tn_profile_enable(ctx.handle, False)
    stats = lib.tn_profile_read(ctx.handle, reset=True)
    ctx.close()
    tb = stats["tree_batch"]
    nl = max(tb["launches"], 1)
    t_launch = tb["seconds"] / nl
    bytes_l, flops_l = tb["algo_bytes"] / nl, tb["algo_flops"] / nl
    # roofline bound of the batch subtree kernel: the larger of its byte time
    # at the HBM peak and its flop time at the attainable FP32 vector rate
    t_bytes = bytes_l / (HBM_PEAK_GBS * 1e9)
    t_flops = flops_l / (FP32_VALU_ATTAINABLE_TFLOPS * 1e12)
    roof = {"bound": "hbm" if t_bytes >= t_flops else "alu",
            "achieved": bytes_l / t_launch / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": max(t_bytes, t_flops) / t_launch, "traffic": traffic_record("k_tree_wave"),
            "kernel": "k_tree_wave", "launches": tb["launches"], "avg_launch_us": t_launch * 1e6,
            "algo_bytes_per_launch": bytes_l, "algo_flops_per_launch": flops_l,
            "alu_tflops": flops_l / t_launch / 1e12,
            "alu_frac_of_attainable": flops_l / t_launch / 1e12 / FP32_VALU_ATTAINABLE_TFLOPS}
    rec = {"workload": w.name + f", {Q} bitstrings per step", "amplitudes_per_s": Q * K / dt,
           "ms_per_step": dt / K * 1e3, "steps": K,
           "overrides": "device-resident before the timed region (basis vectors read in place)",
           "amplitudes_per_s_with_upload": Q * K / dtu,
           "batch_api_amplitudes_per_s": Q * K / dtb, "plain_amplitudes_per_s": plain_amps,
           "speedup_vs_plain": (Q * K / dt) / plain_amps,
           "effective_tflops": 8.0 * costs["con_serial"] * Q * K / dt / 1e12,
           "max_rel_err_vs_statevector": max_err, "results_checked": Q,
           "roofline": roof, "con_serial": costs["con_serial"],
           "largest_intermediate": costs["largest_intermediate"], "planning_s": w.planning_s,
           "kernel_classes": {k: v for k, v in stats.items() if v["launches"]},
           "cost_point": (w.name, int(costs["con_serial"]), roofline_seconds(net, plan), 1.0 / plain_amps)}
    log(f"brickwork: {rec['amplitudes_per_s']:.3e} amplitudes/s ({rec['ms_per_step']:.3f} ms per step), "
        f"with upload {rec['amplitudes_per_s_with_upload']:.3e}, plain {plain_amps:.0f}/s, "
        f"max err {max_err:.1e} over {Q}; k_tree_wave {roof['avg_launch_us']:.1f} us, frac {roof['frac']:.2f}")
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--queries", type=int, default=8, help="30-qubit amplitudes per step")
    ap.add_argument("--prec", choices=["fp32", "bf16x3"], default="fp32")
    ap.add_argument("--form", choices=["4m", "3m"], default="3m")
    ap.add_argument("--arena-gib", type=int, default=48)
    ap.add_argument("--bw-queries", type=int, default=4096)
    ap.add_argument("--bw-steps", type=int, default=20)
    ap.add_argument("--plain-queries", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 512 MiB device-to-device copy (known traffic) so "
                         "that hardware byte counters can be scaled against it")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="measured window of the serving leg (0 skips it)")
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--no-brickwork", action="store_true", help="skip the 20-qubit brickwork leg")
    ap.add_argument("--no-largest", action="store_true",
                    help="skip the 30-qubit GEMM-phase leg (every precision and form)")
    ap.add_argument("--no-mix", action="store_true", help="skip the uneven 64-circuit batch leg")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}, WORLD_SIZE={world}): this "
              "build measures one MI355X; a run on several GPUs would place the partitions on "
              "different devices and exchange partition results on the reduction path.",
              file=sys.stderr)
        sys.exit(2)

    # the serving pool is planned first, in forked processes, before anything
    # touches the GPU
    pool = plan_s = None
    if args.serve_seconds > 0:
        pool, plan_s = serve_pool(processes=min(16, os.cpu_count() or 1))
        log(f"serving pool planned in {plan_s:.1f} s")

    import torch
    from paper_2507_20667_amd import lib

    if args.copy_calibration:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w, head = headline_random30(lib, torch, args)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_random30(w, 10.0)
        log(f"oracle: {cpu['value']:.4f} amplitudes/s on {cpu['cores']} threads "
            f"({cpu['gmac_per_s']:.2f} GMAC/s), one thread {cpu['single_thread']['value']:.5f}/s")
    bw = None if args.no_brickwork else brickwork_leg(lib, torch, args)
    largest = None if args.no_largest else gemm_phase_leg(lib)
    mix = None if args.no_mix else batch_mix_leg(lib)
    serve = serve_bf16 = None
    if args.serve_seconds > 0:
        torch.cuda.empty_cache()
        free, total = torch.cuda.mem_get_info()
        arena = int(min(free - (4 << 30), 256 << 30)) // 256 * 256
        sctx = lib.Context(arena)
        desc = ("128 random-family circuits (n ~ U{12..32}, depth ~ U{8..24}, n/4 CX pairs per layer), "
                "amplitude + 2 <Z_i Z_j> networks each (light-cone pruned), 4 partitions each, largest "
                "intermediate <= 2^32, con_serial <= 2^36; Poisson arrivals, circuit ~ Zipf(1.1), 50/50 "
                f"amplitude/<ZZ>; arena {arena / 2**30:.0f} GiB (free memory - 4 GiB)")
        serve = serve_bench(lib, sctx, pool, 0, args.serve_rate, args.serve_warmup, args.serve_seconds)
        serve_bf16 = serve_bench(lib, sctx, pool, lib.TN_PREC_BF16X3 | lib.TN_FORM_3M, args.serve_rate,
                                 args.serve_warmup, args.serve_seconds, seed=1)
        for rec, name in ((serve, "fp32"), (serve_bf16, "bf16x3_3m")):
            rec.update(pool=desc, planning_s=plan_s, precision=name)
            log(f"serve {name}: offered {rec['offered_per_s']:.0f}/s, achieved {rec['achieved_per_s']:.0f}/s, "
                f"p50 {rec['p50_ms']:.2f} ms, p99 {rec['p99_ms']:.2f} ms, alone-vs-mix "
                f"{rec['alone_vs_mix_max_err']:.1e}")
        sctx.close()
    # the paper's cost model against MI355X time over every measured plan
    pts = [head.pop("cost_point")]
    if bw:
        pts.append(bw.pop("cost_point"))
    if mix:
        pts.extend(mix.pop("cost_points"))
    cost_fit = cost_model_fit(pts) if len(pts) > 2 else None
    out = {
        "metric": METRIC,
        "value": head["amplitudes_per_s"],
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": head["workload"] + f", {args.queries} bitstrings per step",
                   "precision": args.prec, "form": args.form, "queries_per_step": args.queries,
                   "con_serial": head["con_serial"], "con_dist": head["con_dist"],
                   "largest_intermediate": head["largest_intermediate"]},
        "effective_tflops": head["effective_tflops"],
        "executed_tflops": head["executed_tflops"],
        "plain_fp32_amplitudes_per_s": head["plain_fp32_amplitudes_per_s"],
        "speedup_vs_plain_fp32": head["speedup_vs_plain_fp32"],
        "max_rel_err": head["max_rel_err_vs_statevector"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "permute": head["permute"],
        "headline_detail": {k: v for k, v in head.items() if k not in ("roofline", "permute")},
        "brickwork20": bw,
        "largest_config_gemm_phase": largest,
        "uneven_batch": mix,
        "serve": serve,
        "serve_bf16x3": serve_bf16,
        "cost_model_vs_time": cost_fit,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
