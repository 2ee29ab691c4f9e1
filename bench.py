"""Throughput of partitioned tensor-network contraction on one MI355X.

Workload (default): the 20-qubit brickwork circuit of depth 14 (CZ brick
layers alternating with RX/RZ rotation layers, seed 0), one closed network per
output bitstring, 4 partitions refined by simulated annealing.  One step
contracts a batch of `--queries` amplitude queries (random bitstrings) through
the whole path: leaf overrides, every partition's tree in turn, the reduction
path and the FP64 final contraction.  The overrides of all steps are placed in
device memory before the timed region.

Printed: one JSON line with amplitudes/s of the batched path (`value`:
tn_contract_strided, the overridden output vectors read in place from one
device buffer; tn_contract_batch with per-query descriptors beside it), the
plain per-query path (tn_contract, one query at a time) for the same
workload, effective complex TFLOP/s (8 * con_serial per amplitude), the
roofline position of the dominant kernel class (event-timed inside this run)
the CPU oracle timed on a bounded sample, and (unless --no-largest) the GEMM
phase of the 30-qubit configuration in FP32 and three-term split BF16 with its
MFMA utilisation and its error against stored state-vector amplitudes.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--queries 4096]
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(args):
    from paper_2507_20667_amd.inputs import amplitude_network, brickwork_circuit
    from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
    from paper_2507_20667_amd.planner.plan import tree_partition
    circ = brickwork_circuit(20, 14, 0)
    net = amplitude_network(circ, 0)
    t0 = time.perf_counter()
    init = tree_partition(net.legs, net.dims, 4)
    plan = simulated_annealing(net.legs, net.dims, init, 4,
                               SAConfig(iterations=20, n_steps=32, workers=4, rg_samples=8, seed=0))
    return circ, net, plan, time.perf_counter() - t0


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


def serve_bench(lib, ctx, seconds, rate, flags, seed=0):
    """Poisson arrivals of amplitude and <Z_i Z_j> requests over a pool of
    seeded random circuits (12-22 qubits, depth 8-16, the 30-qubit family's
    generator with n/4 CX pairs per layer): p50/p99 of submit-to-ready latency,
    offered and achieved rates; then the same requests all at once
    (saturation throughput)."""
    import threading
    from paper_2507_20667_amd.inputs import (amplitude_network, amplitude_overrides,
                                             random_circuit, zz_network)
    from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
    from paper_2507_20667_amd.planner.plan import tree_partition
    rng = np.random.default_rng(seed)
    pool = []
    t0 = time.perf_counter()
    for c in range(8):
        n = int(rng.integers(12, 23))
        d = int(rng.integers(8, 17))
        circ = random_circuit(n, d, 100 + c)
        nets = [("amp", amplitude_network(circ, 0), None)]
        for _ in range(2):
            i, j = sorted(int(v) for v in rng.choice(n, 2, replace=False))
            nets.append(("zz", zz_network(circ, i, j), (i, j)))
        for kind, net, ij in nets:
            k = 2 if net.num_tensors < 200 else 4
            pl = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, k), k,
                                     SAConfig(iterations=3, n_steps=8, workers=2, rg_samples=4))
            p = ctx.plan_load(net.legs, net.dims, net.tensors, pl.partition_of, k, pl.tree, None,
                              flags)
            pool.append((kind, circ, net, p))
    plan_s = time.perf_counter() - t0
    amp_plans = [x for x in pool if x[0] == "amp"]
    zz_plans = [x for x in pool if x[0] == "zz"]
    nreq = max(1, int(seconds * rate))
    reqs = []
    for _ in range(nreq):
        if rng.random() < 0.5:
            kind, circ, net, p = amp_plans[int(rng.integers(0, len(amp_plans)))]
            x = int(rng.integers(0, 1 << circ.n))
            reqs.append((p, amplitude_overrides(net, circ, x)))
        else:
            kind, circ, net, p = zz_plans[int(rng.integers(0, len(zz_plans)))]
            reqs.append((p, {}))
    gaps = rng.exponential(1.0 / rate, size=nreq)

    def run(paced):
        tickets = [None] * nreq

        def submitter():
            t_next = time.perf_counter()
            for i, (p, ovr) in enumerate(reqs):
                if paced:
                    t_next += gaps[i]
                    while time.perf_counter() < t_next:
                        time.sleep(min(1e-3, max(0.0, t_next - time.perf_counter())))
                tickets[i] = lib.tn_serve_submit(ctx.handle, p, ovr)

        th = threading.Thread(target=submitter)
        start = time.perf_counter()
        th.start()
        lat = []
        done = 0
        while done < nreq:
            progressed = False
            for i in range(nreq):
                t = tickets[i]
                if t is None or t < 0:
                    continue
                st, out, _, l = lib.tn_serve_poll(ctx.handle, t)
                if st == lib.TN_PENDING:
                    continue
                tickets[i] = -1
                lat.append(l)
                done += 1
                progressed = True
            if not progressed:
                time.sleep(2e-4)
        th.join()
        wall = time.perf_counter() - start
        return np.array(lat), wall

    lat, wall = run(True)
    lat_s, wall_s = run(False)
    return dict(requests=nreq, offered_per_s=rate, achieved_per_s=nreq / wall,
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                saturated_per_s=nreq / wall_s,
                saturated_p50_ms=float(np.percentile(lat_s, 50) * 1e3),
                saturated_p99_ms=float(np.percentile(lat_s, 99) * 1e3),
                pool="8 random circuits 12-22 qubits depth 8-16 (n/4 CX per layer, 70% nearest-"
                     "neighbour), amplitude + 2 <ZZ> networks each, 50/50 mix",
                planning_s=plan_s)


KERNEL_SOURCES = {"tree": "tree.hip", "tree_batch": "tree.hip", "stream": "kernels.hip",
                  "permute": "kernels.hip", "dot": "kernels.hip", "gemm": "kernels.hip"}
KERNEL_NAMES = {"tree": "k_tree", "tree_batch": "k_tree_wave"}


def measured_traffic(cls, launches):
    """HBM bytes per launch from the committed counter record, if the kernel
    source is unchanged since the counters were taken (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    name = KERNEL_NAMES.get(cls)
    if not name or not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(name)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if sha != rec["source_sha256_16"]:
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


def roofline(stats, prec):
    """Roofline position of the kernel class with the largest event-timed
    share: achieved = algorithmic work per launch / average launch time."""
    dom = max(stats, key=lambda k: stats[k]["seconds"])
    ds = stats[dom]
    n = max(ds["launches"], 1)
    if dom == "gemm":
        achieved = ds["algo_flops"] / ds["seconds"] / 1e12
        peak = MFMA_PEAK_TFLOPS[prec]
        roof = dict(bound="mfma", achieved=achieved, peak=peak, unit="TFLOP/s")
    elif dom in ("tree", "tree_batch"):
        # every intermediate stays in LDS: its bound is arithmetic, not HBM
        achieved = ds["algo_flops"] / ds["seconds"] / 1e12
        peak = FP32_VECTOR_PEAK_TFLOPS
        roof = dict(bound="alu", achieved=achieved, peak=peak, unit="TFLOP/s")
    else:
        achieved = ds["algo_bytes"] / ds["seconds"] / 1e9
        peak = HBM_PEAK_GBS
        roof = dict(bound="hbm", achieved=achieved, peak=peak, unit="GB/s")
    roof["frac"] = achieved / peak
    roof["traffic"] = measured_traffic(dom, n)
    roof["kernel_class"] = dom
    roof["launches"] = ds["launches"]
    roof["avg_launch_us"] = ds["seconds"] / n * 1e6
    roof["algo_bytes_per_launch"] = ds["algo_bytes"] / n
    roof["algo_flops_per_launch"] = ds["algo_flops"] / n
    return roof


def cpu_baseline(net, plan, circ, budget_s):
    import oracle
    from paper_2507_20667_amd.inputs import amplitude_overrides, random_bitstrings
    threads = oracle.default_threads()
    xs = random_bitstrings(circ.n, 100000, 99)
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and done < len(xs):
        ovr = amplitude_overrides(net, circ, xs[done])
        oracle.contract_tree(net.legs, net.dims, net.copy_with(ovr).tensors, plan.tree,
                             nthreads=threads)
        done += 1
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="amplitudes/s", cores=threads, kind="oracle",
                sample=f"{done} amplitudes of the same 20-qubit brickwork network and plan, "
                       f"complex128 loop-nest contraction, {dt:.1f} s")


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
    out = {"workload": f"random circuit {c['n']} qubits depth {c['depth']} seed {c['seed']}, "
                       f"{c['cx_per_layer']} CX pairs per layer (p_nn {c['p_nn']}), single-amplitude "
                       "networks, 8 SA partitions", "planning_s": plan_s}
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
        out[name] = {"gemm_effective_tflops": eff, "mfma_peak_tflops": peak,
                     "mfma_util": eff * mul / peak, "gemm_ms_per_amplitude": g["seconds"] / reps * 1e3,
                     "gemm_launches_per_amplitude": g["launches"] // reps,
                     "plain_ms_per_amplitude": amp_ms,
                     "plain_concurrent_ms_per_amplitude": camp_ms,
                     "con_serial_over_con_par": float(costs["con_serial"]) / float(costs["con_par"]),
                     "batched_ms_per_amplitude": bamp_ms,
                     "permute_ms_per_amplitude": st["permute"]["seconds"] / reps * 1e3,
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
    from paper_2507_20667_amd.inputs import amplitude_network, amplitude_overrides, circuit_mix, zipf_indices
    from paper_2507_20667_amd.planner import SAConfig, simulated_annealing
    from paper_2507_20667_amd.planner.cost import largest_intermediate
    from paper_2507_20667_amd.planner.plan import tree_partition
    t0 = time.perf_counter()
    circs, seed = [], 0
    while len(circs) < 64:
        (s, circ), = circuit_mix(1, seed)
        seed += 1
        net = amplitude_network(circ, 0)
        plan = simulated_annealing(net.legs, net.dims, tree_partition(net.legs, net.dims, 4), 4,
                                   SAConfig(iterations=4, n_steps=16, workers=2, rg_samples=4, seed=s))
        li = largest_intermediate(net.legs, net.dims, plan.tree)
        if li > 1 << 24 or li < 1 << 4:
            continue
        circs.append((circ, net, plan))
    plan_s = time.perf_counter() - t0
    idx = zipf_indices(len(circs), queries, 1.2, 7)
    rng = np.random.default_rng(8)
    bits = [int(rng.integers(0, 1 << circs[i][0].n)) for i in idx]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--queries", type=int, default=4096)
    ap.add_argument("--plain-queries", type=int, default=64)
    ap.add_argument("--prec", choices=["fp32", "bf16x3"], default="fp32")
    ap.add_argument("--form", choices=["4m", "3m"], default="4m")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 512 MiB device-to-device copy (known traffic) so "
                         "that hardware byte counters can be scaled against it")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--no-largest", action="store_true",
                    help="skip the 30-qubit GEMM-phase leg")
    ap.add_argument("--no-mix", action="store_true",
                    help="skip the uneven 64-circuit batch leg")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}, WORLD_SIZE={world}): "
              "this build measures a single MI355X; see DESIGN.md for how the path shards.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_20667_amd import lib
    import oracle
    from paper_2507_20667_amd.inputs import amplitude_overrides, random_bitstrings

    if args.copy_calibration:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    circ, net, plan, plan_s = make_workload(args)
    n = circ.n
    log(f"planned in {plan_s:.1f}s: {plan.meta.get('con_dist')}")
    flags = (lib.TN_PREC_BF16X3 if args.prec == "bf16x3" else 0) | \
            (lib.TN_FORM_3M if args.form == "3m" else 0)
    ctx = lib.Context(16 << 30)
    p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 4, plan.tree, None, flags)
    costs = lib.tn_plan_costs_get(p)
    con_serial = costs["con_serial"]
    Q, K, W = args.queries, args.steps, args.warmup
    steps_bits = [random_bitstrings(n, Q, 1000 + s) for s in range(K + W)]
    devs, calls, bcalls = [], [], []
    for s in range(K + W):
        dev, leaves = device_overrides(torch, net, n, steps_bits[s])
        devs.append((dev, leaves))
        calls.append(strided_call(lib, p, dev, net, n))
        bcalls.append(batch_call(lib, ctx.handle, p, leaves, n))
    torch.cuda.synchronize()

    # parity spot check outside the timed region
    res = calls[0]()
    errs = []
    for qi in range(0, Q, max(1, Q // 8)):
        x = steps_bits[0][qi]
        ovr = amplitude_overrides(net, circ, x)
        ref = complex(oracle.contract_tree(net.legs, net.dims, net.copy_with(ovr).tensors,
                                           plan.tree))
        got = complex(res[qi, 0], res[qi, 1])
        errs.append(abs(got - ref) / max(abs(ref), 2.0 ** (-n / 2)))
    max_err = max(errs)
    log(f"spot-check max relative error {max_err:.2e}")

    for s in range(W):
        calls[s]()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(W, W + K):
        calls[s]()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    amps = Q * K / dt
    eff_tflops = 8.0 * con_serial * Q * K / dt / 1e12
    # the same steps through tn_contract_batch (one descriptor per query and leaf)
    for s in range(W):
        bcalls[s]()
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for s in range(W, W + K):
        bcalls[s]()
    torch.cuda.synchronize()
    batch_api_amps = Q * K / (time.perf_counter() - tb)

    # plain path: tn_contract, one query at a time, device-resident overrides
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
                           plain_out.ctypes.data_as(ctypes.c_void_p), lib.TN_C128,
                           ctypes.byref(l2), 0)
        assert rc == 0, lib.tn_last_error()
    torch.cuda.synchronize()
    plain_amps = P / (time.perf_counter() - t1)

    # event-timed kernel classes over the same steps
    lib.tn_profile_enable(ctx.handle, True)
    lib.tn_profile_read(ctx.handle, reset=True)
    for s in range(W, W + K):
        calls[s]()
    lib.tn_profile_enable(ctx.handle, False)
    stats = lib.tn_profile_read(ctx.handle, reset=True)
    roof = roofline(stats, args.prec)
    # executed work (vertices actually run, shared parts once) per unprofiled step time
    exec_tflops = sum(v["algo_flops"] for v in stats.values()) / K / (dt / K) / 1e12

    serve = serve_bf16 = None
    if args.serve_seconds > 0:
        serve = serve_bench(lib, ctx, args.serve_seconds, args.serve_rate, flags)
        serve_bf16 = serve_bench(lib, ctx, args.serve_seconds, args.serve_rate,
                                 lib.TN_PREC_BF16X3 | (lib.TN_FORM_3M if args.form == "3m" else 0))

    largest = None
    if not args.no_largest:
        largest = gemm_phase_leg(lib)

    mix = None
    if not args.no_mix:
        mix = batch_mix_leg(lib)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(net, plan, circ, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": amps,
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "brickwork 20 qubits depth 14 seed 0, single-amplitude networks "
                               f"(247 tensors), 4 SA partitions, {Q} bitstrings per step",
                   "form": args.form, "queries_per_step": Q,
                   "con_serial": con_serial, "con_dist": costs["con_dist"],
                   "largest_intermediate": costs["largest_intermediate"]},
        "effective_tflops": eff_tflops,
        "executed_tflops": exec_tflops,
        "batch_api_amplitudes_per_s": batch_api_amps,
        "plain_amplitudes_per_s": plain_amps,
        "speedup_vs_plain": amps / plain_amps,
        "max_rel_err": max_err,
        "planning_s": plan_s,
        "roofline": roof,
        "cpu_baseline": cpu,
        "serve": serve,
        "serve_bf16x3": serve_bf16,
        "largest_config_gemm_phase": largest,
        "uneven_batch": mix,
        "kernel_classes": {k: v for k, v in stats.items() if v["launches"]},
    }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
