"""Autotuner: times launch choices on the GPU and writes the tuning table
(tune.json beside libtn.so) that tn_plan_load reads.

    python -m paper_2507_20667_amd.tune [--out PATH] [--quick]

GEMM vertices (the G of TTGT, Section 5.1): every GEMM shape of the 30-qubit
plan in FP32 and split BF16 (4M and 3M) and of the uneven batch's plans, in
buckets of ceil(log2) of M, N and K.  Candidates: the FP32 plane kernel's
tile shape (128 x 128; 64 x 256 when M <= 128; 256 x 64 when N <= 128), the
BF16x3 4M tile (128 x 128; 128 x 256 or 256 x 128 on the two wave-group
kernel) and the number of k chunks (1 to 32, each chunk at least 256 deep).  Each candidate
runs a network of that one GEMM vertex (A[m, k] B[k, n], closed by C[m, n],
seeded random entries) with TN_GEMM_FORCE, and the event-timed GEMM launches
are compared (median of three after a warm-up).

Subtree kernel (the batched path of the small vertices): for the 20-qubit
brickwork plan, queries per workgroup, the size from which a per-query
intermediate lives in device memory, and the size limit of packed gate
steps, timed on 4096-query strided calls.

Every entry keeps the time of its choice and of the built-in heuristic's,
so the table states what tuning gained.  Choices are only launch shapes:
results are the same up to the order of additions in a split k.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tune.json")


def _ceil_log2(x: int) -> int:
    return max(0, (int(x) - 1).bit_length())


class _Stderr:
    """Captures what the library writes to file descriptor 2."""

    def __enter__(self):
        sys.stderr.flush()
        self.f = tempfile.TemporaryFile(mode="w+b")
        self.saved = os.dup(2)
        os.dup2(self.f.fileno(), 2)
        return self

    def __exit__(self, *exc):
        os.dup2(self.saved, 2)
        os.close(self.saved)
        self.f.seek(0)
        self.text = self.f.read().decode(errors="replace")
        self.f.close()


def gemm_shapes(lib, net, plan, k, flags):
    """(M, N, K) of every GEMM vertex of a plan (from the library's own
    schedule, host-only load)."""
    os.environ["TN_DEBUG"] = "1"
    try:
        with _Stderr() as cap:
            p = lib.tn_plan_load(None, net.legs, net.dims, net.tensors, plan.partition_of, k, plan.tree,
                                 None, flags)
            lib.tn_plan_free(p)
    finally:
        del os.environ["TN_DEBUG"]
    out = []
    for line in cap.text.splitlines():
        if "gemm vertex" in line:
            w = line.split()
            out.append((int(w[w.index("M") + 1]), int(w[w.index("N") + 1]), int(w[w.index("K") + 1])))
    return out


_OPERANDS = {}


def _operands(M, N, K):
    """Seeded random tensors of one GEMM shape (entries uniform in the unit
    square around 0), made once per shape.  Random, not constant: the clock
    the device holds under a matrix-core load depends on how many operand
    bits switch, so constant data would time a faster device than real
    data meets."""
    key = (M, N, K)
    if key not in _OPERANDS:
        _OPERANDS.clear()
        rng = np.random.default_rng(M * 1000003 + N * 1009 + K)

        def r(*sh):
            x = np.empty(sh, dtype=np.complex64)
            x.real = rng.random(sh, dtype=np.float32) - 0.5
            x.imag = rng.random(sh, dtype=np.float32) - 0.5
            return x
        _OPERANDS[key] = [r(M, K), r(K, N), r(M, N)]
    return _OPERANDS[key]


def time_gemm(lib, ctx, M, N, K, flags, force, reps=3):
    """Event-timed GEMM launches (ms) of the network A[m,k] B[k,n] C[m,n]
    with TN_GEMM_FORCE = force (None: the heuristic)."""
    legs = [[1, 2], [2, 3], [1, 3]]
    dims = {1: M, 2: K, 3: N}
    ts = _operands(M, N, K)
    if force is not None:
        os.environ["TN_GEMM_FORCE"] = f"{force[0]},{force[1]}"
    try:
        p = ctx.plan_load(legs, dims, ts, [0, 0, 1], 2, [(0, 1), (3, 2)], None, flags, lib.TN_C64)
    finally:
        os.environ.pop("TN_GEMM_FORCE", None)
    try:
        lib.tn_contract(p)
        times = []
        for _ in range(reps):
            lib.tn_profile_enable(ctx.handle, True)
            lib.tn_profile_read(ctx.handle, reset=True)
            lib.tn_contract(p)
            st = lib.tn_profile_read(ctx.handle, reset=True)
            lib.tn_profile_enable(ctx.handle, False)
            times.append((st["gemm"]["seconds"] + st["gemm_small"]["seconds"]) * 1e3)
        return float(np.median(times))
    finally:
        ctx.free_plan(p)


def gemm_candidates(M, N, K, bf16, form3m):
    if bf16:
        tiles = [0] if form3m else [0, 1, 2]
    else:
        tiles = [0] + ([1] if M <= 128 else []) + ([2] if N <= 128 else [])
    ks = [s for s in (1, 2, 4, 8, 16, 32) if s == 1 or K // s >= 256]
    return [(t, s) for t in tiles for s in ks]


def tune_gemm(lib, quick=False):
    from .planner.workloads import random30, uneven_mix
    w = random30()
    combos = [("fp32", "4m", 0), ("fp32", "3m", lib.TN_FORM_3M),
              ("bf16x3", "4m", lib.TN_PREC_BF16X3), ("bf16x3", "3m", lib.TN_PREC_BF16X3 | lib.TN_FORM_3M)]
    buckets = {}
    for prec, form, flags in combos:
        for (M, N, K) in gemm_shapes(lib, w.net, w.plan, 8, flags):
            key = (prec, form, _ceil_log2(M), _ceil_log2(N), _ceil_log2(K))
            buckets.setdefault(key, (M, N, K, flags))
    if not quick:
        circs, idx, bits, _ = uneven_mix()
        for prec, form, flags in combos[:2]:
            for circ, net, plan in circs:
                for (M, N, K) in gemm_shapes(lib, net, plan, 4, flags):
                    if K % 16 == 0 and M * N * K >= 1 << 20:   # plane kernels, worth a launch
                        key = (prec, form, _ceil_log2(M), _ceil_log2(N), _ceil_log2(K))
                        buckets.setdefault(key, (M, N, K, flags))
    rules = []
    with lib.Context(24 << 30) as ctx:
        for key, (M, N, K, flags) in sorted(buckets.items()):
            if K % 16 or M * N * K < 1 << 16:
                continue        # not on the plane kernels, or too small to matter
            prec, form = key[0], key[1]
            base = time_gemm(lib, ctx, M, N, K, flags, None)
            best, best_t = None, base
            for cand in gemm_candidates(M, N, K, prec == "bf16x3", form == "3m"):
                t = time_gemm(lib, ctx, M, N, K, flags, cand)
                if t < best_t * 0.98:
                    best, best_t = cand, t
            print(f"[tune] {prec} {form} M {M} N {N} K {K}: heuristic {base:.3f} ms, "
                  f"best {best} {best_t:.3f} ms", file=sys.stderr, flush=True)
            if best is not None:
                rules.append(dict(prec=prec, form=form, lm=key[2], ln=key[3], lk=key[4], tile=best[0],
                                  ksplit=best[1], shape=[M, N, K], ms=best_t, default_ms=base))
    return rules


def tune_tree(lib, torch, quick=False):
    from .inputs import output_tensor_ids, random_bitstrings
    from .planner.workloads import brickwork20
    w = brickwork20()
    net, plan, n = w.net, w.plan, w.circ.n
    Q = 4096
    xs = random_bitstrings(n, Q, 1000)
    bits = np.array([[(x >> q) & 1 for q in range(n)] for x in xs], dtype=np.int64)
    host = np.zeros((Q, n, 2), dtype=np.complex64)
    host[np.arange(Q)[:, None], np.arange(n)[None, :], bits] = 1.0
    dev = torch.from_numpy(host).to("cuda")
    ids = output_tensor_ids(net)
    arr = (lib.tn_leaf * n)()
    strides = (ctypes.c_int64 * n)()
    for i, t in enumerate(ids):
        arr[i] = lib.tn_leaf(t, dev.data_ptr() + i * 16, lib.TN_C64_DEVICE)
        strides[i] = n * 16
    out = torch.zeros((Q, 2), dtype=torch.float64, pin_memory=True)

    def run(ctx, knobs):
        saved = {}
        for k, v in knobs.items():
            saved[k] = os.environ.get(k)
            os.environ[k] = str(v)
        try:
            p = ctx.plan_load(net.legs, net.dims, net.tensors, plan.partition_of, 4, plan.tree)
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        fp = lib.tn_plan_costs_get(p)["fingerprint"]
        fn = lib.load().tn_contract_strided
        a = (ctypes.c_void_p(p), Q, n, ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(strides, ctypes.c_void_p),
             ctypes.c_void_p(out.data_ptr()), 1, lib.TN_C128, None, 0)
        for _ in range(3):
            assert fn(*a) == 0, lib.tn_last_error()
        ts = []
        for _ in range(15):
            t0 = time.perf_counter()
            assert fn(*a) == 0, lib.tn_last_error()
            ts.append(time.perf_counter() - t0)
        ctx.free_plan(p)
        return float(np.median(ts)) * 1e3, fp

    with lib.Context(16 << 30) as ctx:
        base, fp = run(ctx, {})
        best, best_t = None, base
        grid = [(qw, sp, pk) for qw in (0, 8) for sp in (256, 512, 1024, 4096) for pk in (64, 128)]
        if quick:
            grid = grid[:4]
        for qw, sp, pk in grid:
            t, _ = run(ctx, {"TN_TREE_QW": qw, "TN_TREE_SPILL": sp, "TN_TREE_PACK_NC": pk})
            print(f"[tune] brickwork qw {qw} spill {sp} pack {pk}: {t:.4f} ms (heuristic {base:.4f})",
                  file=sys.stderr, flush=True)
            if t < best_t * 0.98:
                best, best_t = (qw, sp, pk), t
    rules = []
    if best is not None:
        rules.append(dict(fingerprint=fp, qw=best[0], spill=best[1], pack_nc=best[2], workload=w.name,
                          ms=best_t, default_ms=base))
    return rules, dict(workload=w.name, fingerprint=fp, default_ms=base, best=best, best_ms=best_t)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    # measure the heuristics and the candidates, never an older table
    os.environ["TN_TUNE_FILE"] = "off"
    import torch
    from . import lib
    t0 = time.perf_counter()
    gemm = tune_gemm(lib, args.quick)
    tree, tree_summary = tune_tree(lib, torch, args.quick)
    table = dict(device="gfx950", generated_by="python -m paper_2507_20667_amd.tune",
                 seconds=time.perf_counter() - t0, gemm=gemm, tree=tree, tree_searched=tree_summary)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(dict(out=args.out, gemm_rules=len(gemm), tree_rules=len(tree))))


if __name__ == "__main__":
    main()
