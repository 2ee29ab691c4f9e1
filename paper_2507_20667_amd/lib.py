"""ctypes binding of libtn (include/tn.h).

Argument marshalling only: every step of a contraction runs in libtn's HIP
kernels.  The functions carry the C names; `Context` adds the one convenience
of taking its arena from a torch device tensor and its stream from torch.

If libtn.so is missing this module raises on first use: there is no other
code path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtn.so")

TN_OK, TN_PENDING = 0, 1
TN_E_INVALID_ARG, TN_E_INVALID_PLAN, TN_E_NOMEM, TN_E_DEVICE = -1, -2, -3, -4
TN_E_AGAIN, TN_E_CANCELLED, TN_E_UNKNOWN_TICKET = -5, -6, -7
TN_C64, TN_C128, TN_C64_DEVICE = 0, 1, 2
TN_PREC_FP32, TN_PREC_BF16X3 = 0, 1
TN_FORM_4M, TN_FORM_3M = 0, 1 << 4
TN_FLAG_KEEP_SCALE = 1 << 8
TN_FLAG_GRAPH = 1 << 9
TN_FLAG_CONCURRENT = 1 << 10
TN_PROBE_CONST_OPERANDS = 1 << 8   # tn_probe_mfma only

STATUS_NAMES = {0: "TN_OK", 1: "TN_PENDING", -1: "TN_E_INVALID_ARG", -2: "TN_E_INVALID_PLAN",
                -3: "TN_E_NOMEM", -4: "TN_E_DEVICE", -5: "TN_E_AGAIN", -6: "TN_E_CANCELLED",
                -7: "TN_E_UNKNOWN_TICKET"}

EXPORTED = ["tn_ctx_create", "tn_ctx_destroy", "tn_last_error", "tn_plan_load",
            "tn_plan_costs_get", "tn_plan_free", "tn_contract", "tn_contract_batch", "tn_contract_strided",
            "tn_contract_strided_noalloc", "tn_plan_slice", "tn_serve_submit", "tn_serve_poll",
            "tn_profile_enable", "tn_profile_read", "tn_probe_mfma"]


class TnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class tn_plan_desc(ctypes.Structure):
    _fields_ = [("num_tensors", ctypes.c_int32),
                ("rank", ctypes.c_void_p),
                ("legs", ctypes.c_void_p),
                ("leg_dims", ctypes.c_void_p),
                ("data", ctypes.c_void_p),
                ("data_dtype", ctypes.c_int),
                ("partition_of", ctypes.c_void_p),
                ("num_partitions", ctypes.c_int32),
                ("tree", ctypes.c_void_p),
                ("output_legs", ctypes.c_void_p),
                ("num_output_legs", ctypes.c_int32)]


class tn_plan_costs(ctypes.Structure):
    _fields_ = [("con_serial", ctypes.c_uint64 * 2), ("con_par", ctypes.c_uint64 * 2),
                ("con_dist", ctypes.c_uint64 * 2), ("mem_elems", ctypes.c_uint64 * 2),
                ("live_peak_bytes", ctypes.c_uint64),
                ("largest_intermediate_elems", ctypes.c_uint64),
                ("num_internal_nodes", ctypes.c_int32), ("num_gemm_nodes", ctypes.c_int32),
                ("num_tiny_nodes", ctypes.c_int32), ("num_stream_nodes", ctypes.c_int32),
                ("num_permutations", ctypes.c_int32), ("fingerprint", ctypes.c_uint64)]


class tn_leaf(ctypes.Structure):
    _fields_ = [("tensor", ctypes.c_int32), ("data", ctypes.c_void_p), ("dtype", ctypes.c_int)]


class tn_query(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("num_overrides", ctypes.c_int32),
                ("overrides", ctypes.c_void_p)]


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2507_20667_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        P, I32, U32, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
        sig = {
            "tn_ctx_create": [P, SZ, P, U32, P],
            "tn_ctx_destroy": [P],
            "tn_plan_load": [P, P, U32, P],
            "tn_plan_costs_get": [P, P],
            "tn_plan_free": [P],
            "tn_contract": [P, I32, P, P, ctypes.c_int, P, U32],
            "tn_contract_batch": [P, I32, P, P, ctypes.c_int, P, P, U32],
            "tn_contract_strided": [P, I32, I32, P, P, P, ctypes.c_int64, ctypes.c_int, P, U32],
            "tn_contract_strided_noalloc": [P, I32, I32, P, P, P, ctypes.c_int64, U32],
            "tn_plan_slice": [P, I32, P, ctypes.c_int64, P],
            "tn_probe_mfma": [P, U32, P],
            "tn_serve_submit": [P, P, P],
            "tn_serve_poll": [P, ctypes.c_uint64, P, ctypes.c_int, P, P],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        lib.tn_last_error.argtypes = []
        lib.tn_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def tn_last_error() -> str:
    return load().tn_last_error().decode(errors="replace")


def _check(st):
    if st < 0:
        raise TnError(st, tn_last_error())
    return st


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------------ context

def tn_ctx_create(arena_ptr: int, arena_bytes: int, stream_ptr: int = 0, flags: int = 0):
    out = ctypes.c_void_p()
    _check(load().tn_ctx_create(ctypes.c_void_p(arena_ptr), arena_bytes,
                                ctypes.c_void_p(stream_ptr), flags, ctypes.byref(out)))
    return out.value


def tn_ctx_destroy(ctx):
    _check(load().tn_ctx_destroy(ctypes.c_void_p(ctx)))


# -------------------------------------------------------------------- plans

def tn_plan_load(ctx, legs, dims, tensors, partition_of, num_partitions, tree,
                 output_legs=None, flags: int = 0, data_dtype: int = TN_C128):
    """legs: list of label lists; dims: label -> dimension; tensors: arrays in
    leg order; tree: SSA pairs.  ctx None loads a host-only plan."""
    nv = len(legs)
    rank = np.array([len(l) for l in legs], dtype=np.int32)
    lab = np.array([x for l in legs for x in l] or [0], dtype=np.int64)
    ld = np.array([dims[x] for l in legs for x in l] or [1], dtype=np.int64)
    npdt = np.complex128 if data_dtype == TN_C128 else np.complex64
    arrs = [np.ascontiguousarray(t, dtype=npdt) for t in tensors]
    ptrs = (ctypes.c_void_p * max(1, nv))(*[a.ctypes.data for a in arrs])
    po = np.ascontiguousarray(partition_of, dtype=np.int32)
    tr = np.array([x for pr in tree for x in pr] or [0], dtype=np.int32)
    ol = np.array(list(output_legs or []) or [0], dtype=np.int64)
    d = tn_plan_desc(nv, _p(rank).value, _p(lab).value, _p(ld).value,
                     ctypes.cast(ptrs, ctypes.c_void_p).value, data_dtype, _p(po).value,
                     num_partitions, _p(tr).value,
                     _p(ol).value if output_legs else None, len(output_legs or []))
    out = ctypes.c_void_p()
    _check(load().tn_plan_load(ctypes.c_void_p(ctx) if ctx else None, ctypes.byref(d), flags,
                               ctypes.byref(out)))
    return out.value


def _u128(a):
    return (int(a[0]) << 64) | int(a[1])


def tn_plan_costs_get(plan) -> dict:
    c = tn_plan_costs()
    _check(load().tn_plan_costs_get(ctypes.c_void_p(plan), ctypes.byref(c)))
    return dict(con_serial=_u128(c.con_serial), con_par=_u128(c.con_par),
                con_dist=_u128(c.con_dist), mem=_u128(c.mem_elems),
                live_peak_bytes=int(c.live_peak_bytes),
                largest_intermediate=int(c.largest_intermediate_elems),
                num_internal_nodes=c.num_internal_nodes, num_gemm_nodes=c.num_gemm_nodes,
                num_tiny_nodes=c.num_tiny_nodes, num_stream_nodes=c.num_stream_nodes,
                num_permutations=c.num_permutations, fingerprint=f"{c.fingerprint:016x}")


def tn_plan_free(plan):
    _check(load().tn_plan_free(ctypes.c_void_p(plan)))


def tn_plan_slice(plan, labels=(), max_intermediate=0):
    """A sliced copy of a loaded plan: the given bound legs fixed, or legs
    chosen until no intermediate exceeds max_intermediate entries."""
    lab = np.array(list(labels) or [0], dtype=np.int64)
    out = ctypes.c_void_p()
    _check(load().tn_plan_slice(ctypes.c_void_p(plan), len(labels), _p(lab), int(max_intermediate),
                                ctypes.byref(out)))
    return out.value


# -------------------------------------------------------------- contraction

def _leaves(overrides):
    keep = []
    arr = (tn_leaf * max(1, len(overrides)))()
    for i, (t, data) in enumerate(sorted(overrides.items())):
        a = np.ascontiguousarray(data, dtype=np.complex128)
        keep.append(a)
        arr[i] = tn_leaf(int(t), a.ctypes.data, TN_C128)
    return arr, keep


def tn_contract(plan, overrides=None, result_shape=(), out_dtype=TN_C128, flags=0):
    """Returns (result array, log2 scale)."""
    overrides = overrides or {}
    arr, keep = _leaves(overrides)
    out = np.zeros(result_shape, dtype=np.complex128 if out_dtype == TN_C128 else np.complex64)
    out = np.ascontiguousarray(out)
    l2 = ctypes.c_double(0.0)
    _check(load().tn_contract(ctypes.c_void_p(plan), len(overrides), ctypes.cast(arr, ctypes.c_void_p),
                              _p(out), out_dtype, ctypes.byref(l2), flags))
    return out, l2.value


def tn_contract_batch(ctx, queries, result_shapes, out_dtype=TN_C128, flags=0):
    """queries: list of (plan, overrides dict).  Returns (results, log2 scales,
    per-query statuses)."""
    n = len(queries)
    qarr = (tn_query * max(1, n))()
    keep = []
    outs = []
    for i, (plan, ovr) in enumerate(queries):
        arr, k = _leaves(ovr or {})
        keep.append((arr, k))
        qarr[i] = tn_query(plan, len(ovr or {}), ctypes.cast(arr, ctypes.c_void_p).value)
        outs.append(np.zeros(result_shapes[i], dtype=np.complex128 if out_dtype == TN_C128
                             else np.complex64))
    optrs = (ctypes.c_void_p * max(1, n))(*[o.ctypes.data for o in outs])
    l2 = np.zeros(max(1, n), dtype=np.float64)
    st = np.zeros(max(1, n), dtype=np.int32)
    _check(load().tn_contract_batch(ctypes.c_void_p(ctx), n, ctypes.cast(qarr, ctypes.c_void_p),
                                    ctypes.cast(optrs, ctypes.c_void_p), out_dtype, _p(l2), _p(st),
                                    flags))
    return outs, l2[:n], st[:n]


def tn_contract_strided(plan, num_queries, overrides, result_shape=(), out_dtype=TN_C128, flags=0,
                        out=None, out_stride=None, scales=True):
    """overrides: list of (tensor id, data, stride bytes, dtype) where data is a
    numpy array holding every query's copy (its base address is query 0's) or
    a device address (int) with dtype TN_C64_DEVICE.  Returns (results of
    shape (num_queries,) + result_shape, log2 scales).  out: an array to write
    the results into instead (query q's at element q * out_stride, out_stride
    defaulting to a result's size; pinned host memory lets the kernels write
    complex128 results there themselves), returned as given; scales=False asks
    for no log2 scales (None returned)."""
    n = len(overrides)
    arr = (tn_leaf * max(1, n))()
    strides = (ctypes.c_int64 * max(1, n))()
    keep = []
    for i, (t, data, stride, dt) in enumerate(overrides):
        if isinstance(data, np.ndarray):
            a = np.ascontiguousarray(data)
            keep.append(a)
            ptr = a.ctypes.data
        else:
            ptr = int(data)
        arr[i] = tn_leaf(int(t), ptr, dt)
        strides[i] = int(stride)
    res = int(np.prod(result_shape)) if result_shape else 1
    stride = res if out_stride is None else int(out_stride)
    if out is None:
        out = np.zeros((num_queries,) + tuple(result_shape),
                       dtype=np.complex128 if out_dtype == TN_C128 else np.complex64)
        stride = res
    else:
        want = np.complex128 if out_dtype == TN_C128 else np.complex64
        if out.dtype != want or not out.flags.c_contiguous or out.size < max(0, num_queries - 1) * stride + res:
            raise ValueError("out: wrong dtype, not contiguous or too small")
    l2 = np.zeros(max(1, num_queries), dtype=np.float64) if scales else None
    _check(load().tn_contract_strided(ctypes.c_void_p(plan), int(num_queries), n,
                                      ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(strides, ctypes.c_void_p),
                                      _p(out), ctypes.c_int64(stride), out_dtype,
                                      _p(l2) if scales else None, flags))
    return out, (l2[:num_queries] if scales else None)


def tn_contract_strided_noalloc(plan, num_queries, overrides, out_ptr, out_stride=1):
    """overrides: list of (tensor id, device address, stride bytes); out_ptr:
    device address of num_queries complex128 results (out_stride elements
    apart).  Allocates nothing."""
    n = len(overrides)
    arr = (tn_leaf * max(1, n))()
    strides = (ctypes.c_int64 * max(1, n))()
    for i, (t, ptr, stride) in enumerate(overrides):
        arr[i] = tn_leaf(int(t), int(ptr), TN_C64_DEVICE)
        strides[i] = int(stride)
    _check(load().tn_contract_strided_noalloc(ctypes.c_void_p(plan), int(num_queries), n,
                                              ctypes.cast(arr, ctypes.c_void_p),
                                              ctypes.cast(strides, ctypes.c_void_p),
                                              ctypes.c_void_p(int(out_ptr)), ctypes.c_int64(out_stride), 0))


def tn_serve_submit(ctx, plan, overrides=None) -> int:
    overrides = overrides or {}
    arr, keep = _leaves(overrides)
    q = tn_query(plan, len(overrides), ctypes.cast(arr, ctypes.c_void_p).value)
    t = ctypes.c_uint64()
    _check(load().tn_serve_submit(ctypes.c_void_p(ctx), ctypes.byref(q), ctypes.byref(t)))
    return t.value


def tn_serve_poll(ctx, ticket, result_shape=(), out_dtype=TN_C128, keep_scale=False):
    """Returns (status, result or None, log2 scale, latency seconds).  With
    keep_scale the result is the mantissa and the scale is returned apart."""
    out = np.zeros(result_shape, dtype=np.complex128 if out_dtype == TN_C128 else np.complex64)
    l2 = ctypes.c_double(0.0)
    lat = ctypes.c_double(0.0)
    st = load().tn_serve_poll(ctypes.c_void_p(ctx), ctypes.c_uint64(ticket), _p(out), out_dtype,
                              ctypes.byref(l2) if keep_scale else None, ctypes.byref(lat))
    if st < 0:
        raise TnError(st, tn_last_error())
    return st, (out if st == TN_OK else None), l2.value, lat.value


# --------------------------------------------------------- torch plumbing

class Context:
    """A libtn context whose arena is a torch uint8 device tensor and whose
    stream is torch's current stream on `device`."""

    def __init__(self, arena_bytes: int, device: str = "cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libtn needs a GPU; torch.cuda.is_available() is False")
        load()
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.handle = tn_ctx_create(self.arena.data_ptr(), arena_bytes, self.stream.cuda_stream)
        self.plans = []

    def load_network(self, net, partition_of, num_partitions, tree, flags=0):
        p = tn_plan_load(self.handle, net.legs, net.dims, net.tensors, partition_of,
                         num_partitions, tree, net.output_legs or None, flags)
        self.plans.append(p)
        return p

    def plan_load(self, legs, dims, tensors, partition_of, num_partitions, tree,
                  output_legs=None, flags=0, data_dtype=TN_C128):
        p = tn_plan_load(self.handle, legs, dims, tensors, partition_of, num_partitions, tree,
                         output_legs, flags, data_dtype)
        self.plans.append(p)
        return p

    def slice_plan(self, p, labels=(), max_intermediate=0):
        s = tn_plan_slice(p, labels, max_intermediate)
        self.plans.append(s)
        return s

    def free_plan(self, p):
        tn_plan_free(p)
        self.plans.remove(p)

    def close(self):
        for p in list(self.plans):
            tn_plan_free(p)
        self.plans = []
        if self.handle:
            tn_ctx_destroy(self.handle)
            self.handle = None
        self.arena = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ------------------------------------------------------------------ timing

KCLASS_NAMES = ["stream", "permute", "gemm", "dot", "tree", "tree_batch", "gemm_small"]


class tn_kernel_stats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("seconds", ctypes.c_double),
                ("algo_bytes", ctypes.c_double), ("algo_flops", ctypes.c_double)]


def tn_probe_mfma(ctx, precision) -> float:
    """TFLOP/s the matrix cores sustain with no memory traffic
    (TN_PREC_FP32: the FP32 MFMA; TN_PREC_BF16X3: the bf16 MFMA), on operands
    that change from product to product, or, with TN_PROBE_CONST_OPERANDS
    or-ed in, on constant ones."""
    t = ctypes.c_double(0.0)
    _check(load().tn_probe_mfma(ctypes.c_void_p(ctx), int(precision), ctypes.byref(t)))
    return t.value


def tn_profile_enable(ctx, enable=True):
    f = load().tn_profile_enable
    f.argtypes = [ctypes.c_void_p, ctypes.c_int]
    f.restype = ctypes.c_int32
    _check(f(ctypes.c_void_p(ctx), 1 if enable else 0))


def tn_profile_read(ctx, reset=True) -> dict:
    f = load().tn_profile_read
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    f.restype = ctypes.c_int32
    arr = (tn_kernel_stats * len(KCLASS_NAMES))()
    _check(f(ctypes.c_void_p(ctx), ctypes.cast(arr, ctypes.c_void_p), 1 if reset else 0))
    return {KCLASS_NAMES[i]: dict(launches=int(arr[i].launches), seconds=arr[i].seconds,
                                  algo_bytes=arr[i].algo_bytes, algo_flops=arr[i].algo_flops)
            for i in range(len(KCLASS_NAMES))}
