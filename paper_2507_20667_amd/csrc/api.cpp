// C entry points of libtn (declared in include/tn.h).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>

#include <atomic>
#include <string>
#include <thread>

#include "tn_internal.h"

using namespace tn;

// The calling thread's resources for tn_contract*: the context's stream,
// staging and profiler (these calls are serialized by exec_mu).
static ExecRes ctx_res(tn_ctx *ctx) {
  ExecRes r;
  r.st = ctx->stream;
  r.pinned = &ctx->pinned;
  r.pinned_bytes = &ctx->pinned_bytes;
  r.prof = &ctx->prof;
  return r;
}

extern "C" {

const char *tn_last_error(void) { return tn::last_error(); }

tn_status tn_ctx_create(void *arena_dev_ptr, size_t arena_bytes, void *hip_stream, uint32_t flags,
                        tn_ctx **out) {
  if (!out || !arena_dev_ptr || arena_bytes < 4096 || ((uintptr_t)arena_dev_ptr & 255) || flags) {
    set_error("tn_ctx_create: need a 256-byte aligned arena of at least 4 KiB, flags = 0");
    return TN_E_INVALID_ARG;
  }
  tn_ctx *c = new (std::nothrow) tn_ctx;
  if (!c) {
    set_error("out of host memory");
    return TN_E_NOMEM;
  }
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    set_error("hipGetDevice failed");
    return TN_E_DEVICE;
  }
  c->arena.init((uint8_t *)arena_dev_ptr, arena_bytes);
  c->stream = (hipStream_t)hip_stream;
  // budget of the shared-part cache: TN_CACHE_BYTES, else an eighth of the
  // arena up to 8 GiB (0 turns the cache off)
  {
    const char *cb = getenv("TN_CACHE_BYTES");
    c->rcache_budget = cb ? (size_t)strtoull(cb, nullptr, 10)
                          : std::min<size_t>(arena_bytes / 8, (size_t)8 << 30);
  }
  // this device's static scratch (tn_contract_strided_noalloc); without it
  // that call reports an error, every other call works as before
  void *sp = nullptr;
  if (scratch_address(c->device, &sp) == hipSuccess)
    c->scratch = (uint8_t *)sp;
  else
    (void)hipGetLastError();
  *out = c;
  return TN_OK;
}

tn_status tn_ctx_destroy(tn_ctx *ctx) {
  if (!ctx) {
    set_error("tn_ctx_destroy: NULL context");
    return TN_E_INVALID_ARG;
  }
  serve_shutdown(ctx);
  if (ctx->live_plans.load() > 0) {
    set_error("tn_ctx_destroy: %d plan(s) of this context are still loaded", ctx->live_plans.load());
    return TN_E_INVALID_ARG;
  }
  hipStreamSynchronize(ctx->stream);
  if (ctx->pinned) hipHostFree(ctx->pinned);
  if (ctx->graph_st) {
    hipStreamSynchronize(ctx->graph_st);
    hipStreamDestroy(ctx->graph_st);
  }
  if (ctx->graph_ev) hipEventDestroy(ctx->graph_ev);
  for (auto &l : ctx->lanes) {
    if (l.st) {
      hipStreamSynchronize(l.st);
      hipStreamDestroy(l.st);
    }
    if (l.pinned) hipHostFree(l.pinned);
  }
  if (ctx->lanes_ev) hipEventDestroy(ctx->lanes_ev);
  for (size_t k = 0; k < ctx->part_st.size(); ++k) {
    hipStreamSynchronize(ctx->part_st[k]);
    hipStreamDestroy(ctx->part_st[k]);
    hipEventDestroy(ctx->part_ev[k]);
  }
  if (ctx->part_ev0) hipEventDestroy(ctx->part_ev0);
  ctx->prof.destroy();
  delete ctx;
  return TN_OK;
}

tn_status tn_profile_enable(tn_ctx *ctx, int enable) {
  if (!ctx) {
    set_error("tn_profile_enable: NULL context");
    return TN_E_INVALID_ARG;
  }
  std::lock_guard<std::mutex> g(ctx->exec_mu);
  ctx->prof.on = enable != 0;
  return TN_OK;
}

tn_status tn_profile_read(tn_ctx *ctx, tn_kernel_stats *out, int reset) {
  if (!ctx || !out) {
    set_error("tn_profile_read: NULL argument");
    return TN_E_INVALID_ARG;
  }
  std::lock_guard<std::mutex> g(ctx->exec_mu);
  memcpy(out, ctx->prof.stats, sizeof(ctx->prof.stats));
  if (reset) memset(ctx->prof.stats, 0, sizeof(ctx->prof.stats));
  return TN_OK;
}

tn_status tn_probe_mfma(tn_ctx *ctx, uint32_t precision, double *tflops) {
  const uint32_t p = precision & ~(uint32_t)TN_PROBE_CONST_OPERANDS;
  if (!ctx || !tflops || (p != TN_PREC_FP32 && p != TN_PREC_BF16X3)) {
    set_error("tn_probe_mfma: NULL argument or precision not TN_PREC_FP32 / TN_PREC_BF16X3");
    return TN_E_INVALID_ARG;
  }
  const bool random = (precision & TN_PROBE_CONST_OPERANDS) == 0;
  std::lock_guard<std::mutex> g(ctx->exec_mu);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
      cus < 1) {
    set_error("tn_probe_mfma: compute unit count unavailable");
    return TN_E_DEVICE;
  }
  const int blocks = 4 * cus;  // four blocks of four waves per CU: four waves per SIMD
  const size_t bytes = Arena::round((size_t)blocks * 256 * sizeof(float));
  const int64_t off = ctx->arena.alloc(bytes);
  if (off < 0) {
    set_error("tn_probe_mfma: arena cannot hold %zu bytes", bytes);
    return TN_E_NOMEM;
  }
  float *buf = (float *)(ctx->arena.base() + off);
  const int prec = p == TN_PREC_FP32 ? kPrecFP32 : kPrecBF16x3;
  // about 40 ms: long enough for the clock to settle where a long GEMM runs
  const int iters = prec == kPrecFP32 ? 100000 : 200000;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double flops = 0.0;
  float ms = 0.0f;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch_probe_mfma(ctx->stream, prec, random, buf, blocks, 64, &flops);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
  if (e == hipSuccess) e = launch_probe_mfma(ctx->stream, prec, random, buf, blocks, iters, &flops);
  if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(ctx->stream);
  ctx->arena.release(off, bytes);
  if (e != hipSuccess || ms <= 0.0f) {
    set_error("tn_probe_mfma: %s", hipGetErrorString(e));
    return TN_E_DEVICE;
  }
  *tflops = flops / ((double)ms * 1e9);
  return TN_OK;
}

tn_status tn_plan_load(tn_ctx *ctx, const tn_plan_desc *desc, uint32_t flags, tn_plan **out) {
  if (!out) {
    set_error("tn_plan_load: out is NULL");
    return TN_E_INVALID_ARG;
  }
  *out = nullptr;
  const uint32_t known = TN_PREC_BF16X3 | TN_FORM_3M;
  if (flags & ~known) {
    set_error("tn_plan_load: unknown flag bits 0x%x", flags & ~known);
    return TN_E_INVALID_ARG;
  }
  tn_plan *p = new (std::nothrow) tn_plan;
  if (!p) {
    set_error("out of host memory");
    return TN_E_NOMEM;
  }
  p->flags = flags;
  tn_status st = build_plan(p, desc);
  if (st != TN_OK) {
    delete p;
    return st;
  }
  if (ctx) {
    std::lock_guard<std::mutex> g(ctx->exec_mu);
    p->ctx = ctx;
    p->dev_leaf_bytes = std::max<size_t>(p->leaf_host.size() * sizeof(float2), 256);
    p->dev_desc_bytes = std::max<size_t>(p->desc_blob.size(), 256);
    p->dev_leaf = ctx->arena.alloc(p->dev_leaf_bytes, true);
    p->dev_desc = ctx->arena.alloc(p->dev_desc_bytes, true);
    if (p->dev_leaf < 0 || p->dev_desc < 0) {
      ctx->arena.release(p->dev_leaf, p->dev_leaf_bytes, true);
      ctx->arena.release(p->dev_desc, p->dev_desc_bytes, true);
      delete p;
      set_error("tn_plan_load: arena cannot hold the leaves and descriptors");
      return TN_E_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(ctx->arena.base() + p->dev_leaf, p->leaf_host.data(),
                                  p->leaf_host.size() * sizeof(float2), hipMemcpyHostToDevice,
                                  ctx->stream);
    if (e == hipSuccess && !p->desc_blob.empty())
      e = hipMemcpyAsync(ctx->arena.base() + p->dev_desc, p->desc_blob.data(), p->desc_blob.size(),
                         hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      ctx->arena.release(p->dev_leaf, p->dev_leaf_bytes, true);
      ctx->arena.release(p->dev_desc, p->dev_desc_bytes, true);
      delete p;
      set_error("tn_plan_load: upload failed: %s", hipGetErrorString(e));
      return TN_E_DEVICE;
    }
    ctx->live_plans++;
  }
  *out = p;
  return TN_OK;
}

static void put128(uint64_t *dst, u128 v) {
  dst[0] = (uint64_t)(v >> 64);
  dst[1] = (uint64_t)v;
}

tn_status tn_plan_costs_get(const tn_plan *p, tn_plan_costs *out) {
  if (!p || !out) {
    set_error("tn_plan_costs_get: NULL argument");
    return TN_E_INVALID_ARG;
  }
  memset(out, 0, sizeof(*out));
  put128(out->con_serial, p->con_serial);
  put128(out->con_par, p->con_par);
  put128(out->con_dist, p->con_dist);
  put128(out->mem_elems, p->mem);
  out->live_peak_bytes = (uint64_t)p->plain.peak_intermediate;
  out->largest_intermediate_elems = (uint64_t)p->largest;
  out->num_internal_nodes = p->nv - 1;
  out->num_gemm_nodes = p->num_gemm;
  out->num_tiny_nodes = p->num_tiny;
  out->num_stream_nodes = p->num_stream;
  out->num_permutations = p->num_perm;
  out->fingerprint = p->fingerprint;
  return TN_OK;
}

tn_status tn_plan_free(tn_plan *p) {
  if (!p) {
    set_error("tn_plan_free: NULL plan");
    return TN_E_INVALID_ARG;
  }
  if (p->ctx && (serve_pending_on(p->ctx, p) > 0 ||
                 (p->auto_sliced && serve_pending_on(p->ctx, p->auto_sliced) > 0))) {
    set_error("tn_plan_free: serve requests on this plan are still pending");
    return TN_E_INVALID_ARG;
  }
  if (p->auto_sliced) {
    tn_status st = tn_plan_free(p->auto_sliced);
    if (st != TN_OK) return st;
    p->auto_sliced = nullptr;
  }
  if (p->ctx) {
    tn_ctx *ctx = p->ctx;
    std::lock_guard<std::mutex> g(ctx->exec_mu);
    hipStreamSynchronize(ctx->stream);
    ctx->arena.release(p->dev_leaf, p->dev_leaf_bytes, true);
    ctx->arena.release(p->dev_desc, p->dev_desc_bytes, true);
    for (auto &kv : p->layouts) {
      if (kv.second->tree_dev >= 0)
        ctx->arena.release(kv.second->tree_dev, kv.second->tree_dev_bytes, true);
      rcache_drop(ctx, *kv.second);
    }
    if (p->graph) release_graph(ctx, *p->graph);
    ctx->live_plans--;
  }
  delete p;
  return TN_OK;
}

tn_status tn_contract(tn_plan *p, int32_t num_overrides, const tn_leaf *overrides, void *out,
                      tn_dtype out_dtype, double *log2_scale, uint32_t flags) {
  if (!p || !p->ctx) {
    set_error("tn_contract: plan is NULL or host-only (loaded without a context)");
    return TN_E_INVALID_ARG;
  }
  if (num_overrides < 0 || (num_overrides > 0 && !overrides) ||
      (flags & ~(TN_FLAG_KEEP_SCALE | TN_FLAG_CONCURRENT))) {
    set_error("tn_contract: bad overrides or flags");
    return TN_E_INVALID_ARG;
  }
  if (p->nslices > 0) {
    if (!out) {
      set_error("tn_contract: out is NULL");
      return TN_E_INVALID_ARG;
    }
    std::lock_guard<std::mutex> g(p->ctx->exec_mu);
    ExecRes r = ctx_res(p->ctx);
    return run_sliced(p->ctx, p, num_overrides, overrides, out, out_dtype, log2_scale,
                      flags & TN_FLAG_KEEP_SCALE, r);
  }
  QueryIO q;
  q.ovr = overrides;
  q.novr = num_overrides;
  q.out = out;
  q.log2s = log2_scale;
  std::lock_guard<std::mutex> g(p->ctx->exec_mu);
  ExecRes r = ctx_res(p->ctx);
  return run_group(p->ctx, p, {q}, out_dtype, flags, false, r);
}

tn_status tn_contract_strided(tn_plan *p, int32_t num_queries, int32_t num_overrides,
                              const tn_leaf *overrides, const int64_t *strides, void *out,
                              int64_t out_stride, tn_dtype out_dtype, double *log2_scales,
                              uint32_t flags) {
  if (!p || !p->ctx) {
    set_error("tn_contract_strided: plan is NULL or host-only (loaded without a context)");
    return TN_E_INVALID_ARG;
  }
  if (num_queries < 0 || num_overrides < 0 || (num_overrides > 0 && (!overrides || !strides)) ||
      (num_queries > 0 && !out) || (flags & ~(TN_FLAG_KEEP_SCALE | TN_FLAG_GRAPH)) ||
      (out_dtype != TN_C64 && out_dtype != TN_C128)) {
    set_error("tn_contract_strided: bad arguments");
    return TN_E_INVALID_ARG;
  }
  if (p->nslices > 0) {
    set_error("tn_contract_strided: a sliced plan runs through tn_contract or serving");
    return TN_E_INVALID_ARG;
  }
  if (out_stride < (int64_t)result_elems(p)) {
    set_error("tn_contract_strided: out_stride %lld is smaller than a result (%zu elements)",
              (long long)out_stride, result_elems(p));
    return TN_E_INVALID_ARG;
  }
  if (num_queries == 0) return TN_OK;
  StridedOvr so;
  so.leaves.assign(overrides, overrides + num_overrides);
  so.strides.assign(strides, strides + num_overrides);
  const size_t esz = out_dtype == TN_C128 ? 16 : 8;
  // complex128 results in pinned host memory (the first and the last result
  // pinned, with one host-to-device mapping): the kernels may write them
  // there themselves
  so.log2s = log2_scales != nullptr;
  if (out_dtype == TN_C128 && (uintptr_t)out % 16 == 0) {
    const char *o0 = (const char *)out;
    const char *o1 = o0 + ((size_t)num_queries - 1) * (size_t)out_stride * esz;
    hipPointerAttribute_t a0, a1;
    memset(&a0, 0, sizeof(a0));
    memset(&a1, 0, sizeof(a1));
    const bool got = hipPointerGetAttributes(&a0, o0) == hipSuccess &&
                     hipPointerGetAttributes(&a1, o1) == hipSuccess;
    if (!got) (void)hipGetLastError();  // pageable memory: not the caller's error
    if (got && a0.type == hipMemoryTypeHost && a1.type == hipMemoryTypeHost && a0.hostPointer &&
        a0.devicePointer && a1.hostPointer && a1.devicePointer &&
        (const char *)a0.devicePointer - (const char *)a0.hostPointer ==
            (const char *)a1.devicePointer - (const char *)a1.hostPointer) {
      so.dout = (double2 *)((char *)a0.devicePointer + (o0 - (const char *)a0.hostPointer));
      so.dout_stride = out_stride;
    }
  }
  std::vector<QueryIO> qs((size_t)num_queries);
  for (int32_t i = 0; i < num_queries; ++i) {
    qs[i].out = (char *)out + (size_t)i * (size_t)out_stride * esz;
    qs[i].log2s = log2_scales ? &log2_scales[i] : nullptr;
  }
  std::lock_guard<std::mutex> g(p->ctx->exec_mu);
  ExecRes r = ctx_res(p->ctx);
  return run_group(p->ctx, p, qs, out_dtype, flags, true, r, &so);
}

tn_status tn_plan_slice(tn_plan *plan, int32_t num_labels, const int64_t *labels,
                        int64_t max_intermediate, tn_plan **out) {
  if (!plan || !out || num_labels < 0 || (num_labels > 0 && !labels) ||
      (num_labels == 0 && max_intermediate < 1)) {
    set_error("tn_plan_slice: bad arguments (a plan, labels or max_intermediate >= 1, out)");
    return TN_E_INVALID_ARG;
  }
  *out = nullptr;
  std::vector<int64_t> l(labels, labels + num_labels);
  return make_sliced_plan(plan->ctx, plan, l, max_intermediate, out);
}

tn_status tn_contract_strided_noalloc(tn_plan *p, int32_t num_queries, int32_t num_overrides,
                                      const tn_leaf *overrides, const int64_t *strides, void *out,
                                      int64_t out_stride, uint32_t flags) {
  if (!p || !p->ctx) {
    set_error("tn_contract_strided_noalloc: plan is NULL or host-only (loaded without a context)");
    return TN_E_INVALID_ARG;
  }
  if (num_queries < 0 || num_overrides < 0 || (num_overrides > 0 && (!overrides || !strides)) ||
      (num_queries > 0 && !out) || out_stride < 1 || flags != 0 || ((uintptr_t)out & 15)) {
    set_error("tn_contract_strided_noalloc: bad arguments (out: 16-byte aligned device memory, "
              "out_stride >= 1, flags = 0)");
    return TN_E_INVALID_ARG;
  }
  if (!p->closed || p->nv < 2 || p->nslices > 0) {
    set_error("tn_contract_strided_noalloc: only closed networks of two or more tensors (one "
              "amplitude per query), not sliced");
    return TN_E_INVALID_ARG;
  }
  for (int32_t i = 0; i < num_overrides; ++i)
    if (overrides[i].dtype != TN_C64_DEVICE || strides[i] < 0 || strides[i] % 8 != 0) {
      set_error("tn_contract_strided_noalloc: override %d must be TN_C64_DEVICE with a "
                "non-negative stride that is a multiple of 8 bytes", i);
      return TN_E_INVALID_ARG;
    }
  tn_ctx *ctx = p->ctx;
  if (!ctx->scratch) {
    set_error("tn_contract_strided_noalloc: the static scratch of this device is unavailable");
    return TN_E_DEVICE;
  }
  if (num_queries == 0) return TN_OK;
  // the plan's subtree programs for this override set must already be in the
  // arena (put there by an earlier call): this call uploads nothing
  std::vector<char> is(p->nv, 0);
  for (int32_t i = 0; i < num_overrides; ++i) {
    const int t = overrides[i].tensor;
    if (t < 0 || t >= p->nv || is[t] || !overrides[i].data) {
      set_error("tn_contract_strided_noalloc: override %d: tensor id out of range or repeated, or "
                "NULL data", i);
      return TN_E_INVALID_ARG;
    }
    is[t] = 1;
  }
  std::vector<int> ovr;
  for (int t = 0; t < p->nv; ++t)
    if (is[t]) ovr.push_back(t);
  {
    std::shared_ptr<ExecLayout> L = cached_layout(p, ovr, true);
    std::lock_guard<std::mutex> g(p->cache_mu);
    if (L->n_tree_shared + L->n_tree_perq > 0 && L->tree_dev < 0) {
      set_error("tn_contract_strided_noalloc: the plan's subtree programs for these overridden "
                "leaves are not on the device yet; run tn_contract_strided once with them first");
      return TN_E_INVALID_ARG;
    }
  }
  StridedOvr so;
  so.leaves.assign(overrides, overrides + num_overrides);
  so.strides.assign(strides, strides + num_overrides);
  so.dout = (double2 *)out;
  so.dout_stride = out_stride;
  so.device_out = true;
  std::vector<QueryIO> qs((size_t)num_queries);
  for (int32_t i = 0; i < num_queries; ++i) qs[i].out = (char *)out + (size_t)i * (size_t)out_stride * 16;
  std::lock_guard<std::mutex> g(ctx->exec_mu);
  ExecRes r;
  r.st = ctx->stream;
  r.ext_ws = ctx->scratch;
  r.ext_ws_bytes = kScratchBytes;
  return run_group(ctx, p, qs, TN_C128, 0, true, r, &so);
}

tn_status tn_contract_batch(tn_ctx *ctx, int32_t num_queries, const tn_query *queries,
                            void *const *outs, tn_dtype out_dtype, double *log2_scales,
                            tn_status *per_query, uint32_t flags) {
  if (!ctx || num_queries < 0 || (num_queries > 0 && (!queries || !outs)) ||
      (flags & ~(TN_FLAG_KEEP_SCALE | TN_FLAG_GRAPH))) {
    set_error("tn_contract_batch: bad arguments");
    return TN_E_INVALID_ARG;
  }
  // group queries by plan, keeping first-appearance order
  std::vector<tn_plan *> plans;
  std::vector<std::vector<int>> members;
  for (int i = 0; i < num_queries; ++i) {
    tn_plan *p = queries[i].plan;
    if (p && p->nslices > 0) {
      set_error("tn_contract_batch: query %d is on a sliced plan (use tn_contract or serving)", i);
      if (per_query) per_query[i] = TN_E_INVALID_ARG;
      return TN_E_INVALID_ARG;
    }
    if (!p || p->ctx != ctx || queries[i].num_overrides < 0 ||
        (queries[i].num_overrides > 0 && !queries[i].overrides)) {
      set_error("tn_contract_batch: query %d has no plan of this context or bad overrides", i);
      if (per_query) per_query[i] = TN_E_INVALID_ARG;
      return TN_E_INVALID_ARG;
    }
    size_t k = 0;
    while (k < plans.size() && plans[k] != p) ++k;
    if (k == plans.size()) {
      plans.push_back(p);
      members.emplace_back();
    }
    members[k].push_back(i);
  }
  tn_status first = TN_OK;
  std::lock_guard<std::mutex> g(ctx->exec_mu);
  auto group_io = [&](size_t k) {
    std::vector<QueryIO> qs;
    for (int i : members[k]) {
      QueryIO q;
      q.ovr = queries[i].overrides;
      q.novr = queries[i].num_overrides;
      q.out = outs[i];
      q.log2s = log2_scales ? &log2_scales[i] : nullptr;
      q.status = per_query ? &per_query[i] : nullptr;
      qs.push_back(q);
    }
    return qs;
  };
  std::vector<tn_status> sts(plans.size(), TN_OK);
  std::vector<std::string> msgs(plans.size());
  std::vector<char> done(plans.size(), 0);
  // Several plans: their groups run concurrently on up to four lanes (own
  // stream and staging each, ordered after the caller's stream), so that one
  // group's host work and small kernels overlap another's (with
  // TN_FLAG_GRAPH each group captures on its lane).  Not while profiling.  A
  // group that finds the arena taken by the others runs again, alone,
  // afterwards.
  const int W = (plans.size() > 1 && !ctx->prof.on)
                    ? (int)std::min<size_t>(4, plans.size())
                    : 1;
  bool lanes_ok = W > 1;
  if (lanes_ok) {
    if (!ctx->lanes_ev && hipEventCreateWithFlags(&ctx->lanes_ev, hipEventDisableTiming) != hipSuccess) {
      ctx->lanes_ev = nullptr;
      lanes_ok = false;
    }
    while (lanes_ok && (int)ctx->lanes.size() < W) {
      tn_ctx::Lane l;
      if (hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking) != hipSuccess) {
        lanes_ok = false;
        break;
      }
      ctx->lanes.push_back(l);
    }
    if (lanes_ok && hipEventRecord(ctx->lanes_ev, ctx->stream) != hipSuccess) lanes_ok = false;
    for (int w = 0; lanes_ok && w < W; ++w)
      if (hipStreamWaitEvent(ctx->lanes[w].st, ctx->lanes_ev, 0) != hipSuccess) lanes_ok = false;
    (void)hipGetLastError();
  }
  if (lanes_ok) {
    std::atomic<size_t> next{0};
    auto lane_main = [&](int w) {
      tn_ctx::Lane &l = ctx->lanes[w];
      ExecRes r;
      r.st = l.st;
      r.pinned = &l.pinned;
      r.pinned_bytes = &l.pinned_bytes;
      for (size_t k; (k = next.fetch_add(1)) < plans.size();) {
        std::vector<QueryIO> qs = group_io(k);
        sts[k] = run_group(ctx, plans[k], qs, out_dtype, flags, true, r);
        if (sts[k] == TN_E_NOMEM) continue;  // retried alone below
        done[k] = 1;
        if (sts[k] != TN_OK) msgs[k] = last_error();
      }
      hipStreamSynchronize(l.st);
    };
    std::vector<std::thread> th;
    for (int w = 1; w < W; ++w) th.emplace_back(lane_main, w);
    lane_main(0);
    for (auto &t : th) t.join();
  }
  for (size_t k = 0; k < plans.size(); ++k) {
    if (!done[k]) {
      std::vector<QueryIO> qs = group_io(k);
      ExecRes r = ctx_res(ctx);
      sts[k] = run_group(ctx, plans[k], qs, out_dtype, flags, true, r);
      if (sts[k] != TN_OK) msgs[k] = last_error();
    }
    if (sts[k] != TN_OK) {
      if (per_query)
        for (int i : members[k]) per_query[i] = sts[k];
      if (first == TN_OK) {
        first = sts[k];
        set_error("%s", msgs[k].c_str());
      }
    }
  }
  return first;
}

}  // extern "C"
