// Serving: continuous batching of contraction requests.
//
// tn_serve_submit copies a request into the scheduler's queue (sched.h) and
// returns a ticket.  Worker threads, each with its own HIP stream and pinned
// staging, take work as soon as they are idle: the requests of the first plan
// in arrival order whose batch workspace fits the free arena now (admission by
// device footprint; the whole workspace is reserved before the batch runs).  A
// request that arrives while others run joins a later batch; batches of
// different workers overlap on the device.  This file is the device side of
// the scheduler: footprints from the plan's execution layout, reservations in
// the context's arena, and each batch run as one group of queries.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "serve_sched.h"
#include "tn_internal.h"

namespace tn {

struct ServeReq : sched::Req {
  tn_plan *p = nullptr;
  std::vector<tn_leaf> leaves;           // data points into `store` or device memory
  std::vector<std::vector<float2>> store;
  std::vector<double> result;            // interleaved complex128 mantissa
  double log2s = 0.0;
};

struct ServeWorker {
  hipStream_t st = nullptr;
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
};

class DeviceBackend : public sched::Backend {
 public:
  explicit DeviceBackend(tn_ctx *ctx) : ctx_(ctx) {}

  size_t footprint(const std::vector<sched::Req *> &batch, size_t n) override {
    tn_plan *p = static_cast<ServeReq *>(batch[0])->p;
    // a sliced plan runs one request at a time, its slices as one group
    if (p->nslices > 0 && n > 1) return SIZE_MAX / 4;
    return request_bytes(p, batch, n, capacity());
  }
  // Workspace to reserve for n requests of plan p.  A sliced request reserves
  // room for a chunk of its slices (all of them if that takes at most half of
  // `cap`, else halves of them down to one) and runs its slices chunk by chunk.
  static size_t request_bytes(tn_plan *p, const std::vector<sched::Req *> &batch, size_t n,
                              size_t cap) {
    std::shared_ptr<ExecLayout> L = layout_of(p, batch, n);
    int64_t nq = p->nslices > 0 ? p->nslices * (int64_t)n : (int64_t)n;
    size_t b = Arena::round(group_workspace_bytes(p, *L, (int)nq));
    while (p->nslices > 0 && nq > 1 && b > cap / 2) {
      nq = (nq + 1) / 2;
      b = Arena::round(group_workspace_bytes(p, *L, (int)nq));
    }
    return b;
  }
  // The execution layout of n requests of plan p (their overridden tensors,
  // and those a sliced plan overrides per slice).
  static std::shared_ptr<ExecLayout> layout_of(tn_plan *p, const std::vector<sched::Req *> &batch,
                                               size_t n) {
    std::vector<char> is(p->nv, 0);
    for (size_t i = 0; i < n; ++i)
      for (const tn_leaf &l : static_cast<ServeReq *>(batch[i])->leaves) is[l.tensor] = 1;
    for (int t : p->slice_touched) is[t] = 1;
    std::vector<int> ovr;
    for (int t = 0; t < p->nv; ++t)
      if (is[t]) ovr.push_back(t);
    return cached_layout(p, ovr, true);
  }
  int64_t reserve(size_t bytes) override { return ctx_->arena.alloc(bytes); }
  void release(int64_t off, size_t bytes) override { ctx_->arena.release(off, bytes); }
  size_t capacity() override { return ctx_->arena.work_capacity(); }
  uint64_t releases() override { return ctx_->arena.releases(); }

  void *worker_begin() override {
    hipSetDevice(ctx_->device);
    ServeWorker *w = new ServeWorker;
    if (hipStreamCreateWithFlags(&w->st, hipStreamNonBlocking) != hipSuccess) w->st = nullptr;
    return w;
  }
  void worker_end(void *wp) override {
    ServeWorker *w = static_cast<ServeWorker *>(wp);
    if (w->st) {
      hipStreamSynchronize(w->st);
      hipStreamDestroy(w->st);
    }
    if (w->pinned) hipHostFree(w->pinned);
    delete w;
  }

  int32_t run(void *wp, const std::vector<sched::Req *> &batch, int64_t ws, size_t bytes,
              std::vector<int32_t> &st) override {
    ServeWorker *w = static_cast<ServeWorker *>(wp);
    tn_plan *p = static_cast<ServeReq *>(batch[0])->p;
    const size_t relems = result_elems(p);
    std::vector<QueryIO> qs(batch.size());
    std::vector<std::vector<double>> outs(batch.size());
    std::vector<double> l2(batch.size(), 0.0);
    for (size_t i = 0; i < batch.size(); ++i) {
      ServeReq *r = static_cast<ServeReq *>(batch[i]);
      outs[i].assign(2 * relems, 0.0);
      qs[i].ovr = r->leaves.data();
      qs[i].novr = (int32_t)r->leaves.size();
      qs[i].out = outs[i].data();
      qs[i].log2s = &l2[i];
      qs[i].status = &st[i];
    }
    ExecRes res;
    res.st = w->st ? w->st : ctx_->stream;
    res.pinned = &w->pinned;
    res.pinned_bytes = &w->pinned_bytes;
    res.ws = ws;
    res.ws_bytes = bytes;
    if (p->nslices > 0) {  // one request: its slices summed
      ServeReq *r = static_cast<ServeReq *>(batch[0]);
      const tn_status rc = run_sliced(ctx_, p, (int32_t)r->leaves.size(), r->leaves.data(),
                                      outs[0].data(), TN_C128, &l2[0], TN_FLAG_KEEP_SCALE, res);
      if (rc != TN_OK) return rc;
      r->result.swap(outs[0]);
      r->log2s = l2[0];
      st[0] = TN_OK;
      return TN_OK;
    }
    const tn_status rc = run_group(ctx_, p, qs, TN_C128, TN_FLAG_KEEP_SCALE, true, res);
    if (rc != TN_OK) return rc;
    for (size_t i = 0; i < batch.size(); ++i) {
      ServeReq *r = static_cast<ServeReq *>(batch[i]);
      r->result.swap(outs[i]);
      r->log2s = l2[i];
    }
    return TN_OK;
  }

 private:
  tn_ctx *ctx_;
};

struct ServeState {
  DeviceBackend backend;
  sched::Scheduler sched;
  ServeState(tn_ctx *ctx, const sched::Options &o) : backend(ctx), sched(&backend, o) {}
};

static size_t env_size(const char *name, size_t dflt) {
  const char *v = getenv(name);
  if (!v) return dflt;
  const long long x = atoll(v);
  return x > 0 ? (size_t)x : dflt;
}

static ServeState *serve_state(tn_ctx *ctx) {
  std::lock_guard<std::mutex> g(ctx->serve_init_mu);
  if (!ctx->serve) {
    sched::Options o;
    o.workers = (int)env_size("TN_SERVE_WORKERS", 2);
    o.max_queue = env_size("TN_SERVE_QUEUE", o.max_queue);
    o.max_batch = env_size("TN_SERVE_BATCH", o.max_batch);
    ctx->serve = new ServeState(ctx, o);
  }
  return ctx->serve;
}

void serve_shutdown(tn_ctx *ctx) {
  std::lock_guard<std::mutex> g(ctx->serve_init_mu);
  ServeState *S = ctx->serve;
  if (!S) return;
  S->sched.stop();
  S->sched.drop_all();
  delete S;
  ctx->serve = nullptr;
}

// Number of requests of `plan` not yet finished (a plan must not be freed
// while requests on it are queued or running).
int serve_pending_on(tn_ctx *ctx, const tn_plan *plan) {
  std::lock_guard<std::mutex> g(ctx->serve_init_mu);
  if (!ctx->serve) return 0;
  return ctx->serve->sched.pending_on(plan);
}

}  // namespace tn

using namespace tn;

extern "C" {

tn_status tn_serve_submit(tn_ctx *ctx, const tn_query *query, uint64_t *ticket) {
  if (!ctx || !query || !ticket || !query->plan || query->plan->ctx != ctx ||
      query->num_overrides < 0 || (query->num_overrides > 0 && !query->overrides)) {
    set_error("tn_serve_submit: bad arguments (the plan must belong to this context)");
    return TN_E_INVALID_ARG;
  }
  tn_plan *p = query->plan;
  ServeReq *r = new ServeReq;
  r->p = p;
  r->plan = p;
  for (int i = 0; i < query->num_overrides; ++i) {
    const tn_leaf &l = query->overrides[i];
    if (l.tensor < 0 || l.tensor >= p->nv || !l.data ||
        (l.dtype != TN_C64 && l.dtype != TN_C128 && l.dtype != TN_C64_DEVICE)) {
      delete r;
      set_error("tn_serve_submit: override %d is invalid", i);
      return TN_E_INVALID_ARG;
    }
    tn_leaf c = l;
    if (l.dtype != TN_C64_DEVICE) {
      // host data is copied now; device data must stay valid until polled
      const int64_t n = p->leaf[l.tensor].size();
      r->store.emplace_back(n);
      std::vector<float2> &dst = r->store.back();
      if (l.dtype == TN_C128) {
        const double *s = (const double *)l.data;
        for (int64_t k = 0; k < n; ++k) dst[k] = make_float2((float)s[2 * k], (float)s[2 * k + 1]);
      } else {
        memcpy(dst.data(), l.data, sizeof(float2) * n);
      }
      c.data = dst.data();
      c.dtype = TN_C64;
    }
    r->leaves.push_back(c);
  }
  ServeState *S = serve_state(ctx);
  // a request whose workspace can never fit the arena runs on a sliced copy
  // of its plan (made once, kept with the plan): slices small enough to fit.
  // The room is measured with the sliced plan's own persistent data (leaves,
  // subtree programs) already in the arena.
  {
    std::vector<sched::Req *> one{r};
    if (p->nslices == 0 &&
        DeviceBackend::request_bytes(p, one, 1, ctx->arena.work_capacity()) > ctx->arena.work_capacity()) {
      std::lock_guard<std::mutex> g(p->slice_mu);
      for (int64_t target = p->largest / 2; !p->auto_sliced && target >= 1; target /= 2) {
        tn_plan *sl = nullptr;
        if (make_sliced_plan(ctx, p, {}, target, &sl) != TN_OK) break;
        r->p = sl;
        {
          std::shared_ptr<ExecLayout> L = DeviceBackend::layout_of(sl, one, 1);
          std::lock_guard<std::mutex> gl(sl->cache_mu);
          (void)upload_tree_programs(ctx, *L, ctx->stream);
        }
        const size_t cap = ctx->arena.work_capacity();
        if (DeviceBackend::request_bytes(sl, one, 1, cap) <= cap) {
          p->auto_sliced = sl;
        } else {
          tn_plan_free(sl);
          if (target < 2) break;
        }
        r->p = p;
      }
      if (p->auto_sliced) {
        r->p = p->auto_sliced;
        r->plan = p->auto_sliced;
      }
    }
  }
  // the request's subtree programs go to the arena now (persistent), before
  // an admission reserves the room they would need at run time
  {
    std::vector<sched::Req *> one{r};
    std::shared_ptr<ExecLayout> L = DeviceBackend::layout_of(r->p, one, 1);
    std::lock_guard<std::mutex> g(r->p->cache_mu);
    (void)upload_tree_programs(ctx, *L, ctx->stream);  // a failure shows when the request runs
  }
  if (S->sched.submit(r, ticket) != sched::kOk) {
    delete r;
    set_error("tn_serve_submit: queue full");
    return TN_E_AGAIN;
  }
  return TN_OK;
}

tn_status tn_serve_poll(tn_ctx *ctx, uint64_t ticket, void *out, tn_dtype out_dtype,
                        double *log2_scale, double *latency_s) {
  if (!ctx || (out_dtype != TN_C64 && out_dtype != TN_C128)) {
    set_error("tn_serve_poll: bad arguments");
    return TN_E_INVALID_ARG;
  }
  ServeState *S;
  {
    std::lock_guard<std::mutex> g(ctx->serve_init_mu);
    S = ctx->serve;
  }
  if (!S) {
    set_error("tn_serve_poll: ticket %llu was never issued", (unsigned long long)ticket);
    return TN_E_UNKNOWN_TICKET;
  }
  bool bad_out = false;
  const int32_t st = S->sched.take(ticket, [&](sched::Req *rq) -> int32_t {
    ServeReq *r = static_cast<ServeReq *>(rq);
    if (r->status == TN_OK) {
      if (!out) {
        bad_out = true;
        return sched::kPending;  // keep the result for a call with a buffer
      }
      const size_t n = r->result.size() / 2;
      const bool keep = log2_scale != nullptr;
      const int e = (int)r->log2s;
      for (size_t i = 0; i < n; ++i) {
        double re = r->result[2 * i], im = r->result[2 * i + 1];
        if (!keep) {
          re = std::ldexp(re, e);
          im = std::ldexp(im, e);
        }
        if (out_dtype == TN_C128) {
          ((double *)out)[2 * i] = re;
          ((double *)out)[2 * i + 1] = im;
        } else {
          ((float *)out)[2 * i] = (float)re;
          ((float *)out)[2 * i + 1] = (float)im;
        }
      }
      if (log2_scale) *log2_scale = r->log2s;
    }
    if (latency_s) *latency_s = std::chrono::duration<double>(r->finished - r->submitted).count();
    return r->status;
  });
  if (bad_out) {
    set_error("tn_serve_poll: out is NULL");
    return TN_E_INVALID_ARG;
  }
  if (st == sched::kUnknown) {
    set_error("tn_serve_poll: ticket %llu unknown or already consumed", (unsigned long long)ticket);
    return TN_E_UNKNOWN_TICKET;
  }
  if (st < 0) set_error("tn_serve_poll: request failed (status %d)", (int)st);
  return st;
}

}  // extern "C"
