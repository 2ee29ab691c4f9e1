// Serving: continuous batching of contraction requests.
//
// tn_serve_submit copies a request into a queue and returns a ticket.  Worker
// threads, each with its own HIP stream and pinned staging, take work as soon
// as they are idle: the requests queued for the plan at the head of the queue,
// as many as fit the free arena (admission by device footprint: the batch's
// whole workspace is reserved before it runs).  A request that arrives while
// others run joins the next batch; batches of different workers overlap on
// the device.  A request that cannot fit even alone, with nothing else
// running, fails with TN_E_NOMEM without affecting the others.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "tn_internal.h"

namespace tn {

typedef std::chrono::steady_clock clk;

struct ServeReq {
  uint64_t ticket = 0;
  tn_plan *plan = nullptr;
  std::vector<tn_leaf> leaves;           // data points into `store` or device memory
  std::vector<std::vector<float2>> store;
  clk::time_point submitted, finished;
  tn_status status = TN_PENDING;
  std::vector<double> result;            // interleaved complex128 mantissa
  double log2s = 0.0;
};

struct ServeState {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<ServeReq *> queue;
  std::unordered_map<uint64_t, ServeReq *> reqs;
  std::vector<std::thread> workers;
  uint64_t next_ticket = 1;
  bool stop = false;
  int running = 0;           // batches on the device
  size_t max_queue = 1 << 20;
  size_t max_batch = 4096;
};

static void worker_main(tn_ctx *ctx, ServeState *S) {
  hipSetDevice(ctx->device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
    if (S->stop) break;
    // the plan at the head of the queue and everything queued for it
    tn_plan *p = S->queue.front()->plan;
    std::vector<ServeReq *> batch;
    for (ServeReq *r : S->queue)
      if (r->plan == p && batch.size() < S->max_batch) batch.push_back(r);
    // admission: the largest prefix whose workspace the arena can hold now
    std::vector<int> ovr;
    {
      std::vector<char> is(p->nv, 0);
      for (ServeReq *r : batch)
        for (const tn_leaf &l : r->leaves) is[l.tensor] = 1;
      for (int t = 0; t < p->nv; ++t)
        if (is[t]) ovr.push_back(t);
    }
    std::shared_ptr<ExecLayout> L = cached_layout(p, ovr, true);
    size_t n = batch.size();
    int64_t ws = -1;
    size_t bytes = 0;
    while (n > 0) {
      bytes = group_workspace_bytes(p, *L, (int)n);
      ws = ctx->arena.alloc(bytes);
      if (ws >= 0) break;
      n /= 2;
    }
    if (ws < 0) {
      if (S->running == 0) {
        // cannot fit even alone with the device idle: fail the head request
        ServeReq *r = S->queue.front();
        S->queue.pop_front();
        r->status = TN_E_NOMEM;
        r->finished = clk::now();
      } else {
        S->cv.wait(lk);  // a running batch will release memory
      }
      continue;
    }
    batch.resize(n);
    for (ServeReq *r : batch) S->queue.erase(std::find(S->queue.begin(), S->queue.end(), r));
    S->running++;
    lk.unlock();

    std::vector<QueryIO> qs(batch.size());
    std::vector<std::vector<double>> outs(batch.size());
    std::vector<double> l2(batch.size(), 0.0);
    std::vector<tn_status> sts(batch.size(), TN_OK);
    const size_t relems = result_elems(p);
    for (size_t i = 0; i < batch.size(); ++i) {
      outs[i].assign(2 * relems, 0.0);
      qs[i].ovr = batch[i]->leaves.data();
      qs[i].novr = (int32_t)batch[i]->leaves.size();
      qs[i].out = outs[i].data();
      qs[i].log2s = &l2[i];
      qs[i].status = &sts[i];
    }
    ExecRes res;
    res.st = st ? st : ctx->stream;
    res.pinned = &pinned;
    res.pinned_bytes = &pinned_bytes;
    res.ws = ws;
    res.ws_bytes = bytes;
    tn_status rc = run_group(ctx, p, qs, TN_C128, TN_FLAG_KEEP_SCALE, true, res);
    ctx->arena.release(ws, bytes);

    lk.lock();
    const clk::time_point now = clk::now();
    for (size_t i = 0; i < batch.size(); ++i) {
      ServeReq *r = batch[i];
      r->status = rc != TN_OK ? rc : sts[i];
      r->result.swap(outs[i]);
      r->log2s = l2[i];
      r->finished = now;
    }
    S->running--;
    S->cv.notify_all();
  }
  lk.unlock();
  if (st) {
    hipStreamSynchronize(st);
    hipStreamDestroy(st);
  }
  if (pinned) hipHostFree(pinned);
}

static ServeState *serve_state(tn_ctx *ctx) {
  std::lock_guard<std::mutex> g(ctx->serve_init_mu);
  if (!ctx->serve) {
    ServeState *S = new ServeState;
    const char *w = getenv("TN_SERVE_WORKERS");
    int nw = w ? std::max(1, atoi(w)) : 2;
    for (int i = 0; i < nw; ++i) S->workers.emplace_back(worker_main, ctx, S);
    ctx->serve = S;
  }
  return ctx->serve;
}

void serve_shutdown(tn_ctx *ctx) {
  std::lock_guard<std::mutex> g(ctx->serve_init_mu);
  ServeState *S = ctx->serve;
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (std::thread &t : S->workers) t.join();
  for (auto &kv : S->reqs) delete kv.second;
  delete S;
  ctx->serve = nullptr;
}

// Number of requests of `plan` not yet polled (a plan must not be freed while
// requests on it are queued or running).
int serve_pending_on(tn_ctx *ctx, const tn_plan *plan) {
  std::lock_guard<std::mutex> g(ctx->serve_init_mu);
  if (!ctx->serve) return 0;
  std::lock_guard<std::mutex> lk(ctx->serve->mu);
  int n = 0;
  for (auto &kv : ctx->serve->reqs)
    if (kv.second->plan == plan && kv.second->status == TN_PENDING) ++n;
  return n;
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
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->queue.size() >= S->max_queue) {
      delete r;
      set_error("tn_serve_submit: queue full");
      return TN_E_AGAIN;
    }
    r->ticket = S->next_ticket++;
    r->submitted = clk::now();
    S->reqs[r->ticket] = r;
    S->queue.push_back(r);
    *ticket = r->ticket;
  }
  S->cv.notify_one();
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
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    set_error("tn_serve_poll: ticket %llu unknown or already consumed", (unsigned long long)ticket);
    return TN_E_UNKNOWN_TICKET;
  }
  ServeReq *r = it->second;
  if (r->status == TN_PENDING) return TN_PENDING;
  tn_status st = r->status;
  if (st == TN_OK) {
    if (!out) {
      set_error("tn_serve_poll: out is NULL");
      return TN_E_INVALID_ARG;
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
  } else {
    set_error("tn_serve_poll: request failed (status %d)", (int)st);
  }
  if (latency_s) *latency_s = std::chrono::duration<double>(r->finished - r->submitted).count();
  S->reqs.erase(it);
  delete r;
  return st;
}

}  // extern "C"
