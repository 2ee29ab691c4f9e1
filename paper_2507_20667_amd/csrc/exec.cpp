// Execution of a plan for a group of queries: partitions in turn, then the
// reduction path (Section 4, phases 2 and 4, one GPU), one launch sequence per
// tree vertex.  Vertices that no overridden leaf reaches are computed once and
// shared when `share` is set; every other vertex runs once for all queries of
// the group (grid dimension y = query).
#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "tn_internal.h"

namespace tn {

// k-tiled output order of a GEMM operand's split planes (rows = M or N)
static KTile ktile_of(const Node &n, int64_t rows) {
  KTile t{0, 0, -1, 0};
  if (!n.ktile) return t;
  t.rows = rows;
  t.kdim = n.K;
  t.on = 1;
  if ((n.K & (n.K - 1)) == 0)
    for (t.kshift = 0; ((int64_t)1 << t.kshift) < n.K; ++t.kshift) {
    }
  return t;
}

size_t result_elems(const tn_plan *p) {
  return p->closed ? 1 : (size_t)p->result_layout.size();
}

void release_graph(tn_ctx *ctx, GraphEntry &g) {
  if (g.exec) hipGraphExecDestroy(g.exec);
  if (g.ws >= 0) ctx->arena.release(g.ws, g.ws_bytes, true);
  if (g.pinned) hipHostFree(g.pinned);
  g = GraphEntry();
}

static size_t rnd(size_t b) { return (b + 255) & ~(size_t)255; }

// Streams and events for TN_FLAG_CONCURRENT: one stream per partition (default
// priority, not synchronizing with the null stream), created on first use.
static tn_status ensure_part_streams(tn_ctx *ctx, int K) {
  if (!ctx->part_ev0 && hipEventCreateWithFlags(&ctx->part_ev0, hipEventDisableTiming) != hipSuccess) {
    ctx->part_ev0 = nullptr;
    set_error("partition streams: event creation failed");
    return TN_E_DEVICE;
  }
  while ((int)ctx->part_st.size() < K) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      set_error("partition streams: stream creation failed");
      return TN_E_DEVICE;
    }
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      hipStreamDestroy(s);
      set_error("partition streams: event creation failed");
      return TN_E_DEVICE;
    }
    ctx->part_st.push_back(s);
    ctx->part_ev.push_back(e);
  }
  return TN_OK;
}

static tn_status ensure_pinned(ExecRes &r, size_t bytes, hipStream_t st) {
  if (*r.pinned_bytes >= bytes) return TN_OK;
  // the previous staging may still feed a copy in flight on the call's stream
  hipStreamSynchronize(st);
  if (st != r.st) hipStreamSynchronize(r.st);
  if (*r.pinned) hipHostFree(*r.pinned);
  *r.pinned = nullptr;
  *r.pinned_bytes = 0;
  size_t nb = std::max(bytes, (size_t)1 << 20);
  if (hipHostMalloc(r.pinned, nb, hipHostMallocDefault) != hipSuccess) {
    *r.pinned = nullptr;
    set_error("hipHostMalloc of %zu bytes of pinned staging failed", nb);
    return TN_E_DEVICE;
  }
  *r.pinned_bytes = nb;
  return TN_OK;
}

// ------------------------------------------------------ shared-part cache
// A layout's shared part (the vertices no override reaches, computed once per
// call for all its queries) depends only on the plan's own leaves, so it is
// the same on every call (order independence of the contraction, Section
// 2.3): it is kept in the arena after a first call fills it, and later calls
// skip those vertices.  Entries are evicted least recently used first when
// the cached bytes would pass the context's budget, never while a call uses
// them; a plan's entries go with the plan.
enum { RC_NONE = 0, RC_READ = 1, RC_FILL = 2 };

static bool rcache_evict_one(tn_ctx *ctx, const ExecLayout *keep) {
  ExecLayout *victim = nullptr;
  for (ExecLayout *e : ctx->rcache)
    if (e != keep && e->rc_pins == 0 && e->rc_state != 1 && (!victim || e->rc_used < victim->rc_used))
      victim = e;
  if (!victim) return false;
  ctx->arena.release(victim->rc_off, victim->rc_bytes, true);
  ctx->rcache_bytes -= victim->rc_bytes;
  victim->rc_off = -1;
  victim->rc_bytes = 0;
  victim->rc_state = 0;
  ctx->rcache.erase(std::find(ctx->rcache.begin(), ctx->rcache.end(), victim));
  return true;
}

// RC_READ: the cache holds the shared part; RC_FILL: this call computes it
// into the cache; RC_NONE: it computes it in its own workspace.
static int rcache_acquire(tn_ctx *ctx, ExecLayout &L, size_t bytes, bool may_fill) {
  std::lock_guard<std::mutex> g(ctx->rcache_mu);
  if (L.rc_state == 2) {
    L.rc_pins++;
    L.rc_used = ++ctx->rcache_clock;
    return RC_READ;
  }
  if (L.rc_state == 1 || !may_fill || bytes > ctx->rcache_budget) return RC_NONE;
  if (L.rc_off < 0) {
    while (ctx->rcache_bytes + bytes > ctx->rcache_budget && rcache_evict_one(ctx, &L)) {
    }
    if (ctx->rcache_bytes + bytes > ctx->rcache_budget) return RC_NONE;
    int64_t off = ctx->arena.alloc(bytes, true);
    while (off < 0 && rcache_evict_one(ctx, &L)) off = ctx->arena.alloc(bytes, true);
    if (off < 0) return RC_NONE;
    L.rc_off = off;
    L.rc_bytes = bytes;
    ctx->rcache_bytes += bytes;
    ctx->rcache.push_back(&L);
  }
  L.rc_state = 1;
  L.rc_pins++;
  L.rc_used = ++ctx->rcache_clock;
  return RC_FILL;
}

static void rcache_release(tn_ctx *ctx, ExecLayout &L, int mode, bool ok) {
  if (mode == RC_NONE) return;
  std::lock_guard<std::mutex> g(ctx->rcache_mu);
  if (mode == RC_FILL) L.rc_state = ok ? 2 : 0;
  L.rc_pins--;
}

void rcache_drop(tn_ctx *ctx, ExecLayout &L) {
  std::lock_guard<std::mutex> g(ctx->rcache_mu);
  if (L.rc_off < 0) return;
  ctx->arena.release(L.rc_off, L.rc_bytes, true);
  ctx->rcache_bytes -= L.rc_bytes;
  ctx->rcache.erase(std::find(ctx->rcache.begin(), ctx->rcache.end(), &L));
  L.rc_off = -1;
  L.rc_bytes = 0;
  L.rc_state = 0;
}

// First use of a layout: its subtree programs go to the arena (persistent,
// kept with the plan).  The caller holds the plan's cache_mu.
tn_status upload_tree_programs(tn_ctx *ctx, const ExecLayout &L, hipStream_t st) {
  if (L.n_tree_shared + L.n_tree_perq == 0 || L.tree_dev >= 0) return TN_OK;
  ExecLayout &Lm = const_cast<ExecLayout &>(L);
  Lm.tree_dev_bytes = std::max<size_t>(L.tree_blob.size(), 256);
  Lm.tree_dev = ctx->arena.alloc(Lm.tree_dev_bytes, true);
  if (Lm.tree_dev < 0) {
    set_error("arena cannot hold the subtree programs (%zu bytes)", Lm.tree_dev_bytes);
    return TN_E_NOMEM;
  }
  hipError_t e = hipMemcpyAsync(ctx->arena.base() + Lm.tree_dev, L.tree_blob.data(), L.tree_blob.size(),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    ctx->arena.release(Lm.tree_dev, Lm.tree_dev_bytes, true);
    Lm.tree_dev = -1;
    set_error("subtree program upload: %s", hipGetErrorString(e));
    return TN_E_DEVICE;
  }
  return TN_OK;
}

// Device bytes of one execution chunk of Q queries (carved in run_group).
size_t group_workspace_bytes(const tn_plan *p, const ExecLayout &L, int Q) {
  const int nn = 2 * p->nv - 1;
  const size_t relems = result_elems(p);
  const size_t final_bytes = p->fperm.needed ? rnd(relems * 8) : 0;
  int max_blocks = 1;
  for (const Node &n : p->nodes)
    if (n.kind == NK_DOT) max_blocks = std::max(max_blocks, n.dot_blocks);
  return rnd(L.shared_bytes) + rnd(rnd(L.perq_bytes) * Q) + rnd((size_t)nn * sizeof(Slot) * (Q + 1)) +
         rnd((size_t)L.ovr_bytes * Q) + rnd(sizeof(Result) * Q) + rnd(final_bytes * Q) +
         rnd((size_t)max_blocks * 16 * Q);
}

static void to_c64(const tn_leaf &l, int64_t n, float2 *dst) {
  if (l.dtype == TN_C128) {
    const double *s = (const double *)l.data;
    for (int64_t i = 0; i < n; ++i) dst[i] = make_float2((float)s[2 * i], (float)s[2 * i + 1]);
  } else {
    memcpy(dst, l.data, sizeof(float2) * n);
  }
}

// 2^e as a double: built from its bits in the normal range (multiplying by it
// is exact there, as ldexp is), ldexp outside it
static inline double pow2i(int e) {
  if (e >= -1022 && e <= 1023) {
    const uint64_t b = (uint64_t)(e + 1023) << 52;
    double d;
    memcpy(&d, &b, sizeof d);
    return d;
  }
  return std::ldexp(1.0, e);
}

static void write_out(void *out, tn_dtype dt, size_t i, double re, double im) {
  if (dt == TN_C128) {
    ((double *)out)[2 * i] = re;
    ((double *)out)[2 * i + 1] = im;
  } else {
    ((float *)out)[2 * i] = (float)re;
    ((float *)out)[2 * i + 1] = (float)im;
  }
}

#define TN_HIP(call, what)                                                                \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      set_error("%s: %s", what, hipGetErrorString(e_));                                   \
      rc = TN_E_DEVICE;                                                                   \
      goto done;                                                                          \
    }                                                                                     \
  } while (0)

tn_status run_group(tn_ctx *ctx, tn_plan *p, const std::vector<QueryIO> &qs, tn_dtype out_dtype,
                    uint32_t flags, bool share, ExecRes &rs, const StridedOvr *so, SliceSum *sum) {
  const int nv = p->nv, nn = 2 * nv - 1;
  if (qs.empty()) return TN_OK;
  if (out_dtype != TN_C64 && out_dtype != TN_C128) {
    set_error("out_dtype must be TN_C64 or TN_C128");
    return TN_E_INVALID_ARG;
  }
  // overridden leaves of the group
  std::vector<char> is_ovr(nv, 0);
  std::vector<int> so_of(so ? nv : 0, -1);  // strided form: leaf -> its entry
  if (so)
    for (size_t i = 0; i < so->leaves.size(); ++i) {
      const tn_leaf &l = so->leaves[i];
      if (l.tensor < 0 || l.tensor >= nv || !l.data || is_ovr[l.tensor] ||
          (l.dtype != TN_C64 && l.dtype != TN_C128 && l.dtype != TN_C64_DEVICE) ||
          so->strides[i] < 0) {
        set_error("override %zu: tensor id out of range or repeated, NULL data, bad dtype or "
                  "negative stride", i);
        return TN_E_INVALID_ARG;
      }
      is_ovr[l.tensor] = 1;
      so_of[l.tensor] = (int)i;
    }
  for (const QueryIO &q : qs) {
    if (!q.out) {
      set_error("output pointer is NULL");
      return TN_E_INVALID_ARG;
    }
    if (so) continue;
    for (int i = 0; i < q.novr; ++i) {
      const tn_leaf &l = q.ovr[i];
      if (l.tensor < 0 || l.tensor >= nv || !l.data ||
          (l.dtype != TN_C64 && l.dtype != TN_C128 && l.dtype != TN_C64_DEVICE)) {
        set_error("override %d: tensor id out of range, NULL data or bad dtype", i);
        return TN_E_INVALID_ARG;
      }
      is_ovr[l.tensor] = 1;
    }
  }
  std::vector<int> ovr, kidx(nv, -1);
  for (int t = 0; t < nv; ++t)
    if (is_ovr[t]) {
      kidx[t] = (int)ovr.size();
      ovr.push_back(t);
    }
  const bool dbg = getenv("TN_DEBUG") != nullptr;
  // TN_DEBUG=gemm: also time every GEMM launch on its own (synchronizing)
  const bool dbg_gemm = dbg && strcmp(getenv("TN_DEBUG"), "gemm") == 0;
  const auto t_enter = std::chrono::steady_clock::now();
  auto ms_since = [](std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };
  // TN_FLAG_CONCURRENT (single calls): partitions side by side, each on a
  // stream of its own, in a layout that gives each its own memory
  const bool conc = (flags & TN_FLAG_CONCURRENT) && !share && qs.size() == 1 && p->K > 1 &&
                    !(flags & TN_FLAG_GRAPH) && rs.st == ctx->stream;
  if (conc) {
    tn_status cs = ensure_part_streams(ctx, p->K);
    if (cs != TN_OK) return cs;
  }
  std::shared_ptr<ExecLayout> Lp = cached_layout(p, ovr, share, conc);
  const ExecLayout &L = *Lp;
  const double t_layout = dbg ? ms_since(t_enter) : 0.0;
  Profiler idle_prof;
  Profiler &prof = rs.prof ? *rs.prof : idle_prof;
  const hipStream_t st = rs.st;

  // per-query override block: leaves in increasing id order
  const std::vector<int64_t> &ovr_off = L.ovr_off;
  const size_t ovr_bytes = (size_t)L.ovr_bytes;
  const bool trees = L.n_tree_shared + L.n_tree_perq > 0;
  std::unique_lock<std::mutex> upload_lock(p->cache_mu);
  {
    const tn_status us = upload_tree_programs(ctx, L, st);
    if (us != TN_OK) return us;
  }
  // algorithmic traffic and work of the subtree kernel (for the profiler),
  // once per layout
  // (a vertex counts as its subtree runs: once when the subtree's root is
  // shared, once per query otherwise, whatever the vertex itself depends on)
  if (trees && !L.tree_acct) {
    ExecLayout &Lm = const_cast<ExecLayout &>(L);
    std::vector<int> troots(p->tree_roots);
    troots.insert(troots.end(), L.islands.begin(), L.islands.end());
    for (int r : troots) {
      const bool shr = L.shared[r] != 0;
      std::vector<int> stack{r};
      while (!stack.empty()) {
        const int u = stack.back();
        stack.pop_back();
        if (u < nv) continue;
        // an island inside a per-query subtree runs (and counts) on its own
        if (u != r && std::binary_search(L.islands.begin(), L.islands.end(), u)) continue;
        const Node &n = p->nodes[u - nv];
        stack.push_back(n.c1);
        stack.push_back(n.c2);
        auto sz = [&](int t) {
          return (double)(t < nv ? p->leaf[t].size() : std::max<int64_t>(p->nodes[t - nv].out.size(), 1));
        };
        const double b = 8.0 * (sz(n.c1) + sz(n.c2) + sz(n.id)), f = 8.0 * (double)n.weight;
        (shr ? Lm.tree_bytes_sh : Lm.tree_bytes_q) += b;
        (shr ? Lm.tree_flops_sh : Lm.tree_flops_q) += f;
      }
    }
    Lm.tree_acct = true;
  }
  upload_lock.unlock();
  const double tree_bytes_sh = L.tree_bytes_sh, tree_flops_sh = L.tree_flops_sh;
  const double tree_bytes_q = L.tree_bytes_q, tree_flops_q = L.tree_flops_q;
  const size_t perq = rnd(L.perq_bytes);
  const size_t relems = result_elems(p);
  const size_t final_bytes = p->fperm.needed ? rnd(relems * 8) : 0;
  const size_t slot_bytes = (size_t)nn * sizeof(Slot);
  int max_blocks = 1;
  for (const Node &n : p->nodes)
    if (n.kind == NK_DOT) max_blocks = std::max(max_blocks, n.dot_blocks);
  const size_t shared_fixed = rnd(L.shared_bytes) + rnd(slot_bytes);
  const size_t per_query = perq + slot_bytes + ovr_bytes + sizeof(Result) + final_bytes +
                           (size_t)max_blocks * 16;
  // queries per chunk that fit the arena (or the caller's reserved workspace)
  size_t chunk;
  if (rs.ext_ws) {
    const size_t need = group_workspace_bytes(p, L, (int)qs.size());
    if (need > rs.ext_ws_bytes) {
      set_error("the workspace of %zu queries (%zu bytes) exceeds the static scratch (%zu bytes)",
                qs.size(), need, rs.ext_ws_bytes);
      return TN_E_NOMEM;
    }
    chunk = qs.size();
  } else if (rs.ws >= 0) {
    chunk = qs.size();
    if (group_workspace_bytes(p, L, (int)chunk) > rs.ws_bytes) {
      // the slices of a sliced request run in chunks of the reserved
      // workspace: the most queries whose workspace fits it
      size_t lo = 0, hi = sum ? qs.size() : 0;
      while (lo < hi) {
        const size_t mid = (lo + hi + 1) / 2;
        if (group_workspace_bytes(p, L, (int)mid) <= rs.ws_bytes)
          lo = mid;
        else
          hi = mid - 1;
      }
      if (lo == 0) {
        set_error("reserved workspace too small for %zu queries", qs.size());
        return TN_E_NOMEM;
      }
      chunk = lo;
    }
  } else {
    size_t avail = ctx->arena.largest_free();
    if (avail < shared_fixed + per_query + 4096) {
      set_error("arena too small: need %zu bytes for one query, largest free block %zu",
                shared_fixed + per_query + 4096, avail);
      return TN_E_NOMEM;
    }
    chunk = (avail - shared_fixed - 4096) / (per_query + 1024);
    chunk = std::min<size_t>(chunk, 65535);
    chunk = std::max<size_t>(chunk, 1);
  }
  tn_status rc = TN_OK;
  // TN_FLAG_GRAPH (the whole group in one chunk, not profiled, not serving):
  // the call runs on the context's graph stream, after the caller's stream
  bool want_graph = (flags & TN_FLAG_GRAPH) && rs.ws < 0 && !rs.ext_ws && !prof.on && !dbg_gemm &&
                    chunk >= qs.size();
  hipStream_t gst = nullptr;
  // a caller's stream other than the context's (a batch lane, never the null
  // stream) is captured on directly
  if (want_graph && rs.st != ctx->stream && rs.st) gst = rs.st;
  if (want_graph && !gst) {
    if (!ctx->graph_st &&
        (hipStreamCreateWithFlags(&ctx->graph_st, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&ctx->graph_ev, hipEventDisableTiming) != hipSuccess)) {
      (void)hipGetLastError();
      if (ctx->graph_st) hipStreamDestroy(ctx->graph_st);
      ctx->graph_st = nullptr;
      ctx->graph_ev = nullptr;
    }
    if (ctx->graph_st && hipEventRecord(ctx->graph_ev, rs.st) == hipSuccess &&
        hipStreamWaitEvent(ctx->graph_st, ctx->graph_ev, 0) == hipSuccess)
      gst = ctx->graph_st;
    else
      want_graph = false;
  }
  for (size_t q0 = 0; q0 < qs.size() && rc == TN_OK; q0 += chunk) {
    int Q = (int)std::min(chunk, qs.size() - q0);
    const hipStream_t st = gst ? gst : rs.st;
    // carve the workspace of Q queries
    size_t r_shared = 0, r_perq = 0, r_slots = 0, r_ovr = 0, r_res = 0, r_final = 0, r_part = 0,
           total = 0;
    auto carve_all = [&](int nq) {
      size_t o = 0;
      auto carve = [&](size_t b) {
        size_t r = o;
        o += rnd(b);
        return r;
      };
      r_shared = carve(L.shared_bytes);
      r_perq = carve(perq * nq);
      r_slots = carve(slot_bytes * (nq + 1));
      r_ovr = carve(ovr_bytes * nq);
      r_res = carve(sizeof(Result) * nq);
      r_final = carve(final_bytes * nq);
      r_part = carve((size_t)max_blocks * 16 * nq);
      total = o;
    };
    carve_all(Q);
    // TN_FLAG_GRAPH: the whole group in one chunk, not profiled, not serving
    // (a group whose workspace cannot be kept runs without a graph)
    bool gmode = want_graph;
    const double t_carve = dbg ? ms_since(t_enter) : 0.0;
    size_t rb_bytes = (size_t)Q * (relems * 8 + sizeof(Slot) + sizeof(Result));
    if (gmode) {
      if (!p->graph) p->graph.reset(new GraphEntry());
      GraphEntry &E = *p->graph;
      if (E.layout != &L || E.Q != Q || E.ws_bytes != total) {
        hipStreamSynchronize(st);
        release_graph(ctx, E);
        E.ws = ctx->arena.alloc(total, true);
        E.ws_bytes = total;
        if (E.ws < 0 || hipHostMalloc(&E.pinned, rb_bytes, hipHostMallocDefault) != hipSuccess) {
          if (E.ws >= 0 && !E.pinned) (void)hipGetLastError();
          E.pinned = nullptr;
          release_graph(ctx, E);
          gmode = false;
        } else {
          E.pinned_bytes = rb_bytes;
          E.layout = &L;
          E.Q = Q;
        }
      }
    }
    const bool own_ws = rs.ws < 0 && !rs.ext_ws && !gmode;
    int64_t ws = rs.ext_ws ? 0 : gmode ? p->graph->ws : own_ws ? ctx->arena.alloc(total) : rs.ws;
    // the free space measured above may have been taken meanwhile (serve
    // workers share the arena): fewer queries per chunk
    while (ws < 0 && own_ws && Q > 1) {
      Q = (Q + 1) / 2;
      chunk = (size_t)Q;
      carve_all(Q);
      rb_bytes = (size_t)Q * (relems * 8 + sizeof(Slot) + sizeof(Result));
      ws = ctx->arena.alloc(total);
    }
    const double t_alloc = dbg ? ms_since(t_enter) : 0.0;
    if (ws < 0) {
      set_error("arena exhausted (%zu bytes requested)", total);
      return TN_E_NOMEM;
    }
    bool capturing = false;
    uint8_t *base = rs.ext_ws ? rs.ext_ws : ctx->arena.base() + ws;
    uint8_t *shared_base = base + r_shared, *perq_base = base + r_perq;
    Slot *slots = (Slot *)(base + r_slots);
    Slot *slots_sh = slots, *slots_q = slots + nn;
    // the shared part from the context's cache (read, or filled by this
    // call); not with graphs, nor when the root itself is shared (the whole
    // result is then one shared computation), and never filled by a call
    // that must not allocate
    int rcm = RC_NONE;
    if (share && !gmode && !L.shared[p->root] && ctx->rcache_budget > 0) {
      bool any = L.n_tree_shared > 0;
      for (size_t k = 0; k < p->order.size() && !any; ++k) {
        const int id = p->nodes[p->order[k]].id;
        any = L.shared[id] && !(trees && p->in_tree[id]);
      }
      if (any) {
        ExecLayout &Lm = const_cast<ExecLayout &>(L);
        rcm = rcache_acquire(ctx, Lm, rnd(L.shared_bytes) + rnd(slot_bytes), !rs.ext_ws);
        if (rcm != RC_NONE) {
          shared_base = ctx->arena.base() + L.rc_off;
          slots_sh = (Slot *)(shared_base + rnd(L.shared_bytes));
        }
      }
    }
    uint8_t *ovr_base = base + r_ovr;
    Result *res = (Result *)(base + r_res);
    float2 *fin = (float2 *)(base + r_final);
    double2 *partials = (double2 *)(base + r_part);
    const float2 *leaf_base = (const float2 *)(ctx->arena.base() + p->dev_leaf);
    const uint8_t *desc_base = ctx->arena.base() + p->dev_desc;
    const int64_t perq_el = (int64_t)(perq / 8), perq_sl = (int64_t)nn;
    const int64_t ovr_el = (int64_t)(ovr_bytes / 8);

    std::vector<const float2 *> direct_p(nv, nullptr);
    std::vector<int64_t> direct_bs(nv, 0);
    auto operand = [&](int t) -> Operand {
      Operand o2;
      if (t < nv) {
        if (direct_p[t]) {
          o2.p = direct_p[t];
          o2.bs = direct_bs[t];
          o2.slot = slots_q + t;
          o2.sbs = perq_sl;
        } else if (ovr_off[t] >= 0) {
          o2.p = (const float2 *)(ovr_base + ovr_off[t]);
          o2.bs = ovr_el;
          o2.slot = slots_q + t;
          o2.sbs = perq_sl;
        } else {
          o2.p = leaf_base + p->leaf_off[t];
          o2.bs = 0;
          o2.slot = slots_sh + t;
          o2.sbs = 0;
        }
      } else if (L.shared[t]) {
        o2.p = (const float2 *)(shared_base + L.off[t]);
        o2.bs = 0;
        o2.slot = slots_sh + t;
        o2.sbs = 0;
      } else {
        o2.p = (const float2 *)(perq_base + L.off[t]);
        o2.bs = perq_el;
        o2.slot = slots_q + t;
        o2.sbs = perq_sl;
      }
      return o2;
    };
    auto outop = [&](int t) -> OutOperand {
      Operand i = operand(t);
      OutOperand o2;
      o2.p = const_cast<float2 *>(i.p);
      o2.bs = i.bs;
      o2.slot = const_cast<Slot *>(i.slot);
      o2.sbs = i.sbs;
      return o2;
    };

    {
      // stage overrides (complex64) for every query of the chunk.  Device-
      // resident overrides evenly spaced across the chunk are read in place.
      if (ovr_bytes && so) {
        bool any_staged = false;
        for (int t : ovr) {
          const tn_leaf &l = so->leaves[so_of[t]];
          const int64_t stride = so->strides[so_of[t]];
          if (l.dtype == TN_C64_DEVICE && stride % 8 == 0) {
            direct_p[t] = (const float2 *)((const char *)l.data + (int64_t)q0 * stride);
            direct_bs[t] = stride / 8;
          } else {
            direct_p[t] = nullptr;
            any_staged = true;
          }
        }
        if (any_staged && so->device_out) {
          set_error("every override must be device data read in place (TN_C64_DEVICE, a stride "
                    "that is a multiple of 8 bytes)");
          rc = TN_E_INVALID_ARG;
          goto done;
        }
        if (any_staged) {
          rc = ensure_pinned(rs, ovr_bytes * Q, st);
          if (rc) goto done;
          uint8_t *h = (uint8_t *)*rs.pinned;
          for (int qi = 0; qi < Q; ++qi)
            for (int t : ovr) {
              const tn_leaf &l = so->leaves[so_of[t]];
              if (direct_p[t] || l.dtype == TN_C64_DEVICE) continue;
              tn_leaf lq = l;
              lq.data = (const char *)l.data + (int64_t)(q0 + qi) * so->strides[so_of[t]];
              to_c64(lq, p->leaf[t].size(), (float2 *)(h + (size_t)qi * ovr_bytes + ovr_off[t]));
            }
          TN_HIP(hipMemcpyAsync(ovr_base, h, ovr_bytes * Q, hipMemcpyHostToDevice, st),
                 "override upload");
          // device data whose stride the kernels cannot step: one copy per query
          for (int qi = 0; qi < Q; ++qi)
            for (int t : ovr) {
              const tn_leaf &l = so->leaves[so_of[t]];
              if (direct_p[t] || l.dtype != TN_C64_DEVICE) continue;
              TN_HIP(hipMemcpyAsync(ovr_base + (size_t)qi * ovr_bytes + ovr_off[t],
                                    (const char *)l.data + (int64_t)(q0 + qi) * so->strides[so_of[t]],
                                    p->leaf[t].size() * 8, hipMemcpyDeviceToDevice, st),
                     "device override copy");
            }
        }
      } else if (ovr_bytes) {
        const size_t no = ovr.size();
        std::vector<const tn_leaf *> src((size_t)Q * no, nullptr);
        for (int qi = 0; qi < Q; ++qi) {
          const QueryIO &q = qs[q0 + qi];
          for (int i = 0; i < q.novr; ++i) {
            const size_t k = (size_t)kidx[q.ovr[i].tensor];
            src[(size_t)qi * no + k] = &q.ovr[i];
          }
        }
        bool any_staged = false;
        for (size_t k = 0; k < no; ++k) {
          const int t = ovr[k];
          bool dev = true;
          for (int qi = 0; qi < Q && dev; ++qi) {
            const tn_leaf *s = src[(size_t)qi * no + k];
            dev = s && s->dtype == TN_C64_DEVICE;
          }
          int64_t stride = 0;
          if (dev && Q > 1) {
            const char *b0 = (const char *)src[k]->data;
            stride = (const char *)src[no + k]->data - b0;
            for (int qi = 2; qi < Q && dev; ++qi)
              dev = (const char *)src[(size_t)qi * no + k]->data - b0 == stride * qi;
            dev = dev && stride % 8 == 0;
          }
          if (dev) {
            direct_p[t] = (const float2 *)src[k]->data;
            direct_bs[t] = stride / 8;
          } else {
            direct_p[t] = nullptr;
            any_staged = true;
          }
        }
        if (any_staged) {
          rc = ensure_pinned(rs, ovr_bytes * Q, st);
          if (rc) goto done;
          uint8_t *h = (uint8_t *)*rs.pinned;
          for (int qi = 0; qi < Q; ++qi)
            for (size_t k = 0; k < no; ++k) {
              const int t = ovr[k];
              if (direct_p[t]) continue;
              const tn_leaf *s = src[(size_t)qi * no + k];
              float2 *dst = (float2 *)(h + (size_t)qi * ovr_bytes + ovr_off[t]);
              const int64_t n = p->leaf[t].size();
              if (s && s->dtype != TN_C64_DEVICE)
                to_c64(*s, n, dst);
              else if (!s)
                memcpy(dst, p->leaf_host.data() + p->leaf_off[t], sizeof(float2) * n);
            }
          TN_HIP(hipMemcpyAsync(ovr_base, h, ovr_bytes * Q, hipMemcpyHostToDevice, st),
                 "override upload");
          for (int qi = 0; qi < Q; ++qi)
            for (size_t k = 0; k < no; ++k) {
              const int t = ovr[k];
              const tn_leaf *s = src[(size_t)qi * no + k];
              if (direct_p[t] || !s || s->dtype != TN_C64_DEVICE) continue;
              TN_HIP(hipMemcpyAsync(ovr_base + (size_t)qi * ovr_bytes + ovr_off[t], s->data,
                                    p->leaf[t].size() * 8, hipMemcpyDeviceToDevice, st),
                     "device override copy");
            }
        }
      }
      // result staging on the host: the graph's own buffer, or the shared one
      // (growing it synchronizes the stream first: the override copy above may
      // still read it)
      const bool root_shared = L.shared[p->root] != 0;
      const bool dot_root = nv > 1 && p->nodes[p->root - nv].kind == NK_DOT;
      size_t rb_vals = (size_t)Q * relems * 8, rb_slots = (size_t)Q * sizeof(Slot);
      // results into device memory (no host staging at all)
      const bool devout = so && so->device_out;
      uint8_t *h = nullptr;
      if (gmode) {
        h = (uint8_t *)p->graph->pinned;
      } else if (!devout) {
        // a slice sum needs room for one FP64 result and its scale
        rc = ensure_pinned(rs, sum ? std::max(rb_bytes, relems * 16 + 64) : rb_bytes, st);
        if (rc) goto done;
        h = (uint8_t *)*rs.pinned;
      }
      float2 *hv = (float2 *)h;
      Slot *hs = (Slot *)(h + rb_vals);
      Result *hr = (Result *)(h + rb_vals + rb_slots);
      // a closed root's records go straight to the pinned staging buffer
      // (host memory the device writes to; visible after the synchronize
      // below), which saves the copy back
      Result *res_out = dot_root && !devout && !sum ? hr : res;
      // results straight into the caller's pinned array: complex128 values
      // scaled to 1, a closed root computed by the subtree kernel, no graph
      const bool direct = so && so->dout && out_dtype == TN_C128 && !(flags & TN_FLAG_KEEP_SCALE) &&
                          dot_root && !root_shared && trees && p->in_tree[p->root] && !gmode;
      const Operand R = operand(p->root);
      // TN_FLAG_GRAPH: replay the launch sequence captured with the same
      // workspace, layout and in-place overrides, or capture it now
      bool replay = false;
      if (gmode) {
        GraphEntry &E = *p->graph;
        std::vector<std::pair<const void *, int64_t>> dir;
        for (int t : ovr) dir.push_back({direct_p[t], direct_bs[t]});
        replay = E.exec && dir == E.direct;
        if (!replay) {
          if (E.exec) {
            hipGraphExecDestroy(E.exec);
            E.exec = nullptr;
          }
          E.direct = dir;
          TN_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "graph capture");
          capturing = true;
        }
      }
      if (replay) {
        TN_HIP(hipGraphLaunch(p->graph->exec, st), "graph launch");
      } else {
      // scale records start at zero; not needed when the subtree kernel runs
      // every vertex (it keeps its scales in LDS and writes its results' records)
      if (!(trees && L.all_in_tree)) {
        if (rcm == RC_NONE) {
          TN_HIP(launch_init_slots(st, slots, (int64_t)nn * (Q + 1)), "slot init");
        } else {
          TN_HIP(launch_init_slots(st, slots_q, (int64_t)nn * Q), "slot init");
          if (rcm == RC_FILL) TN_HIP(launch_init_slots(st, slots_sh, (int64_t)nn), "slot init");
        }
      }
      const double t_staged = dbg ? ms_since(t_enter) : 0.0;
      if (dbg)
        fprintf(stderr, "[tn] run_group host: layout %.3f, carve %.3f, alloc %.3f, staged %.3f ms\n",
                t_layout, t_carve, t_alloc, t_staged);
      if (trees) {
        const uint8_t *tb = ctx->arena.base() + L.tree_dev;
        TreeLaunch tl;
        memset(&tl, 0, sizeof(tl));
        tl.hdr = (const TreeHdr *)tb;
        tl.chunks = (const TreeChunk *)(tb + L.tree_chunk_off);
        tl.steps = (const TreeStep *)(tb + L.tree_step_off);
        tl.loads = (const TreeLeafLoad *)(tb + L.tree_load_off);
        tl.sloads = (const TreeSharedLoad *)(tb + L.tree_sload_off);
        tl.sgather = (const int2 *)(tb + L.tree_sg_off);
        tl.image = (const float2 *)(tb + L.tree_img_off);
        tl.lanes = (const TreeLaneRec *)(tb + L.tree_lane_off);
        // overridden leaves in id order: read in place or from the staging block
        for (size_t k = 0; k < ovr.size() && k < (size_t)kTreeMaxOvr; ++k) {
          const int t = ovr[k];
          if (direct_p[t]) {
            tl.ovr[k].p = direct_p[t];
            tl.ovr[k].stride = direct_bs[t];
          } else {
            tl.ovr[k].p = (const float2 *)(ovr_base + ovr_off[t]);
            tl.ovr[k].stride = ovr_el;
          }
        }
        tl.shared_base = shared_base;
        tl.perq_base = perq_base;
        tl.perq_stride = (int64_t)perq;
        tl.slots_sh = slots_sh;
        tl.slots_q = slots_q;
        tl.slot_stride = perq_sl;
        tl.res = res_out;
        tl.dres = direct ? so->dout + (int64_t)q0 * so->dout_stride : nullptr;
        tl.dres_stride = so ? so->dout_stride : 0;
        if (L.n_tree_shared && rcm != RC_READ) {
          tl.nq = 1;
          tl.qw = 1;
          TN_HIP(prof.timed(st, TN_KCLASS_TREE, tree_bytes_sh, tree_flops_sh,
                            [&] { return launch_tree(st, tl, L.n_tree_shared, L.lds_shared, false); }),
                 "subtree kernel (shared)");
        }
        if (L.n_tree_perq) {
          tl.hdr = (const TreeHdr *)tb + L.n_tree_shared;
          tl.nq = Q;
          // a single query runs the level kernel (its waves share the query)
          const bool wave = L.tree_wave && Q > 1, single = L.tree_wave && Q == 1;
          tl.qw = single ? 1 : L.tree_qw;
          const size_t lds = single ? L.lds_perq1 : L.lds_perq;
          TN_HIP(prof.timed(st, wave ? TN_KCLASS_TREE_BATCH : TN_KCLASS_TREE, tree_bytes_q * Q,
                            tree_flops_q * Q,
                            [&] {
                              return wave ? launch_tree_wave(st, tl, L.n_tree_perq, lds)
                                          : launch_tree(st, tl, L.n_tree_perq, lds, true);
                            }),
                 "subtree kernel");
        }
      }
      if (conc) {
        // every partition stream starts after the uploads and slot set-up above
        TN_HIP(hipEventRecord(ctx->part_ev0, st), "partition start");
        for (int k = 0; k < p->K; ++k) TN_HIP(hipStreamWaitEvent(ctx->part_st[k], ctx->part_ev0, 0), "partition start");
      }
      std::vector<char> part_dirty(conc ? p->K : 0, 0);
      // the reduction path (and the read-back) waits for the partitions with
      // work launched since it last waited
      auto join_parts = [&]() -> hipError_t {
        for (int k = 0; k < (int)part_dirty.size(); ++k)
          if (part_dirty[k]) {
            hipError_t e = hipEventRecord(ctx->part_ev[k], ctx->part_st[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, ctx->part_ev[k], 0);
            if (e != hipSuccess) return e;
            part_dirty[k] = 0;
          }
        return hipSuccess;
      };
      for (int j : p->order) {
        const Node &n = p->nodes[j];
        if (trees && p->in_tree[n.id]) continue;
        // TN_FLAG_CONCURRENT: a partition's vertices on its own stream
        hipStream_t xs = st;
        if (conc && n.part >= 0) {
          xs = ctx->part_st[n.part];
          part_dirty[n.part] = 1;
        } else if (conc) {
          TN_HIP(join_parts(), "partition join");
        }
        const bool sh = L.shared[n.id] != 0;
        if (sh && rcm == RC_READ) continue;  // in the cache
        const int nb = sh ? 1 : Q;
        const double wflops = 8.0 * (double)n.weight * nb;
        const double c1b = 8.0 * (double)(n.c1 < nv ? p->leaf[n.c1].size()
                                                    : p->nodes[n.c1 - nv].out.size());
        const double c2b = 8.0 * (double)(n.c2 < nv ? p->leaf[n.c2].size()
                                                    : p->nodes[n.c2 - nv].out.size());
        const double nodeb = (c1b + c2b + 8.0 * (double)std::max<int64_t>(n.out.size(), 1)) * nb;
        if (n.kind == NK_STREAM) {
          TN_HIP(prof.timed(xs, TN_KCLASS_STREAM, nodeb, wflops,
                            [&] {
                              return launch_stream(xs,
                                                   (const StreamDesc *)(desc_base + n.sdesc_off),
                                                   n.nfib, n.ns, operand(n.x), operand(n.y),
                                                   outop(n.id), nb);
                            }),
                 "stream contraction");
        } else if (n.kind == NK_GEMM) {
          Operand A = operand(n.ga), B = operand(n.gb);
          uint8_t *pbase = sh ? shared_base : perq_base;
          // batch stride of the staged copies, in their entries: float2, float
          // (FP32 planes) or bf16 (split planes)
          const int64_t pst = sh ? 0 : n.planes == 2 ? perq_el * 2 : n.planes > 0 ? perq_el * 4 : perq_el;
          const void *ga = A.p, *gb = B.p;
          int64_t gabs = A.bs, gbbs = B.bs;
          const double pbytes = n.planes > 2 ? 8.0 + 2.0 * n.planes : 16.0;
          if (n.pa.needed) {
            void *dst = pbase + L.scr_a[j];
            TN_HIP(prof.timed(xs, TN_KCLASS_PERMUTE, pbytes * n.pa.h.nelem * nb, 0.0,
                              [&] {
                                return launch_permute(
                                    xs, (const PermDesc *)(desc_base + n.pa.desc_off), n.pa.h,
                                    A.p, A.bs, dst, pst, nb, n.planes, n.pa.h.nelem, A.slot,
                                    A.sbs, ktile_of(n, n.M));
                              }),
                   "permute A");
            ga = dst;
            gabs = pst;
          }
          if (n.pb.needed) {
            void *dst = pbase + L.scr_b[j];
            TN_HIP(prof.timed(xs, TN_KCLASS_PERMUTE, pbytes * n.pb.h.nelem * nb, 0.0,
                              [&] {
                                return launch_permute(
                                    xs, (const PermDesc *)(desc_base + n.pb.desc_off), n.pb.h,
                                    B.p, B.bs, dst, pst, nb, n.planes, n.pb.h.nelem, B.slot,
                                    B.sbs, ktile_of(n, n.N));
                              }),
                   "permute B");
            gb = dst;
            gbbs = pst;
          }
          OutOperand C = outop(n.id);
          GemmArgs g;
          memset(&g, 0, sizeof(g));
          g.A = ga;
          g.B = gb;
          g.C = C.p;
          g.sa = A.slot;
          g.sb = B.slot;
          g.sc = C.slot;
          g.lda = n.lda;
          g.ldb = n.ldb;
          g.ldc = n.ldc;
          g.abs = gabs;
          g.bbs = gbbs;
          g.cbs = C.bs;
          g.sabs = A.sbs;
          g.sbbs = B.sbs;
          g.scbs = C.sbs;
          g.M = n.M;
          g.N = n.N;
          g.K = n.K;
          g.opA = n.opA;
          g.opB = n.opB;
          g.planes = n.planes;
          g.pa = n.M * n.K;
          g.pb = n.N * n.K;
          g.ksplit = n.ksplit;
          g.ktile = n.ktile ? 1 : 0;
          g.tile = n.tile;
          // an operand whose planes a GEMM child wrote (unscaled): its batch
          // stride in plane entries, two floats or four bf16 to a complex64
          if (n.fuse_a) {
            g.abs = A.bs * (n.planes == 2 ? 2 : 4);
            g.raw_a = 1;
          }
          if (n.fuse_b) {
            g.bbs = B.bs * (n.planes == 2 ? 2 : 4);
            g.raw_b = 1;
          }
          // this GEMM's result written as its parent's operand planes
          if (n.fo) {
            g.fo_on = 1;
            g.fo_nbits = n.fo_nbits;
            g.fo_mbits = n.fo_mbits;
            g.fo_plane = n.fo_plane;
            memcpy(g.fo_d, n.fo_d, sizeof(g.fo_d));
          }
          g.kchunk = n.kchunk;
          if (n.ksplit > 1) {
            g.part = (float2 *)(pbase + L.partial[j]);
            g.partbs = sh ? 0 : perq_el;
          }
          const int prec = (p->flags & TN_PREC_BF16X3) ? kPrecBF16x3 : kPrecFP32;
          const int form = (p->flags & TN_FORM_3M) ? kForm3M : kForm4M;
          const auto tg = std::chrono::steady_clock::now();
          TN_HIP(prof.timed(xs, n.ktile ? TN_KCLASS_GEMM : TN_KCLASS_GEMM_SMALL, nodeb, wflops,
                            [&] { return launch_gemm(xs, g, prec, form, n.variant, nb); }),
                 "complex GEMM");
          if (dbg_gemm) {
            hipStreamSynchronize(xs);
            fprintf(stderr, "[tn] gemm M %lld N %lld K %lld batch %d: %.3f ms\n", (long long)n.M,
                    (long long)n.N, (long long)n.K, nb, ms_since(tg));
          }
        } else {
          const bool is_root = n.id == p->root;
          TN_HIP(prof.timed(xs, TN_KCLASS_DOT, nodeb, wflops,
                            [&] {
                              return launch_dot(xs, (const DotDesc *)(desc_base + n.ddesc_off),
                                                n.nelem, operand(n.c1), operand(n.c2), outop(n.id),
                                                is_root ? res_out : nullptr, 1, partials,
                                                n.dot_blocks, nb);
                            }),
                 "dot");
        }
      }
      if (conc) TN_HIP(join_parts(), "partition join");
      // result into output-leg order
      if (p->fperm.needed) {
        const int nbf = L.shared[p->root] ? 1 : Q;
        TN_HIP(prof.timed(st, TN_KCLASS_PERMUTE, 16.0 * p->fperm.h.nelem * nbf, 0.0,
                          [&] {
                            return launch_permute(
                                st, (const PermDesc *)(desc_base + p->fperm.desc_off), p->fperm.h,
                                R.p, R.bs, fin, (int64_t)(final_bytes / 8), nbf);
                          }),
               "output permutation");
      }
      // device results not written by the subtree kernel: from the records
      if (devout && !direct)
        TN_HIP(launch_results_to_c128(st, res, root_shared ? 0 : 1, Q,
                                      so->dout + (int64_t)q0 * so->dout_stride, so->dout_stride),
               "result conversion");
      // slices: their sum, on the device, into the staging buffer
      if (sum) {
        const int nq = root_shared ? 1 : Q;
        if (dot_root) {
          TN_HIP(launch_slice_sum_records(st, res, root_shared ? 0 : 1, nq, (Result *)h), "slice sum");
        } else {
          Operand S = R;
          if (p->fperm.needed) {
            S.p = fin;
            S.bs = root_shared ? 0 : (int64_t)(final_bytes / 8);
          }
          TN_HIP(launch_slice_sum_tensors(st, S, nq, (int64_t)relems, (double2 *)h,
                                          (double *)(h + relems * 16)),
                 "slice sum");
        }
      }
      // read back
      if (!dot_root && !devout && !sum) {
        const int rq = root_shared ? 1 : Q;
        if (p->fperm.needed) {
          // the permuted results lie final_bytes apart (256-byte rounded)
          TN_HIP(hipMemcpy2DAsync(hv, relems * 8, fin, final_bytes, relems * 8, rq,
                                  hipMemcpyDeviceToHost, st),
                 "result copy");
        } else {
          const size_t pitch = R.bs ? (size_t)R.bs * 8 : relems * 8;
          TN_HIP(hipMemcpy2DAsync(hv, relems * 8, R.p, pitch, relems * 8, rq,
                                  hipMemcpyDeviceToHost, st),
                 "result copy");
        }
        TN_HIP(hipMemcpy2DAsync(hs, sizeof(Slot), R.slot, (R.sbs ? R.sbs : 1) * sizeof(Slot),
                                sizeof(Slot), rq, hipMemcpyDeviceToHost, st),
               "scale copy");
      }
      if (capturing) {
        hipGraph_t g = nullptr;
        capturing = false;
        TN_HIP(hipStreamEndCapture(st, &g), "graph capture end");
        hipError_t e = hipGraphInstantiate(&p->graph->exec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) p->graph->exec = nullptr;
        TN_HIP(e, "graph instantiate");
        TN_HIP(hipGraphLaunch(p->graph->exec, st), "graph launch");
      }
      }  // not a replay
      const double t_launched = dbg ? ms_since(t_enter) : 0.0;
      TN_HIP(hipStreamSynchronize(st), "stream synchronize");
      if (dbg)
        fprintf(stderr, "[tn] run_group %d queries: host prep+launch %.3f ms, device done at %.3f ms%s\n",
                Q, t_launched, ms_since(t_enter), direct ? " (results written by the kernel)" : "");
      if (prof.on) prof.collect();
      // written by the kernel: only the scales (1) remain, if asked for
      for (int qi = 0; qi < Q && direct && so->log2s; ++qi)
        if (qs[q0 + qi].log2s) *qs[q0 + qi].log2s = 0.0;
      if (sum) {
        if (dot_root) {
          const Result &r = *(const Result *)h;
          const double v[2] = {r.re, r.im};
          sum->add(v, 1, r.log2s);
        } else {
          sum->add((const double *)h, relems, *(const double *)(h + relems * 16));
        }
      }
      for (int qi = 0; qi < Q && !direct && !devout && !sum; ++qi) {
        const QueryIO &q = qs[q0 + qi];
        const bool keep = (flags & TN_FLAG_KEEP_SCALE) != 0;
        if (dot_root) {
          const Result &r = hr[root_shared ? 0 : qi];
          if (keep) {
            write_out(q.out, out_dtype, 0, r.re, r.im);
            if (q.log2s) *q.log2s = r.log2s;
          } else {
            const int e = (int)r.log2s;
            if (e >= -1022 && e <= 1023) {
              const double sc = pow2i(e);
              write_out(q.out, out_dtype, 0, r.re * sc, r.im * sc);
            } else {
              write_out(q.out, out_dtype, 0, std::ldexp(r.re, e), std::ldexp(r.im, e));
            }
            if (q.log2s) *q.log2s = 0.0;
          }
        } else {
          const int src = root_shared ? 0 : qi;
          const Slot &s = hs[src];
          const float2 *v = hv + (size_t)src * relems;
          for (size_t i = 0; i < relems; ++i) {
            if (keep)
              write_out(q.out, out_dtype, i, v[i].x, v[i].y);
            else
              write_out(q.out, out_dtype, i, std::ldexp((double)v[i].x, (int)s.log2s),
                        std::ldexp((double)v[i].y, (int)s.log2s));
          }
          if (q.log2s) *q.log2s = keep ? s.log2s : 0.0;
        }
        if (q.status) *q.status = TN_OK;
      }
      if (dbg) fprintf(stderr, "[tn] run_group results written at %.3f ms\n", ms_since(t_enter));
    }
  done:
    if (capturing) {  // an error while capturing: end the capture, keep nothing
      hipGraph_t g = nullptr;
      if (hipStreamEndCapture(st, &g) == hipSuccess && g) hipGraphDestroy(g);
      p->graph->direct.clear();
    }
    if (rc != TN_OK) {
      hipStreamSynchronize(st);
      if (conc)  // partitions still running read and write this workspace
        for (int k = 0; k < p->K; ++k) hipStreamSynchronize(ctx->part_st[k]);
      prof.pend.clear();
      prof.used = 0;
    }
    rcache_release(ctx, const_cast<ExecLayout &>(L), rcm, rc == TN_OK);
    if (own_ws) ctx->arena.release(ws, total);
  }
  return rc;
}

}  // namespace tn
