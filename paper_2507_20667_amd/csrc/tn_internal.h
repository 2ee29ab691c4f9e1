// Host-side structures of libtn: plans, schedule, execution layouts, the arena
// allocator and the context.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/tn.h"
#include "arena.h"
#include "tn_device.h"

namespace tn {

typedef unsigned __int128 u128;

void set_error(const char *fmt, ...);

// Row-major layout of one tensor: its legs (labels) and their dimensions.
struct Layout {
  std::vector<int64_t> lab;
  std::vector<int64_t> dim;
  int64_t size() const {
    int64_t s = 1;
    for (int64_t d : dim) s *= d;
    return s;
  }
  int rank() const { return (int)lab.size(); }
  int find(int64_t l) const {
    for (size_t i = 0; i < lab.size(); ++i)
      if (lab[i] == l) return (int)i;
    return -1;
  }
  std::vector<int64_t> strides() const {
    std::vector<int64_t> s(lab.size());
    int64_t acc = 1;
    for (int i = (int)lab.size() - 1; i >= 0; --i) {
      s[i] = acc;
      acc *= dim[i];
    }
    return s;
  }
};

enum NodeKind { NK_STREAM = 0, NK_GEMM = 1, NK_DOT = 2 };

struct PermStep {
  bool needed = false;
  Layout dst;
  size_t desc_off = 0;  // byte offset of the PermDesc in the descriptor blob
  PermDesc h;           // host copy (grid sizing, bit tiling)
};

// One internal vertex of the contraction tree and how it runs.
struct Node {
  int id = 0;        // SSA id of the result tensor (nv + j)
  int c1 = 0, c2 = 0;
  int part = -1;     // partition whose subtree holds it; -1 on the reduction path
  NodeKind kind = NK_STREAM;
  Layout out;
  u128 weight = 0;   // 2^vc
  bool tiny = false;
  // NK_STREAM
  int x = 0, y = 0;
  size_t sdesc_off = 0;
  int64_t nfib = 0;
  int ns = 0, nfy = 0;
  // NK_GEMM: A = c1 side, B = c2 side
  int ga = 0, gb = 0;
  PermStep pa, pb;
  int opA = 0, opB = 0;
  int planes = 0;    // > 0: both operands staged as split-BF16 planes
  bool ktile = false;  // planes k-tiled for the direct-to-LDS 4M GEMM
  int ksplit = 1;    // k chunks (partials reduced after the GEMM)
  int64_t kchunk = 0;
  int64_t M = 0, N = 0, K = 0, lda = 0, ldb = 0, ldc = 0;
  int variant = 0;
  int tile = 0;      // FP32 plane kernel tile shape (GemmArgs::tile)
  // FP32 plane GEMMs fused with their GEMM children: fuse_a / fuse_b: that
  // operand's planes are written by the child's epilogue (no permutation;
  // read raw); fo: this GEMM writes its result as its parent's operand
  // planes (GemmArgs::fo_*)
  bool fuse_a = false, fuse_b = false;
  bool fo = false;
  int fo_nbits = 0, fo_mbits = 0;
  int64_t fo_plane = 0;
  uint8_t fo_d[48] = {0};
  // NK_DOT
  size_t ddesc_off = 0;
  int64_t nelem = 0;
  int dot_blocks = 1;
};

// Where every tensor of one execution lives.  Intermediates and scratch are
// either in the shared part (computed once for all queries of a batch) or in
// the per-query part (one copy per query, `perq_stride` bytes apart).
struct ExecLayout {
  std::vector<int64_t> off;       // per tensor id: byte offset in its part (-1: leaf region)
  std::vector<uint8_t> shared;    // per tensor id
  std::vector<int64_t> scr_a, scr_b, partial;  // per node index j (partial: dot blocks or split-k)
  std::vector<int64_t> ovr_off;   // per leaf: offset of its per-query override copy, or -1
  int64_t shared_bytes = 0;
  int64_t perq_bytes = 0;
  int64_t ovr_bytes = 0;          // bytes of one query's override block
  int64_t peak_intermediate = 0;  // live peak (per-query part, intermediates + scratch)
  // subtree programs: [TreeHdr...][TreeStep...][TreeLeafLoad...][image float2...]
  std::vector<uint8_t> tree_blob;
  size_t tree_chunk_off = 0, tree_step_off = 0, tree_load_off = 0, tree_img_off = 0;
  size_t tree_lane_off = 0;  // kind 4 lane records
  // algorithmic bytes and flops of the shared and of one query's subtree
  // launch (profiler), filled on first use under the plan's cache lock
  bool tree_acct = false;
  double tree_bytes_sh = 0, tree_flops_sh = 0, tree_bytes_q = 0, tree_flops_q = 0;
  size_t tree_sload_off = 0, tree_sg_off = 0;
  // shared vertices inside per-query subtrees that run as shared subtrees of
  // their own (computed once, read by the per-query programs)
  std::vector<int> islands;
  int n_tree_shared = 0, n_tree_perq = 0;  // headers: shared subtrees first
  size_t lds_shared = 0, lds_perq = 0;     // dynamic LDS of the two launches
  size_t lds_perq1 = 0;                    // the per-query launch of a single query
  int tree_qw = 1;                         // queries per workgroup (per-query launch)
  bool tree_wave = false;                  // batches of queries run the wave kernel
  bool conc = false;                       // partitions in regions of their own (concurrent)
  std::vector<int> spill;                  // per-query subtree vertices kept in device memory
  bool tree_reads_ovr = false;             // per-query subtrees load overridden leaves
  bool tree_error = false;                 // programs failed the bounds check
  bool all_in_tree = false;                // every vertex runs in the subtree kernel
  int64_t tree_dev = -1;                   // arena offset of the uploaded blob
  size_t tree_dev_bytes = 0;
  // device cache of the shared part: the results of the vertices no
  // override reaches (and their scale records), kept across calls of this
  // layout; every field below is guarded by the context's rcache_mu
  int64_t rc_off = -1;     // arena offset (persistent allocation)
  size_t rc_bytes = 0;
  int rc_state = 0;        // 0 empty, 1 being filled by one call, 2 valid
  int rc_pins = 0;         // calls reading or filling it (not evictable)
  uint64_t rc_used = 0;    // last use (LRU clock)
};

struct tn_plan_impl;

// Launch choices of the subtree kernel for one plan: queries per workgroup
// (0: chosen from the LDS budget), per-query intermediates of at least
// `spill` entries in device memory, packed gate steps of at most `pack_nc`
// entries.
struct TreeKnobs {
  int qw = 0;
  int spill = kTreeSpillElems;
  int pack_nc = 64;
};
// Tuning table (tune.cpp)
struct GemmRule {
  bool bf16 = false, m3 = false;
  int lm = 0, ln = 0, lk = 0;  // ceil log2 of M, N, K
  int tile = 0, ksplit = 0;    // ksplit 0: the heuristic's
};
struct TreeRule {
  uint64_t fingerprint = 0;
  TreeKnobs knobs;
};
struct TuneTable {
  bool loaded = false;
  std::string path;
  std::vector<GemmRule> gemm;
  std::vector<TreeRule> tree;
};
const TuneTable &tune_table();
const GemmRule *tune_gemm(bool bf16, bool m3, int64_t M, int64_t N, int64_t K);
const TreeKnobs *tune_tree(uint64_t fingerprint);

struct ServeState;  // serve.cpp

// Event timing of kernel launches by class (tn_profile_enable).
struct Profiler {
  bool on = false;
  tn_kernel_stats stats[TN_KCLASS_COUNT] = {};
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Pending> pend;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  template <typename F>
  hipError_t timed(hipStream_t st, int cls, double bytes, double flops, F &&launch) {
    if (!on) return launch();
    Pending p{cls, get(), nullptr, bytes, flops};
    if (p.a) hipEventRecord(p.a, st);
    hipError_t e = launch();
    p.b = get();
    if (p.a && p.b) {
      hipEventRecord(p.b, st);
      pend.push_back(p);
    }
    return e;
  }
  // after the stream has synchronized
  void collect() {
    for (const Pending &p : pend) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        stats[p.cls].launches += 1;
        stats[p.cls].seconds += ms * 1e-3;
        stats[p.cls].algo_bytes += p.bytes;
        stats[p.cls].algo_flops += p.flops;
      }
    }
    pend.clear();
    used = 0;
  }
  void destroy() {
    for (hipEvent_t e : pool) hipEventDestroy(e);
    pool.clear();
    pend.clear();
    used = 0;
  }
};

}  // namespace tn

struct tn_ctx {
  tn::Arena arena;
  hipStream_t stream = nullptr;
  int device = 0;
  std::mutex exec_mu;              // tn_contract* are serialized per context
  std::atomic<int> live_plans{0};
  // pinned host staging for overrides and results
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
  tn::ServeState *serve = nullptr;
  std::mutex serve_init_mu;
  tn::Profiler prof;
  // TN_FLAG_GRAPH calls run on a stream of their own (graphs cannot be
  // captured on the null stream), ordered after the caller's stream
  hipStream_t graph_st = nullptr;
  hipEvent_t graph_ev = nullptr;
  // lanes of concurrent plan groups in tn_contract_batch: a stream and a
  // pinned staging buffer each (created on first use)
  struct Lane {
    hipStream_t st = nullptr;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
  };
  std::vector<Lane> lanes;
  hipEvent_t lanes_ev = nullptr;
  // TN_FLAG_CONCURRENT: a stream and an event per partition, and the event
  // that starts them (created on first use)
  std::vector<hipStream_t> part_st;
  std::vector<hipEvent_t> part_ev;
  hipEvent_t part_ev0 = nullptr;
  // this device's static scratch (tn_contract_strided_noalloc), or NULL
  uint8_t *scratch = nullptr;
  // layouts whose shared part is cached in the arena, least recently used
  // evicted first when the cached bytes would exceed the budget
  std::mutex rcache_mu;
  std::vector<tn::ExecLayout *> rcache;
  size_t rcache_bytes = 0, rcache_budget = 0;
  uint64_t rcache_clock = 0;
};

namespace tn {
// A captured launch sequence of one plan group (TN_FLAG_GRAPH) and what it
// was captured with: replayed only when all of it matches.
struct GraphEntry {
  const ExecLayout *layout = nullptr;
  int Q = 0;
  size_t ws_bytes = 0;
  int64_t ws = -1;                 // arena offset of the group's workspace (kept)
  void *pinned = nullptr;          // result staging the graph copies into (kept)
  size_t pinned_bytes = 0;
  std::vector<std::pair<const void *, int64_t>> direct;  // in-place overrides
  hipGraphExec_t exec = nullptr;
};
}  // namespace tn

struct tn_plan {
  tn_ctx *ctx = nullptr;
  uint32_t flags = 0;
  uint64_t fingerprint = 0;      // of the network, partition, tree and flags
  tn::TreeKnobs knobs;           // subtree kernel launch choices
  bool tuned = true;             // the tuning table applies
  int nv = 0;
  int K = 0;
  std::vector<tn::Layout> leaf;
  std::vector<int32_t> partition_of;
  std::vector<int32_t> tree;
  std::vector<tn::Node> nodes;   // SSA order: nodes[j] makes tensor nv + j
  std::vector<int> order;        // execution order (indices into nodes)
  std::vector<int64_t> out_labels;
  bool closed = true;
  int root = 0;                  // SSA id of the root tensor
  tn::PermStep fperm;            // root layout -> output-leg order
  tn::Layout result_layout;
  // leaves as complex64 on the host (for per-query copies) and on the device
  std::vector<float2> leaf_host;
  std::vector<int64_t> leaf_off;  // element offset of each leaf in leaf_host / the leaf region
  std::vector<uint8_t> desc_blob;
  int64_t dev_leaf = -1, dev_desc = -1;  // arena offsets
  size_t dev_leaf_bytes = 0, dev_desc_bytes = 0;
  tn::u128 con_serial = 0, con_par = 0, con_dist = 0, mem = 0;
  int64_t largest = 0;
  int num_gemm = 0, num_tiny = 0, num_stream = 0, num_perm = 0;
  // subtrees of small vertices run by the subtree kernel
  std::vector<char> in_tree;     // per tensor id: internal vertex inside such a subtree
  std::vector<int> tree_roots;   // their root tensor ids, SSA order
  bool use_tree = true;
  tn::ExecLayout plain;          // nothing shared, one query
  std::mutex cache_mu;
  std::map<std::vector<int>, std::shared_ptr<tn::ExecLayout>> layouts;  // by override set
  std::unique_ptr<tn::GraphEntry> graph;  // TN_FLAG_GRAPH: the captured launch sequence
  // slicing (tn_plan_slice): the fixed legs (their dimensions in the sliced
  // network are 1) and, per slice, the sub-tensors of the tensors that carry
  // one; slice s fixes label k to digit k of s in the radix of their original
  // dimensions (the last label fastest)
  int64_t nslices = 0;
  std::vector<int64_t> slice_labels, slice_radix;
  std::vector<int> slice_touched;        // tensor ids
  std::vector<int64_t> slice_sub_off;    // per touched tensor: offset in one slice's block
  int64_t slice_block = 0;               // float2 entries per slice
  std::vector<float2> slice_data;        // nslices * slice_block
  std::vector<tn::Layout> slice_full;    // per touched tensor: its layout before slicing
  // serving: a sliced copy made when a request on this plan cannot fit the
  // arena (freed with the plan)
  std::mutex slice_mu;
  tn_plan *auto_sliced = nullptr;
};

namespace tn {

// plan.cpp
tn_status build_plan(tn_plan *p, const tn_plan_desc *d);
ExecLayout make_exec_layout(const tn_plan *p, const std::vector<int> &overridden, bool share,
                            bool allow_trees, bool conc = false);
std::shared_ptr<ExecLayout> cached_layout(tn_plan *p, const std::vector<int> &overridden,
                                          bool share, bool conc = false);
const char *last_error();

// exec.cpp
struct QueryIO {
  const tn_leaf *ovr = nullptr;
  int32_t novr = 0;
  void *out = nullptr;
  double *log2s = nullptr;
  tn_status *status = nullptr;
};
// Overrides of a group given once with per-query byte strides (query q's copy
// of leaf k at leaves[k].data + q * strides[k]); QueryIO::ovr is then unused.
struct StridedOvr {
  std::vector<tn_leaf> leaves;
  std::vector<int64_t> strides;
  // the results' complex128 array when the device can write it (pinned host
  // memory): its device address and the stride in complex128 elements; the
  // subtree kernel then writes a closed root's values there itself
  double2 *dout = nullptr;
  int64_t dout_stride = 0;
  bool log2s = false;  // the caller asked for scales (written on the host)
  // dout is device memory: every closed root's complex128 value goes there
  // (from the subtree kernel, else converted from its record on the device);
  // nothing is staged through host memory
  bool device_out = false;
};
// Resources of one executing thread: its stream, its pinned staging, an
// optional profiler and optionally a workspace reserved beforehand.
struct ExecRes {
  hipStream_t st = nullptr;
  void **pinned = nullptr;
  size_t *pinned_bytes = nullptr;
  Profiler *prof = nullptr;
  int64_t ws = -1;
  size_t ws_bytes = 0;
  // a workspace outside the arena (the static scratch): its device address
  // and size; the whole group must fit it
  uint8_t *ext_ws = nullptr;
  size_t ext_ws_bytes = 0;
};
// The queries of one group are the slices of a sliced plan: run_group adds
// their results on the device (FP64, scales aligned) instead of returning
// them one by one, and adds each chunk's sum here on the host.
struct SliceSum {
  std::vector<double> acc;  // interleaved complex128 mantissas
  double log2s = 0.0;
  bool any = false;
  void add(const double *v, size_t n, double l) {
    if (!any) {
      acc.assign(v, v + 2 * n);
      log2s = l;
      any = true;
      return;
    }
    const double e = l > log2s ? l : log2s;
    const int sa = (int)(log2s - e), sb = (int)(l - e);
    for (size_t i = 0; i < 2 * n; ++i) acc[i] = std::ldexp(acc[i], sa) + std::ldexp(v[i], sb);
    log2s = e;
  }
};
tn_status run_group(tn_ctx *ctx, tn_plan *p, const std::vector<QueryIO> &qs, tn_dtype out_dtype,
                    uint32_t flags, bool share, ExecRes &rs, const StridedOvr *so = nullptr,
                    SliceSum *sum = nullptr);
// slice.cpp: a sliced copy of a plan (labels given, or chosen so that no
// intermediate exceeds max_intermediate entries), and the contraction of a
// sliced plan (every slice one query, summed)
tn_status make_sliced_plan(tn_ctx *ctx, const tn_plan *p, std::vector<int64_t> labels,
                           int64_t max_intermediate, tn_plan **out);
tn_status run_sliced(tn_ctx *ctx, tn_plan *p, int32_t novr, const tn_leaf *ovr, void *out,
                     tn_dtype out_dtype, double *log2_scale, uint32_t flags, ExecRes &rs);
size_t group_workspace_bytes(const tn_plan *p, const ExecLayout &L, int Q);
tn_status upload_tree_programs(tn_ctx *ctx, const ExecLayout &L, hipStream_t st);
size_t result_elems(const tn_plan *p);
// drops a captured graph with its workspace and pinned buffer (stream idle)
void release_graph(tn_ctx *ctx, GraphEntry &g);

// cache of shared parts (exec.cpp): drop a layout's entry (its plan is freed)
void rcache_drop(tn_ctx *ctx, ExecLayout &L);

// serve.cpp
void serve_shutdown(tn_ctx *ctx);
int serve_pending_on(tn_ctx *ctx, const tn_plan *plan);

}  // namespace tn
