/*
 * tn.h - C ABI of libtn: contraction of a partitioned tensor network on one
 * MI355X (gfx950) GPU.
 *
 * The problem is stated as in Sections 2.1-2.4 and 4 of "Optimizing tensor
 * network partitioning using Simulated Annealing":
 *   - a tensor network G = (V, E) of dense complex tensors with labelled legs;
 *     a label on two slots is a bound edge (the two dimensions must agree), a
 *     label on one slot is an open edge (Section 2.1);
 *   - every bound edge is contracted, pairwise, into one tensor (Section 2.2);
 *   - the order is a full binary contraction tree whose leaves are in
 *     bijection with the tensors (Section 2.3);
 *   - a partitioning K of V that the tree accepts: for every partition a tree
 *     vertex whose leaves are exactly that partition (Section 2.4);
 *   - the partitions are contracted in turn (on one GPU), then the part of the
 *     tree above the partition roots, the reduction path (Section 4, phases 2
 *     and 4).
 * Every pairwise contraction runs as leg permutations and a complex GEMM
 * (TTGT, Section 5.1), or, where one operand is tiny, as a single streaming
 * pass that applies the small tensor in place.
 *
 * Conventions
 *   - No C++ types or exceptions cross this interface.  Every function returns
 *     a tn_status; a negative value is an error and tn_last_error() returns a
 *     thread-local message describing it.  Nothing aborts on bad input.
 *   - Tensors are dense, row-major in the order of their legs (the last leg
 *     varies fastest); complex values are interleaved (re, im).
 *   - Arrays passed in are borrowed for the duration of the call only;
 *     tn_plan_load and tn_serve_submit copy whatever they keep.
 *   - Device memory: the library never allocates device memory on its own.
 *     All device data (leaves, descriptors, intermediates, caches) live in
 *     the arena handed to tn_ctx_create, which stays owned by the caller and
 *     must outlive the context.
 *   - Precision: data on the GPU are complex64; the GEMMs run either in FP32
 *     on the FP32 matrix cores or as a three-term split-BF16 product with FP32
 *     accumulation.  Every intermediate carries an FP64 power-of-two scale
 *     (log2) so that amplitudes cannot underflow, and the final contraction of
 *     a closed network accumulates in FP64.
 */
#ifndef TN_H
#define TN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tn_status;

enum {
  TN_OK = 0,
  TN_PENDING = 1,              /* serve: result not ready yet */
  TN_E_INVALID_ARG = -1,       /* bad pointer, size, dtype or flag */
  TN_E_INVALID_PLAN = -2,      /* the network / partition / tree violates Section 2 */
  TN_E_NOMEM = -3,             /* the arena cannot hold what the call needs */
  TN_E_DEVICE = -4,            /* a HIP runtime call failed */
  TN_E_AGAIN = -5,             /* serve queue full; retry later */
  TN_E_CANCELLED = -6,         /* serve request cancelled (context destroyed) */
  TN_E_UNKNOWN_TICKET = -7     /* serve ticket never issued or already consumed */
};

/* TN_C64_DEVICE is accepted for leaf overrides only: complex64 data already in
 * device memory.  When, within one call, the overrides of a leaf are evenly
 * spaced in memory from query to query, the kernels read them in place;
 * otherwise they are copied device to device.  Such data must stay valid
 * until the call returns (for serving: until the request is polled). */
typedef enum { TN_C64 = 0, TN_C128 = 1, TN_C64_DEVICE = 2 } tn_dtype;

/* flags of tn_plan_load (precision and GEMM form) and of tn_contract* */
enum {
  TN_PREC_FP32 = 0,        /* FP32 complex GEMM on the FP32 matrix cores */
  TN_PREC_BF16X3 = 1,      /* x = h + l split into two BF16 terms; a*b ~ hh + hl + lh */
  TN_FORM_4M = 0,          /* four real products per complex product */
  TN_FORM_3M = 1 << 4,     /* three real products (Gauss) */
  TN_FLAG_KEEP_SCALE = 1 << 8, /* return mantissa and log2 scale separately */
  TN_FLAG_GRAPH = 1 << 9,      /* batched calls: capture each plan group's launch
                                  sequence as a HIP graph and replay it (see
                                  tn_contract_batch) */
  TN_FLAG_CONCURRENT = 1 << 10 /* tn_contract: run the partitions' subtrees side
                                  by side, one stream each (see tn_contract) */
};

typedef struct tn_ctx tn_ctx;   /* arena, stream, caches, scheduler */
typedef struct tn_plan tn_plan; /* immutable after load; shareable across threads */

/*
 * The network, its partitioning and its contraction tree (Sections 2.1-2.4).
 *   num_tensors   |V| >= 1.
 *   rank          d_v for every tensor (0 allowed: a scalar), length |V|.
 *   legs          concatenated edge labels, length sum(d_v).  A bound label
 *                 occurs on exactly two slots of two different tensors, an
 *                 open label on one slot.  Self-loops and labels on three or
 *                 more slots are rejected.
 *   leg_dims      n_{v,a} for every slot (>= 1), same length as legs; both
 *                 slots of a bound label must agree.
 *   data          |V| host pointers, tensor v row-major in its leg order,
 *                 prod(n_{v,.}) elements of data_dtype.
 *   partition_of  partition index of every tensor, values 0..num_partitions-1,
 *                 each value used (cover, disjoint, non-empty).
 *   tree          SSA pairs: internal vertex |V|+j contracts tree[2j] and
 *                 tree[2j+1]; |V|-1 pairs; every vertex but the last is used
 *                 exactly once; the last pair is the root.  The tree must
 *                 accept the partitioning.
 *   output_legs   order of the open labels in the result (each exactly once);
 *                 NULL with num_output_legs == 0 takes them in order of first
 *                 appearance.  A closed network has none and yields a scalar.
 */
typedef struct {
  int32_t num_tensors;
  const int32_t *rank;
  const int64_t *legs;
  const int64_t *leg_dims;
  const void *const *data;
  tn_dtype data_dtype;
  const int32_t *partition_of;
  int32_t num_partitions;
  const int32_t *tree;
  const int64_t *output_legs;
  int32_t num_output_legs;
} tn_plan_desc;

/*
 * Exact cost integers of the loaded plan (Section 3), as (hi, lo) 64-bit
 * halves of 128-bit values:
 *   con_serial  eq. con_serial: sum over internal vertices of 2^vc;
 *   con_par     eq. con_par: heaviest leaf-to-root path, leaf excluded;
 *   con_dist    eq. con_dist with con = con_serial and comm = 0;
 *   mem_elems   eq. mem, in elements.
 * live_peak_bytes is the peak of this library's own execution order (every
 * live intermediate plus TTGT scratch, 256-byte aligned), which eq. mem
 * bounds from below.
 */
typedef struct {
  uint64_t con_serial[2], con_par[2], con_dist[2], mem_elems[2];
  uint64_t live_peak_bytes, largest_intermediate_elems;
  int32_t num_internal_nodes, num_gemm_nodes, num_tiny_nodes;
  int32_t num_stream_nodes, num_permutations;
  uint64_t fingerprint;  /* hash of the network, partition, tree and flags: the
                            key of the plan's entry in the tuning table */
} tn_plan_costs;

/* A leaf override: tensor `tensor` takes `data` (same size) for one query. */
typedef struct {
  int32_t tensor;
  const void *data;
  tn_dtype dtype;
} tn_leaf;

typedef struct {
  tn_plan *plan;
  int32_t num_overrides;
  const tn_leaf *overrides;
} tn_query;

/*
 * Create a context on the current HIP device.
 *   arena_dev_ptr  device memory of arena_bytes bytes (256-byte aligned),
 *                  borrowed until tn_ctx_destroy.
 *   hip_stream     the hipStream_t every launch of this context goes to
 *                  (NULL = the null stream), borrowed.
 *   flags          0.
 * Errors: TN_E_INVALID_ARG for a NULL or misaligned arena; TN_E_DEVICE if
 * pinned staging memory cannot be allocated.
 */
tn_status tn_ctx_create(void *arena_dev_ptr, size_t arena_bytes, void *hip_stream, uint32_t flags,
                        tn_ctx **out);

/* Stop the serve scheduler (pending requests end TN_E_CANCELLED), wait for
 * the device, release host resources.  Plans of this context must be freed
 * first; returns TN_E_INVALID_ARG otherwise. */
tn_status tn_ctx_destroy(tn_ctx *ctx);

/* Message for the last negative status returned on this thread. */
const char *tn_last_error(void);

/*
 * Validate the network, partitioning and tree (TN_E_INVALID_PLAN names the
 * violated condition), derive legs(v) and 2^vc of every vertex, fix the TTGT
 * schedule (leg order of every intermediate, GEMM shapes, which permutations
 * are needed), compute the cost integers and the arena layout, and copy the
 * leaves to the device as complex64.
 *   ctx    may be NULL: the plan is then host-only (validation, schedule and
 *          costs; no device upload) and can only be inspected.
 *   flags  TN_PREC_* | TN_FORM_*.
 * The plan stays valid until tn_plan_free and is read-only.
 */
tn_status tn_plan_load(tn_ctx *ctx, const tn_plan_desc *desc, uint32_t flags, tn_plan **out);
tn_status tn_plan_costs_get(const tn_plan *plan, tn_plan_costs *out);
tn_status tn_plan_free(tn_plan *plan);

/*
 * Slicing on top of partitioning (the paper slices on top of its partitions,
 * Section 5.3.2).  A contraction sums over every bound index (Section 2.2),
 * so fixing some bound legs value by value and adding the results of the
 * fixed networks (the slices) gives the same result with smaller
 * intermediates.  tn_plan_slice makes a new plan of the same network,
 * partitioning and tree in which the bound legs `labels` (num_labels > 0)
 * have dimension 1, or, with num_labels == 0, legs chosen greedily (the leg
 * whose fixing shrinks the current largest intermediate most) until no
 * intermediate holds more than max_intermediate entries.  tn_contract and
 * serving on the sliced plan run every slice as one query of one batch and
 * add the slice results on the device in FP64 (their scales aligned to the
 * largest): the result is the original network's.  Overrides of tensors
 * that carry a sliced leg must be host data of the original (unsliced)
 * shape.  tn_plan_costs_get reports one slice's costs.  The batched calls
 * refuse a sliced plan (TN_E_INVALID_ARG).  The sliced plan is freed with
 * tn_plan_free; the original stays valid.
 * Errors: TN_E_INVALID_ARG (a label that is not a bound leg, no leg to fix,
 * more than 2^24 slices, an already sliced plan), those of tn_plan_load.
 */
tn_status tn_plan_slice(tn_plan *plan, int32_t num_labels, const int64_t *labels,
                        int64_t max_intermediate, tn_plan **out);

/*
 * Contract the plan's network once (the plain path: one launch sequence per
 * tree vertex, nothing cached).  Leaves listed in `overrides` are replaced
 * for this call only.  Synchronous: returns when `out` (host memory, the
 * product of the output dimensions elements of out_dtype, in output-leg order)
 * holds the result.  With TN_FLAG_KEEP_SCALE in `flags` the mantissa is
 * written and *log2_scale receives the FP64 exponent (value = out *
 * 2^log2_scale); otherwise the scale is folded in and log2_scale, if not
 * NULL, receives 0.
 * TN_FLAG_CONCURRENT: the partitions are independent until the
 * cross-partition tree (§3, eqs. con_par and con_dist), so each partition's
 * subtree runs on a stream of its own, side by side, and the cross-partition
 * vertices run on the context's stream once the partitions they read are
 * done.  Each partition takes memory of its own (the workspace is the sum of
 * the partitions' live peaks plus the reduction path's, not their maximum).
 * The results are bit-identical to the serial order: every vertex computes
 * the same values either way.  Without effect on a plan of one partition.
 * Errors: TN_E_INVALID_ARG (host-only plan, bad override or flag), TN_E_NOMEM
 * (the arena cannot hold the workspace), TN_E_DEVICE.
 */
tn_status tn_contract(tn_plan *plan, int32_t num_overrides, const tn_leaf *overrides, void *out,
                      tn_dtype out_dtype, double *log2_scale, uint32_t flags);

/*
 * Contract several queries.  Queries on the same plan run together: every
 * tree vertex whose leaves include no overridden leaf is computed once and
 * shared, and each remaining vertex is one launch over all queries of the
 * plan.  Results as for tn_contract; per_query[i] receives each query's
 * status (may be NULL).  Returns the first error, or TN_OK.
 * TN_FLAG_GRAPH: the launch sequence of each plan's group is captured as a
 * HIP graph on its first run and replayed on later calls with the same plan,
 * overridden leaves, query count and output type (overrides are staged into
 * the group's own workspace first; device overrides read in place are part of
 * the match).  The plan then keeps that workspace and a pinned result buffer
 * until it is freed or a call with another group replaces the graph.  Groups
 * that do not fit the arena at once, and calls while profiling is on, run
 * without a graph.
 */
tn_status tn_contract_batch(tn_ctx *ctx, int32_t num_queries, const tn_query *queries,
                            void *const *outs, tn_dtype out_dtype, double *log2_scales,
                            tn_status *per_query, uint32_t flags);

/*
 * Contract num_queries queries of one plan whose overridden leaves are laid
 * out with fixed strides, as tn_contract_batch does, without per-query
 * descriptors: the host work is independent of the number of queries.
 * This is the batched amplitude form of Section 4: every query keeps the
 * network and the tree and replaces the same leaves (for amplitudes, the
 * output basis vectors).
 *   overrides[k]   leaf tensor id, dtype and query 0's copy of overridden
 *                  leaf k (layout as in tn_leaf);
 *   strides[k]     bytes from one query's copy to the next (0: all queries
 *                  share query 0's copy).  TN_C64_DEVICE data with a stride
 *                  that is a multiple of 8 is read in place by the kernels,
 *                  other data is staged.  The caller keeps the data alive
 *                  and unchanged until the call returns.
 *   out            host memory; query q's result (the product of the output
 *                  dimensions elements of out_dtype) starts out_stride
 *                  elements after query q - 1's.  When out is pinned host
 *                  memory (hipHostMalloc), 16-byte aligned, the results are
 *                  TN_C128 closed amplitudes without TN_FLAG_KEEP_SCALE or
 *                  TN_FLAG_GRAPH, the kernel that computes them writes each
 *                  value into out itself (no staging or conversion on the
 *                  host); the values are the same either way.
 *   log2_scales    num_queries values (TN_FLAG_KEEP_SCALE) or NULL.
 * Errors: TN_E_INVALID_ARG (bad ids, dtypes, strides, out_stride smaller
 * than a result, host-only plan), TN_E_NOMEM, TN_E_DEVICE.  Synchronous.
 */
tn_status tn_contract_strided(tn_plan *plan, int32_t num_queries, int32_t num_overrides,
                              const tn_leaf *overrides, const int64_t *strides, void *out,
                              int64_t out_stride, tn_dtype out_dtype, double *log2_scales,
                              uint32_t flags);

/*
 * tn_contract_strided for callers that cannot allocate memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * The call performs no device or pinned-host allocation of any kind (no
 * hipMalloc, hipHostMalloc, hipFree, no arena allocation): its workspace is a
 * fixed static array in device memory (64 MiB; every GPU the library runs on
 * holds one for the life of the process), the overrides are read in place
 * and the results are written to device memory by the kernels.
 *   overrides, strides  as tn_contract_strided, but every override must be
 *               TN_C64_DEVICE with a stride that is a multiple of 8 bytes.
 *   out         device memory, 16-byte aligned: query q's amplitude as a
 *               complex128 value (scale folded in) at element q * out_stride.
 *   flags       0.
 * Only closed networks (one amplitude per query).  The plan's subtree
 * programs for this set of overridden leaves must already be on the device:
 * run tn_contract_strided once with the same leaves overridden first.
 * Synchronous.  Every call on one GPU shares that GPU's scratch array, which
 * keeps the last call's contents: calls that overlap on one GPU (from two
 * contexts, or with another process's calls) race on it; calls on one
 * context are serialized.
 * Errors: TN_E_INVALID_ARG (host override data, bad stride, open network,
 * programs not yet on the device, bad out), TN_E_NOMEM (the workspace of
 * num_queries queries exceeds the 64 MiB scratch; split the call),
 * TN_E_DEVICE.
 */
tn_status tn_contract_strided_noalloc(tn_plan *plan, int32_t num_queries, int32_t num_overrides,
                                      const tn_leaf *overrides, const int64_t *strides, void *out,
                                      int64_t out_stride, uint32_t flags);

/*
 * Serving.  tn_serve_submit copies the query and returns a ticket at once
 * (TN_E_AGAIN when the queue is full).  A library thread admits queued
 * requests while their workspace fits the free arena, groups admitted
 * requests on the same plan into one batched launch sequence and completes
 * them, so requests that arrive while others run join the next batch
 * (continuous batching); batches of different worker threads (each with its
 * own stream; TN_SERVE_WORKERS, default 2) overlap on the device.  Admission
 * reserves a batch's whole workspace in the arena first; a request that cannot
 * fit even alone on an idle device ends with TN_E_NOMEM.  Host override data
 * is copied at submit; TN_C64_DEVICE data must stay valid until polled.
 * tn_serve_poll returns TN_PENDING until the result is ready; then it writes
 * the result (as tn_contract does: the mantissa with *log2_scale = the FP64
 * exponent when log2_scale is not NULL, the scaled value otherwise), sets
 * *latency_s (may be NULL) to the submit-to-ready time in seconds and
 * consumes the ticket.  A plan cannot be freed while requests on it are
 * pending.  Both calls are thread-safe.
 */
tn_status tn_serve_submit(tn_ctx *ctx, const tn_query *query, uint64_t *ticket);
tn_status tn_serve_poll(tn_ctx *ctx, uint64_t ticket, void *out, tn_dtype out_dtype,
                        double *log2_scale, double *latency_s);

/*
 * Kernel timing.  While enabled, every launch of the classes below is
 * bracketed by HIP events on the context's stream, and its algorithmic
 * traffic and work are accumulated (per tree vertex instance: 8 bytes per
 * complex64 entry of each operand and of the result, 16 bytes per entry moved
 * by a permutation; 8 * 2^vc real flops, the 4M count, per contraction).
 * The figures are collected when a contraction call synchronizes.
 * tn_profile_read copies TN_KCLASS_COUNT records and, with reset != 0,
 * clears them.  Timing adds two event records per launch; measure throughput
 * with it disabled.
 */
enum {
  TN_KCLASS_STREAM = 0,   /* small-operand contraction */
  TN_KCLASS_PERMUTE = 1,  /* leg permutation */
  TN_KCLASS_GEMM = 2,     /* complex GEMM */
  TN_KCLASS_DOT = 3,      /* FP64 inner product */
  TN_KCLASS_TREE = 4,     /* whole small subtrees in one workgroup: one query
                             per launch (the shared subtrees, single queries) */
  TN_KCLASS_TREE_BATCH = 5, /* the same for a batch of queries, every wave
                               taking its own queries through the subtree */
  TN_KCLASS_GEMM_SMALL = 6, /* complex GEMM on the register-tiled kernels
                               (operands not stored as k-tiled planes); the
                               GEMM class above is the k-tiled matrix-core
                               kernels with their split-k reduction */
  TN_KCLASS_COUNT = 7
};
typedef struct {
  uint64_t launches;
  double seconds;     /* sum of event-measured launch durations */
  double algo_bytes;  /* algorithmic HBM bytes */
  double algo_flops;  /* algorithmic real flops */
} tn_kernel_stats;

tn_status tn_profile_enable(tn_ctx *ctx, int enable);
tn_status tn_profile_read(tn_ctx *ctx, tn_kernel_stats *out, int reset);

/*
 * Measurement support, not an operation of the method: the rate the matrix
 * cores sustain on this device with no memory traffic (four independent
 * accumulation chains per wave, four waves per SIMD, one timed launch of
 * about 40 ms on the context's stream, long enough for the clock to settle
 * where a long GEMM runs).  precision: TN_PREC_FP32
 * (v_mfma_f32_32x32x2_f32) or TN_PREC_BF16X3 (v_mfma_f32_32x32x16_bf16),
 * optionally or-ed with TN_PROBE_CONST_OPERANDS.  By default each product
 * takes operands of pseudo-random values that change from one product to
 * the next, as a GEMM on real data does: the matrix cores then draw more
 * power and the device may lower its clock, so this rate, not the nominal
 * peak, is the ceiling a GEMM kernel can approach.  With
 * TN_PROBE_CONST_OPERANDS every product repeats the same operands (little
 * switching, the top clock).  *tflops receives the achieved TFLOP/s.
 * Borrows 1 MiB of the arena for the call.
 * Errors: TN_E_INVALID_ARG, TN_E_NOMEM (arena full), TN_E_DEVICE.
 */
#define TN_PROBE_CONST_OPERANDS (1u << 8)
tn_status tn_probe_mfma(tn_ctx *ctx, uint32_t precision, double *tflops);

#ifdef __cplusplus
}
#endif

#endif /* TN_H */
