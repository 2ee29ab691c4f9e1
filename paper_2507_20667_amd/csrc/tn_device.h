// Descriptor layouts shared by the host scheduler and the gfx950 kernels, and
// the kernel launchers.  Plain structs only; every pointer is a device
// address.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tn {

// Scale record of one tensor: stored values times 2^log2s are the true values;
// maxbits is the IEEE bit pattern of max(|re|, |im|) over the stored values
// (non-negative floats order like their bit patterns, so atomicMax on the bits
// gives the maximum).  A consumer multiplies the stored values by 2^-e, with
// e = floor(log2(max)), and adds e to its own log2s.
struct Slot {
  double log2s;
  uint32_t maxbits;
  uint32_t pad;
};

constexpr int kMaxSeg = 40;     // fused index segments per map (>= legs of dim > 1 of any tensor below 2^40 elements)
constexpr int kStreamMax = 64;  // largest tensor applied by the streaming kernel

// An index space split into segments, innermost first.  Segment i has extent
// ext[i] and contributes idx * s0[i] to a first offset and idx * s1[i] to a
// second one.  pow2 = every extent is a power of two (lg = log2 extent).
struct SegMap {
  int32_t nseg;
  int32_t pow2;
  int64_t ext[kMaxSeg];
  int64_t s0[kMaxSeg];
  int64_t s1[kMaxSeg];
  int32_t lg[kMaxSeg];
};

// Small-operand contraction C = X (.) Y, |Y| <= kStreamMax.  Fibers are the
// values of X's free index; fiber f sits at X offset / C offset given by
// `fib`.  For shared-index value s and Y-free value j:
//   C[co + cy[j]] = sum_s X[xo + xs[s]] * Y[ymap[s * nfy + j]].
struct StreamDesc {
  int64_t nfib;
  int32_t ns, nfy;
  SegMap fib;
  int64_t xs[kStreamMax];
  int64_t cy[kStreamMax];
  int32_t ymap[kStreamMax];
};

// out[o] = in[map(o)]: `map` runs over the output index (innermost first),
// s0 = input stride, s1 = output stride.
struct PermDesc {
  int64_t nelem;
  SegMap map;
  // bit form, valid when bits > 0: element counts are 2^bits and output bit j
  // is input bit inbit[j].
  int32_t bits;
  int32_t inbit[48];
};

// Full inner product of two tensors with the same legs: i runs over A's
// row-major index; map gives (A offset, B offset).
struct DotDesc {
  int64_t nelem;
  SegMap map;
};

// Complex GEMM C[M x N] = op(A) op(B) on interleaved complex64 data.
// opA = 0: A is M x K row-major (lda >= K); 1: A is stored K x M (lda >= M).
// opB = 0: B is K x N row-major (ldb >= N); 1: B is stored N x K (ldb >= K).
// Batched over gridDim.y with element strides *bs (0 = shared operand).
// planes > 0: A and B are instead planes, with opA = 0 and opB = 1: 2 float
// planes (re, im) for FP32, 4 or 6 bf16 planes (the split form of the
// three-term BF16 product) for BF16x3; pa / pb are the plane strides and
// lda / ldb / abs / bbs count plane entries.
// ksplit > 1: the k range is cut into ksplit chunks of kchunk; chunk s of batch
// q writes its M x N partial product (row-major) to part + q * partbs + s * M * N
// and launch_gemm follows with a reduction into C (fixed order: deterministic).
struct GemmArgs {
  const void *A;
  const void *B;
  float2 *C;
  const Slot *sa;
  const Slot *sb;
  Slot *sc;
  int64_t lda, ldb, ldc;
  int64_t abs, bbs, cbs;
  int64_t sabs, sbbs, scbs;
  int64_t M, N, K;
  int32_t opA, opB;
  int32_t tiles_m, tiles_n;
  int32_t planes, ksplit;
  int64_t pa, pb;
  float2 *part;
  int64_t partbs, kchunk;
  // ktile = 1: the planes are k-tiled (row r, k at ((k / 16) * rows + r) * 16
  // + k % 16, rows = M for A and N for B), K a multiple of 16
  int32_t ktile;
  // tile shape (M x N) of the FP32 plane kernel: 0 = 128 x 128, 1 = 64 x
  // 256, 2 = 256 x 64; of the BF16x3 4M kernels on k-tiled planes: 0 = 128 x
  // 128, 1 = 128 x 256, 2 = 256 x 128 (the two wave-group kernel)
  int32_t tile;
  // Kernels on k-tiled planes only (FP32 and BF16x3).  raw_a / raw_b:
  // that operand's planes hold its values as they are, not divided by 2^e of
  // its scale record (a producer GEMM wrote them, see fo_on): the result is
  // multiplied by 2^-e instead, which is exact (and so is the bf16 split of
  // a value times a power of two), so it is the same as from divided planes
  // (values in the normal FP32 range).
  // fo_on: write the result not to C as complex64 but as the consumer's
  // k-tiled operand planes, d of the result index m N + n given bit by bit
  // (bit b of it goes to bit fo_d[b] of d; fo_nbits = log2 N bits of n, then
  // those of m), plane p at C + p fo_plane + d: two float planes (re, im)
  // from the FP32 kernel, four bf16 planes (re hi, re lo, im hi, im lo) from
  // the BF16x3 4M kernels, six (those and (re+im) hi, (re+im) lo) from the
  // BF16x3 3M kernel; fo_plane at most 2^29
  int32_t raw_a, raw_b;
  int32_t fo_on, fo_nbits, fo_mbits;
  int64_t fo_plane;
  uint8_t fo_d[48];
};

// Plane offsets of the result entries a lane holds (GemmArgs::fo_on), in
// bytes from the first plane's base (ES bytes an entry; the planner keeps
// every plane within 4 GiB of it, so offsets are 32-bit).  In the 32 x 32
// accumulator tiles entry v of 32-row block mb and 32-column block nb is row
// mlane + mb 32 + (v / 4) 8 + v % 4 and column ncol + nb 32, with mlane = m0 +
// (the wave's row base) + (lane / 32) 4 and ncol = n0 + (the wave's column
// base) + lane % 32.  The map is linear over disjoint bits: the lane's part is
// mapped once, the entry's (row bits 0, 1, 3, 4, 5, the same for every lane)
// is a sum of per-bit terms.
template <int ES>
struct PlaneOut {
  uint32_t dl[2];
  uint32_t rbit[6];
  __device__ __forceinline__ static int64_t map(const GemmArgs &g, int64_t idx, int base, int nbits) {
    int64_t d = 0;
    for (int b = 0; b < nbits; ++b)
      if ((idx >> b) & 1) d += (int64_t)1 << g.fo_d[base + b];
    return d;
  }
  __device__ __forceinline__ void init(const GemmArgs &g, int64_t mlane, int64_t ncol) {
    const int64_t dm = map(g, mlane, g.fo_nbits, g.fo_mbits);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) dl[nb] = (uint32_t)((dm + map(g, ncol + nb * 32, 0, g.fo_nbits)) * ES);
#pragma unroll
    for (int b = 0; b < 6; ++b) rbit[b] = b < g.fo_mbits ? (uint32_t)(((int64_t)1 << g.fo_d[g.fo_nbits + b]) * ES) : 0u;
  }
  __device__ __forceinline__ uint32_t at(int mb, int nb, int v) const {
    return dl[nb] + (((v & 1) ? rbit[0] : 0u) + ((v & 2) ? rbit[1] : 0u) + ((v & 4) ? rbit[3] : 0u) +
                     ((v & 8) ? rbit[4] : 0u) + (mb ? rbit[5] : 0u));
  }
};

// Block -> (k chunk ks, output tile t) of a GEMM launch.  Blocks go to the
// eight XCDs round robin (block b on XCD b % 8), each XCD with its own L2.
// Without k chunks each XCD takes a contiguous run of tiles, M-tiles
// fastest, so the tiles that share a B panel share an L2.  With k chunks the
// chunk is the fastest index: the blocks of one chunk sit on 8 / gcd(8,
// chunks) XCDs (one when the chunk count is a multiple of eight), so each
// chunk's panels are fetched into that many L2s instead of all eight.
__device__ __forceinline__ void gemm_block_tile(const GemmArgs &g, int &ks, int64_t &t) {
  const int64_t ntiles = (int64_t)g.tiles_m * g.tiles_n;
  if (g.ksplit > 1) {
    ks = (int)(blockIdx.x % (unsigned)g.ksplit);
    t = (int64_t)(blockIdx.x / (unsigned)g.ksplit);
  } else {
    ks = 0;
    t = blockIdx.x;
    if (ntiles % 8 == 0 && ntiles >= 64) t = (t % 8) * (ntiles / 8) + t / 8;
  }
}

// Output order of a permutation into split planes: ktile.on = 1 writes the
// row-major [rows][kdim] index o = r * kdim + k at ((k / 16) * rows + r) * 16
// + k % 16, so that 16 consecutive k of consecutive rows are contiguous (one
// GEMM stage of a tile is one block); kshift = log2(kdim), or -1.
struct KTile {
  int64_t rows, kdim;
  int32_t kshift, on;
};

// One operand of a batched launch: base pointer plus per-query stride.
struct Operand {
  const float2 *p;
  int64_t bs;
  const Slot *slot;
  int64_t sbs;
};
struct OutOperand {
  float2 *p;
  int64_t bs;
  Slot *slot;
  int64_t sbs;
};

// Result of a closed network: FP64 mantissa and FP64 log2 scale.
struct Result {
  double re, im, log2s, pad;
};

// ----------------------------------------------------------- subtree kernel
// A subtree whose vertices are all small runs in one workgroup for a group of
// queries, every operand in LDS.  LDS holds a shared region (leaves no query
// overrides) and one region per query (its overridden leaves and the live
// intermediates).  Locations are float2 offsets; kPerQuery marks the
// per-query region.
constexpr int kTreeSeg = 6;
constexpr int32_t kPerQuery = 1 << 30;
constexpr int kTreeMaxElems = 4096;
constexpr int kTreeChunk = 16;     // steps of one level run between two barriers
constexpr int kTreeMaxOvr = 64;    // overridden leaves read in place per launch
// a per-query subtree's intermediates of at least this many entries live in
// the query's device workspace instead of LDS (kind 3 steps reach them)
constexpr int kTreeSpillElems = 512;

// kind 0, a contraction: C[i] = sum_s A[ca(i) + sa(s)] B[cb(i) + sb(s)].
// kind 1, the closed root: the FP64 inner product sum_s A[sa(s)] B[sb(s)].
// kind 3, kind 0 with some of A, B, C (bits 0, 1, 2 of glob) in the query's
// device workspace: their locations are float2 offsets from its start.
// kind 2, a small operand (a gate) applied along the fibers of a large one:
// A is the large operand X, B the small one Y (<= 16 entries); for every value
// f of X's free index (the map: f -> (X offset ca, C offset cb), nc / nfy
// values) and j < nfy: C[cb(f) + cy[j]] = sum_{s < ns} X[ca(f) + xs[s]] *
// Y[ymap[s * nfy + j]], with ns, nfy in {1, 2, 4}.
// kind 4, result entries of kind 2 steps of one level (one step or several
// independent ones), one entry per lane: lane l < nc reads lane record tab + l
// of the launch's lane table (TreeLaneRec) and computes
// C[c] = sum_{s < ns} X[xa_s] * Y[ya_s] with the scales of its own step
// (nss = 1: the entries of one whole step).  Only single-query groups run
// kind 4 (every group of a program that holds one).
// In the copy the kernels read, a map whose extents are all powers of two
// (pow2) holds extent - 1 (the mask) in place of each extent and zeros in its
// unused segments, and xs, cy and ymap are byte offsets.
struct TreeStep {
  int32_t a, b, c;        // LDS locations of the operands and the result
  int32_t asl, bsl, csl;  // scale index of each (-1: a leaf, scale 1)
  int32_t nc, ns;         // result entries, shared-index entries
  int32_t ncs, nss;       // segment counts of the two maps (kind 2: nss = nfy)
  int32_t kind;
  int32_t pow2;           // every extent a power of two
  // result index -> (A offset, B offset), innermost first (kind 2: fibers)
  int32_t cext[kTreeSeg], ca[kTreeSeg], cb[kTreeSeg], clg[kTreeSeg];
  union {
    struct {  // kinds 0 and 1: shared index -> (A offset, B offset)
      int32_t sext[kTreeSeg], sa[kTreeSeg], sb[kTreeSeg], slg[kTreeSeg];
    };
    struct {  // kind 2
      int32_t xs[4], cy[4], ymap[16];
    };
  };
  int32_t glob;           // kind 3: operands in the query's device workspace
  int32_t tab;            // kind 4: the first lane's record in the lane table
};

// A kind 4 lane's record (32 bytes); kind 5 links use the same layout (see
// tree_chain in tree.hip).  Each address is a 16-bit byte offset in
// its operand's LDS region.  w[0]: xa_0 | xa_1 << 16, w[1]: ya_0 | ya_1 << 16,
// w[2]: c (query region) | csl << 16 | (the step's first entry) << 31,
// w[3]: asl | (X in the shared region) << 15 | bsl << 16 | (Y in the shared
// region) << 31 (scale indices of 15 bits; a leaf operand has the program's
// last record, which no step writes and the prologue clears),
// w[4]: xa_2 | xa_3 << 16, w[5]: ya_2 | ya_3 << 16 (ns = 4 only), w[6], w[7]: 0.
struct TreeLaneRec {
  uint32_t w[8];
};
constexpr int kTreeStepWords = (int)(sizeof(TreeStep) / 4);

struct TreeLeafLoad {
  int32_t lds;      // LDS location (kPerQuery set: per-query region)
  int32_t n;        // entries
  int32_t src;      // which overridden leaf (index into TreeLaunch::ovr)
  int32_t pad;
};

// A chunk: up to kTreeChunk steps of one level (mutually independent).
struct TreeChunk {
  int32_t step0, nsteps;
};

struct TreeHdr {
  int32_t chunk0, nchunks;
  int32_t load0, nloads;             // per-query leaf loads (overridden leaves)
  int32_t shared_elems, perq_elems;  // LDS sizes (float2)
  int32_t nscale;                    // scale records per query
  int32_t root_loc;                  // LDS location of the subtree result
  int32_t root_scale;
  int32_t final_dot;                 // the subtree root is the network's closed root
  int32_t root_elems;
  int32_t root_in_perq;              // result goes to the per-query part
  int64_t root_off;                  // byte offset of the result in its part
  int64_t image_off;                 // shared leaves: offset in the leaf image
  int32_t root_slot;                 // tensor id (slot index) of the result
  int32_t sload0;                    // shared intermediates read from device memory
  int32_t nsloads;                   // (their scale records are 0 .. nsloads-1)
  int32_t nimg;                      // shared leaves copied from the image
  int32_t step0, nsteps;             // the program: every step, chunk by chunk
  int32_t sg0, nsg;                  // gather list of the shared intermediates
  int32_t rec0, nrec;                // kind 4 lane records [rec0, rec0 + nrec)
  int32_t rec_lds;                   // the level kernel copies them into LDS
  int32_t wstep0, wnsteps;           // the batch kernel's program (kind 5 chains)
  int32_t pad;
};

// A shared intermediate that a per-query subtree takes as an input: computed
// once by the shared launch, read from the shared part into the LDS shared
// region, its scale record into every query's scale table.
struct TreeSharedLoad {
  int32_t lds;    // float2 offset in the LDS shared region
  int32_t n;      // entries
  int32_t scale;  // index in the subtree's scale table
  int32_t slot;   // tensor id (its record in the shared scale records)
  int64_t off;    // byte offset in the shared part
};

struct OvrSrc {
  const float2 *p;      // query 0's copy of an overridden leaf
  int64_t stride;       // float2 from one query to the next
};

struct TreeLaunch {
  const TreeHdr *hdr;
  const TreeChunk *chunks;
  const TreeStep *steps;
  const TreeLeafLoad *loads;
  const TreeSharedLoad *sloads;
  const int2 *sgather;  // (LDS float2 offset, shared-part float2 offset) per entry
  const float2 *image;  // shared leaves of every subtree, each in its LDS order
  const TreeLaneRec *lanes;  // kind 4 lane records
  OvrSrc ovr[kTreeMaxOvr];
  uint8_t *shared_base;
  uint8_t *perq_base;
  int64_t perq_stride;  // bytes per query
  Slot *slots_sh;
  Slot *slots_q;
  int64_t slot_stride;  // Slot records per query
  Result *res;
  // when set, a closed root's value goes straight to dres[q * dres_stride]
  // as complex128 (scaled to 1) instead of a Result record
  double2 *dres;
  int64_t dres_stride;
  int32_t nq;           // queries in this launch
  int32_t qw;           // queries per workgroup
};

// Exponent of a scale record's max: floor(log2 x) of the non-negative float
// with bits `bits`; -126 for subnormals, 0 for zero (an all-zero operand is
// scaled by 1, never by an overflowing power of two), 127 for infinity and
// NaN.  A consumer multiplies its operand by 2^-e (exact).
__device__ __forceinline__ int tn_scale_exp(uint32_t bits) {
  const int e = min(max((int)(bits >> 23) - 127, -126), 127);
  return bits == 0u ? 0 : e;
}

// Split x = h + l with h = bf16(x) and l = bf16(x - h), both rounded to nearest
// even (finite inputs; the hardware conversion): the two terms carry 16
// significant bits of x.
typedef __bf16 tn_bf16x2 __attribute__((ext_vector_type(2)));
typedef float tn_f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void tn_split_bf16(float x, uint16_t &h, uint16_t &l) {
  const __bf16 hb = (__bf16)x;
  h = __builtin_bit_cast(uint16_t, hb);
  l = __builtin_bit_cast(uint16_t, (__bf16)(x - (float)hb));
}
// The same for two values at once (one packed conversion for the high and
// one for the low terms): h and l hold the terms of a in bits 0-15 and of b
// in bits 16-31.
__device__ __forceinline__ void tn_split_bf16x2(float a, float b, uint32_t &h, uint32_t &l) {
  const tn_f32x2 v = {a, b};
  h = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, tn_bf16x2));
  const tn_f32x2 r = {a - __uint_as_float(h << 16), b - __uint_as_float(h & 0xffff0000u)};
  l = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, tn_bf16x2));
}

enum GemmForm { kForm4M = 0, kForm3M = 1 };
enum GemmPrec { kPrecFP32 = 0, kPrecBF16x3 = 1 };

// ---------------------------------------------------------------- launchers
hipError_t launch_init_slots(hipStream_t st, Slot *slots, int64_t n);
hipError_t launch_stream(hipStream_t st, const StreamDesc *d_desc, int64_t nfib, int ns,
                         Operand X, Operand Y, OutOperand C, int nbatch);
// out: complex64 (np = 0) or np bf16 planes `pstride` entries apart, holding
// the input divided by 2^e of its scale record `sl` (query stride sbs); obs in
// units of the output's entries (float2, or uint16 for planes)
hipError_t launch_permute(hipStream_t st, const PermDesc *d_desc, const PermDesc &h_desc,
                          const float2 *in, int64_t ibs, void *out, int64_t obs, int nbatch,
                          int np = 0, int64_t pstride = 0, const Slot *sl = nullptr,
                          int64_t sbs = 0, KTile kt = KTile{0, 0, -1, 0});
hipError_t launch_gemm(hipStream_t st, const GemmArgs &g, int prec, int form, int variant,
                       int nbatch);
hipError_t launch_gemm_bf16x3(hipStream_t st, const GemmArgs &g, int form, int nbatch);
hipError_t launch_gemm_f32_planes(hipStream_t st, const GemmArgs &g, int form, int nbatch);
int gemm_planes_tile_m(int v);
int gemm_planes_tile_n(int v);
// tile rows / columns of the BF16x3 kernels: 0 = 128 x 128, 1 = 128 x 256,
// 2 = 256 x 128 (the last two 4M from k-tiled planes only)
int gemm_bf16_tile_m(int v);
int gemm_bf16_tile_n(int v);
hipError_t launch_splitk_reduce(hipStream_t st, const GemmArgs &g, int nbatch);
// k chunks of a GEMM with tiles_m x tiles_n output tiles (1: no split)
int gemm_ksplit(int64_t M, int64_t N, int64_t K, int tile_m, int tile_n, int64_t *kchunk);
hipError_t launch_dot(hipStream_t st, const DotDesc *d_desc, int64_t nelem, Operand A, Operand B,
                      OutOperand C, Result *res, int64_t rbs, double2 *partials, int nblocks,
                      int nbatch);

// dev: the subtrees may hold kind 3 steps (per-query subtrees)
hipError_t launch_tree(hipStream_t st, const TreeLaunch &t, int nsub, size_t lds_bytes, bool dev);
// Per-query launches: every wave takes ceil(qw / 4) queries of its workgroup
// through the whole program on its own (no barrier after the leaves load).
hipError_t launch_tree_wave(hipStream_t st, const TreeLaunch &t, int nsub, size_t lds_bytes);
size_t tree_lds_limit();

// The static scratch array of tn_contract_strided_noalloc (kernels.hip): its
// size, and its device address on `device` (taken once per device with the
// device current, then kept).
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kScratchMaxDevices = 64;
hipError_t scratch_address(int device, void **ptr);
// slice sums (FP64, scales aligned to the largest): nq closed-root records
// into one record, or nq result tensors of n entries into FP64 values and one
// log2 scale
hipError_t launch_slice_sum_records(hipStream_t st, const Result *res, int64_t rbs, int nq, Result *out);
hipError_t launch_slice_sum_tensors(hipStream_t st, Operand R, int nq, int64_t n, double2 *out,
                                    double *out_log2);
// matrix-core rate probe (random or constant operands): `out` holds blocks *
// 256 floats, iters a multiple of 4; the launch's flops in *flops
hipError_t launch_probe_mfma(hipStream_t st, int prec, bool random, float *out, int blocks, int iters,
                             double *flops);
// closed-root records of nq queries (query q's at res[q * rbs]) to
// complex128 values at out[q * stride]
hipError_t launch_results_to_c128(hipStream_t st, const Result *res, int64_t rbs, int nq,
                                  double2 *out, int64_t stride);

// Tile shape variants of the GEMM (index into a table in the kernel file).
int gemm_num_variants();
int gemm_variant_tile_m(int v);
int gemm_variant_tile_n(int v);
int dot_blocks_for(int64_t nelem);

}  // namespace tn
