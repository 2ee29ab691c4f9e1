// gfx950 kernels for the pairwise contractions of a tensor network.
//
//   k_stream       small-operand contraction in one pass over the large operand
//   k_perm_*       leg permutation (the T steps of TTGT, Section 5.1)
//   k_cgemm_*      complex GEMM on the matrix cores (the G step of TTGT),
//                  4M and 3M forms, FP32 and three-term split BF16
//   k_dot_*        full inner product with FP64 accumulation (the closed
//                  network's last contraction)
//
// Every kernel reads the scale records of its operands, multiplies by the
// power of two that brings their maxima to [1, 2), writes the scale of its
// output and contributes to the output's running max (Slot).
#include <mutex>

#include "tn_device.h"

namespace tn {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void wave_atomic_max(uint32_t *p, float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(p, __float_as_uint(v));
}

__device__ __forceinline__ float absmax2(float2 v) { return fmaxf(fabsf(v.x), fabsf(v.y)); }

// --------------------------------------------------------------- slot init
__global__ void k_init_slots(Slot *s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    s[i].log2s = 0.0;
    s[i].maxbits = 0u;
    s[i].pad = 0u;
  }
}

hipError_t launch_init_slots(hipStream_t st, Slot *slots, int64_t n) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_init_slots, dim3((unsigned)blocks), dim3(256), 0, st, slots, n);
  return hipGetLastError();
}

// Segment decode helpers: the map is staged in LDS once per block.
struct SegLds {
  int64_t ext[kMaxSeg], s0[kMaxSeg], s1[kMaxSeg];
  int32_t lg[kMaxSeg];
};

__device__ __forceinline__ void seg_stage(SegLds &L, const SegMap &m, int tid) {
  if (tid < m.nseg) {
    L.ext[tid] = m.ext[tid];
    L.s0[tid] = m.s0[tid];
    L.s1[tid] = m.s1[tid];
    L.lg[tid] = m.lg[tid];
  }
}

__device__ __forceinline__ void seg_decode(const SegLds &L, int nseg, bool pow2, int64_t idx,
                                           int64_t &o0, int64_t &o1) {
  o0 = 0;
  o1 = 0;
  if (pow2) {
    for (int i = 0; i < nseg; ++i) {
      const int64_t v = idx & (L.ext[i] - 1);
      idx >>= L.lg[i];
      o0 += v * L.s0[i];
      o1 += v * L.s1[i];
    }
  } else {
    for (int i = 0; i < nseg; ++i) {
      const int64_t v = idx % L.ext[i];
      idx /= L.ext[i];
      o0 += v * L.s0[i];
      o1 += v * L.s1[i];
    }
  }
}

// ------------------------------------------------------------ stream kernel
// One thread per fiber of X: gather the ns shared-index values, multiply by
// the ns x nfy matrix of Y held in LDS, scatter nfy outputs.  Consecutive
// threads take consecutive fibers, so reads and writes follow X's and C's
// innermost free legs.
template <int NSMAX>
__global__ __launch_bounds__(256) void k_stream(const StreamDesc *__restrict__ d, Operand X,
                                                Operand Y, OutOperand C) {
  __shared__ float2 ys[kStreamMax];
  __shared__ int64_t xs[kStreamMax], cy[kStreamMax];
  __shared__ SegLds L;
  const int tid = threadIdx.x;
  const int q = blockIdx.y;
  const float2 *xp = X.p + q * X.bs;
  const float2 *yp = Y.p + q * Y.bs;
  float2 *cp = C.p + q * C.bs;
  const Slot *xsl = X.slot + q * X.sbs;
  const Slot *ysl = Y.slot + q * Y.sbs;
  Slot *csl = C.slot + q * C.sbs;
  const int ns = d->ns, nfy = d->nfy, nseg = d->fib.nseg;
  const bool p2 = d->fib.pow2 != 0;
  const int64_t nfib = d->nfib;
  const int ex = tn_scale_exp(xsl->maxbits), ey = tn_scale_exp(ysl->maxbits);
  const float fx = ldexpf(1.0f, -ex), fy = ldexpf(1.0f, -ey);
  if (tid < ns * nfy) {
    const float2 v = yp[d->ymap[tid]];
    ys[tid] = make_float2(v.x * fy, v.y * fy);
  }
  if (tid < ns) xs[tid] = d->xs[tid];
  if (tid < nfy) cy[tid] = d->cy[tid];
  seg_stage(L, d->fib, tid);
  __syncthreads();
  if (blockIdx.x == 0 && tid == 0) csl->log2s = xsl->log2s + ysl->log2s + (double)(ex + ey);
  float mx = 0.0f;
  for (int64_t f = (int64_t)blockIdx.x * 256 + tid; f < nfib; f += (int64_t)gridDim.x * 256) {
    int64_t xo, co;
    seg_decode(L, nseg, p2, f, xo, co);
    float2 xv[NSMAX];
#pragma unroll
    for (int s = 0; s < NSMAX; ++s)
      if (s < ns) xv[s] = xp[xo + xs[s]];
    for (int j = 0; j < nfy; ++j) {
      float re = 0.0f, im = 0.0f;
#pragma unroll
      for (int s = 0; s < NSMAX; ++s) {
        if (s < ns) {
          const float2 y = ys[s * nfy + j];
          re = fmaf(xv[s].x, y.x, re);
          re = fmaf(-xv[s].y, y.y, re);
          im = fmaf(xv[s].x, y.y, im);
          im = fmaf(xv[s].y, y.x, im);
        }
      }
      const float2 r = make_float2(re * fx, im * fx);
      cp[co + cy[j]] = r;
      mx = fmaxf(mx, absmax2(r));
    }
  }
  wave_atomic_max(&csl->maxbits, mx);
}

static int grid_for(int64_t work, int64_t per_block, int64_t cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

hipError_t launch_stream(hipStream_t st, const StreamDesc *d_desc, int64_t nfib, int ns, Operand X,
                         Operand Y, OutOperand C, int nbatch) {
  const dim3 grid(grid_for(nfib, 256, 16384), nbatch);
#define TN_STREAM_CASE(NS)                                                            \
  if (ns <= NS) {                                                                     \
    hipLaunchKernelGGL(k_stream<NS>, grid, dim3(256), 0, st, d_desc, X, Y, C);       \
    return hipGetLastError();                                                         \
  }
  TN_STREAM_CASE(1)
  TN_STREAM_CASE(2)
  TN_STREAM_CASE(4)
  TN_STREAM_CASE(8)
  TN_STREAM_CASE(16)
  TN_STREAM_CASE(32)
  TN_STREAM_CASE(64)
#undef TN_STREAM_CASE
  return hipErrorInvalidValue;
}

// -------------------------------------------------------------- permutation
// The output is complex64 (NP = 0); or, for the FP32 GEMM, two float planes
// (NP = 2: re, im); or, for the split-BF16 GEMM, NP bf16 planes (re hi, re
// lo, im hi, im lo [, (re+im) hi, (re+im) lo]).  Planes have the output's
// element order and lie `pstride` entries apart: the split runs once per
// element here instead of once per GEMM tile that reads it.
template <int NP>
__device__ __forceinline__ void perm_emit(void *out, int64_t pstride, int64_t idx, float2 v,
                                          float fs) {
  if (NP == 0) {
    ((float2 *)out)[idx] = v;
  } else if (NP == 2) {
    float *o = (float *)out;
    o[idx] = v.x * fs;
    o[pstride + idx] = v.y * fs;
  } else {
    uint16_t *o = (uint16_t *)out;
    uint16_t h, l;
    v.x *= fs;
    v.y *= fs;
    tn_split_bf16(v.x, h, l);
    o[idx] = h;
    o[pstride + idx] = l;
    tn_split_bf16(v.y, h, l);
    o[2 * pstride + idx] = h;
    o[3 * pstride + idx] = l;
    if (NP == 6) {
      tn_split_bf16(v.x + v.y, h, l);
      o[4 * pstride + idx] = h;
      o[5 * pstride + idx] = l;
    }
  }
}

template <int NP>
__device__ __forceinline__ void *perm_out_base(void *out, int64_t obs, int q) {
  return NP == 0 ? (void *)((float2 *)out + q * obs)
                 : NP == 2 ? (void *)((float *)out + q * obs) : (void *)((uint16_t *)out + q * obs);
}

__device__ __forceinline__ int64_t ktile_index(const KTile &t, int64_t o) {
  if (!t.on) return o;
  int64_t r, k;
  if (t.kshift >= 0) {
    r = o >> t.kshift;
    k = o & (t.kdim - 1);
  } else {
    r = o / t.kdim;
    k = o - r * t.kdim;
  }
  return ((k >> 4) * t.rows + r) * 16 + (k & 15);
}

// Split planes carry the operand divided by 2^e (e from its scale record), as
// the GEMM that reads them expects; complex64 output is copied unscaled.
template <int NP>
__device__ __forceinline__ float perm_scale(const Slot *sl, int64_t sbs, int q) {
  return NP == 0 ? 1.0f : ldexpf(1.0f, -tn_scale_exp(sl[q * sbs].maxbits));
}

// Generic: one thread per output element; writes are contiguous, reads follow
// the map.  Used for small tensors, non-power-of-two legs and permutations
// that keep the innermost legs in place (then reads are contiguous too).
template <int NP>
__global__ __launch_bounds__(256) void k_perm_generic(const PermDesc *__restrict__ d,
                                                      const float2 *in, int64_t ibs, void *out,
                                                      int64_t obs, int64_t pstride,
                                                      const Slot *sl, int64_t sbs, KTile kt) {
  __shared__ SegLds L;
  const int tid = threadIdx.x;
  const int q = blockIdx.y;
  in += q * ibs;
  void *ob = perm_out_base<NP>(out, obs, q);
  const float fs = perm_scale<NP>(sl, sbs, q);
  seg_stage(L, d->map, tid);
  __syncthreads();
  const int nseg = d->map.nseg;
  const bool p2 = d->map.pow2 != 0;
  const int64_t n = d->nelem;
  for (int64_t o = (int64_t)blockIdx.x * 256 + tid; o < n; o += (int64_t)gridDim.x * 256) {
    int64_t io, oo;
    seg_decode(L, nseg, p2, o, io, oo);
    perm_emit<NP>(ob, pstride, ktile_index(kt, oo), in[io], fs);
  }
}

// Tiled bit permutation.  With every extent a power of two the permutation
// moves index bits: output bit j takes input bit inbit[j].  A tile spans the
// lowest input bits and the input bits that feed the lowest output bits
// (nu <= 10 bits, <= 1024 complex values = 8 KiB of LDS); the remaining
// "outer" bits select the tile.  Loads run along the input's low bits and
// stores along the output's low bits, so both sides move whole 256-byte runs.
// A workgroup moves two tiles per round (3.65 -> 4.02 TB/s on the 30-qubit
// operands against one).
struct BitTile {
  int32_t nu;          // tile bits
  int32_t nouter;      // outer bits
  int32_t u_in[12];    // tile bit k -> input bit
  int32_t u_out[12];   // tile bit k -> output bit
  int32_t g_to_k[12];  // output-ordered tile bit -> tile bit
  int32_t o_in[48];    // outer bit -> input bit
  int32_t o_out[48];   // outer bit -> output bit
};

template <int NP>
__global__ __launch_bounds__(256) void k_perm_tiled(BitTile t, const float2 *in, int64_t ibs,
                                                    void *out, int64_t obs, int64_t pstride,
                                                    const Slot *sl, int64_t sbs, KTile kt) {
  // two tiles per round: the loads of both are in flight before the barrier,
  // twice the bytes in flight per workgroup of one round trip
  __shared__ float2 tile[2][1024 + 32];
  const int tid = threadIdx.x;
  const int q = blockIdx.y;
  in += q * ibs;
  void *ob = perm_out_base<NP>(out, obs, q);
  const float fs = perm_scale<NP>(sl, sbs, q);
  const int nt = 1 << t.nu;
  // per-thread offsets of the tile elements this thread loads and stores
  int64_t lin[4], lout[4];
  int le[4], ge[4];
  int cnt = 0;
  for (int e = tid; e < nt; e += 256, ++cnt) {
    int64_t a = 0;
    for (int k = 0; k < t.nu; ++k)
      if ((e >> k) & 1) a += (int64_t)1 << t.u_in[k];
    lin[cnt] = a;
    le[cnt] = e + (e >> 5);
    // output-ordered index g = e: g bit i corresponds to tile bit g_to_k[i]
    int src = 0;
    int64_t b = 0;
    for (int i = 0; i < t.nu; ++i)
      if ((e >> i) & 1) {
        const int k = t.g_to_k[i];
        src |= 1 << k;
        b += (int64_t)1 << t.u_out[k];
      }
    lout[cnt] = b;
    ge[cnt] = src + (src >> 5);
  }
  const int64_t ntiles = (int64_t)1 << t.nouter;
  auto base = [&](int64_t w, int64_t &bin, int64_t &bout) {
    bin = 0;
    bout = 0;
    for (int k = 0; k < t.nouter; ++k)
      if ((w >> k) & 1) {
        bin += (int64_t)1 << t.o_in[k];
        bout += (int64_t)1 << t.o_out[k];
      }
  };
  for (int64_t w = blockIdx.x; w < ntiles; w += 2 * (int64_t)gridDim.x) {
    const int64_t w2 = w + gridDim.x;
    const bool two = w2 < ntiles;
    int64_t bin, bout, bin2 = 0, bout2 = 0;
    base(w, bin, bout);
    if (two) base(w2, bin2, bout2);
    for (int c = 0; c < cnt; ++c) tile[0][le[c]] = in[bin + lin[c]];
    if (two)
      for (int c = 0; c < cnt; ++c) tile[1][le[c]] = in[bin2 + lin[c]];
    __syncthreads();
    for (int c = 0; c < cnt; ++c) perm_emit<NP>(ob, pstride, ktile_index(kt, bout + lout[c]), tile[0][ge[c]], fs);
    if (two)
      for (int c = 0; c < cnt; ++c)
        perm_emit<NP>(ob, pstride, ktile_index(kt, bout2 + lout[c]), tile[1][ge[c]], fs);
    __syncthreads();
  }
}

static bool build_bit_tile(const PermDesc &h, BitTile &t) {
  const int r = h.bits;
  if (r <= 0 || r > 47) return false;
  int outpos[48];
  for (int j = 0; j < r; ++j) outpos[h.inbit[j]] = j;
  // innermost output bits already innermost in the input: nothing to tile
  int same = 0;
  while (same < r && h.inbit[same] == same) ++same;
  if (same >= 5 || same == r) return false;
  bool inu[48] = {false};
  int nu = 0;
  int u_in[12];
  const int b = r < 5 ? r : 5;
  for (int i = 0; i < b; ++i) {
    inu[i] = true;
    u_in[nu++] = i;
  }
  for (int j = 0; j < b; ++j) {
    const int i = h.inbit[j];
    if (!inu[i]) {
      inu[i] = true;
      u_in[nu++] = i;
    }
  }
  for (int i = 0; i < r && nu < 10; ++i)
    if (!inu[i]) {
      inu[i] = true;
      u_in[nu++] = i;
    }
  t.nu = nu;
  for (int k = 0; k < nu; ++k) {
    t.u_in[k] = u_in[k];
    t.u_out[k] = outpos[u_in[k]];
  }
  // output-ordered tile bits: sort tile bits by output position
  int order[12];
  for (int k = 0; k < nu; ++k) order[k] = k;
  for (int a = 0; a < nu; ++a)
    for (int c = a + 1; c < nu; ++c)
      if (t.u_out[order[c]] < t.u_out[order[a]]) {
        const int tmp = order[a];
        order[a] = order[c];
        order[c] = tmp;
      }
  for (int i = 0; i < nu; ++i) t.g_to_k[i] = order[i];
  int no = 0;
  for (int i = 0; i < r; ++i)
    if (!inu[i]) {
      t.o_in[no] = i;
      t.o_out[no] = outpos[i];
      ++no;
    }
  t.nouter = no;
  return true;
}

hipError_t launch_permute(hipStream_t st, const PermDesc *d_desc, const PermDesc &h, const float2 *in,
                          int64_t ibs, void *out, int64_t obs, int nbatch, int np,
                          int64_t pstride, const Slot *sl, int64_t sbs, KTile kt) {
  if (np != 0 && np != 2 && np != 4 && np != 6) return hipErrorInvalidValue;
  if (np != 0 && (!sl || pstride < h.nelem)) return hipErrorInvalidValue;
  if (kt.on && (np == 0 || kt.kdim % 16 != 0 || kt.rows * kt.kdim != h.nelem ||
                (kt.kshift >= 0 && ((int64_t)1 << kt.kshift) != kt.kdim)))
    return hipErrorInvalidValue;
  BitTile t;
  if (h.nelem >= 4096 && build_bit_tile(h, t)) {
    const int64_t ntiles = (int64_t)1 << t.nouter;
    const dim3 grid(grid_for(ntiles, 1, 8192), nbatch);
    if (np == 0)
      hipLaunchKernelGGL(k_perm_tiled<0>, grid, dim3(256), 0, st, t, in, ibs, out, obs, pstride, sl, sbs, kt);
    else if (np == 2)
      hipLaunchKernelGGL(k_perm_tiled<2>, grid, dim3(256), 0, st, t, in, ibs, out, obs, pstride, sl, sbs, kt);
    else if (np == 4)
      hipLaunchKernelGGL(k_perm_tiled<4>, grid, dim3(256), 0, st, t, in, ibs, out, obs, pstride, sl, sbs, kt);
    else
      hipLaunchKernelGGL(k_perm_tiled<6>, grid, dim3(256), 0, st, t, in, ibs, out, obs, pstride, sl, sbs, kt);
    return hipGetLastError();
  }
  const dim3 grid(grid_for(h.nelem, 256, 16384), nbatch);
  if (np == 0)
    hipLaunchKernelGGL(k_perm_generic<0>, grid, dim3(256), 0, st, d_desc, in, ibs, out, obs, pstride, sl, sbs, kt);
  else if (np == 2)
    hipLaunchKernelGGL(k_perm_generic<2>, grid, dim3(256), 0, st, d_desc, in, ibs, out, obs, pstride, sl, sbs, kt);
  else if (np == 4)
    hipLaunchKernelGGL(k_perm_generic<4>, grid, dim3(256), 0, st, d_desc, in, ibs, out, obs, pstride, sl, sbs, kt);
  else
    hipLaunchKernelGGL(k_perm_generic<6>, grid, dim3(256), 0, st, d_desc, in, ibs, out, obs, pstride, sl, sbs, kt);
  return hipGetLastError();
}

// ----------------------------------------------------------------- GEMM FP32
// Block = 4 waves in a 2 x 2 grid; each wave owns (32*WM) x (32*WN) outputs
// as WM x WN tiles of v_mfma_f32_32x32x2_f32.  For that instruction lane l
// supplies A[l%32][l/32] and B[l/32][l%32] of a 32x2 / 2x32 step and holds
// C[8*(v/4) + 4*(l/32) + v%4][l%32] in accumulator v.  A and B tiles are
// staged in LDS as [k][m] / [k][n] interleaved complex, scaled on the way in.
template <int WM, int WN, int FORM>
__global__ __launch_bounds__(256) void k_cgemm_f32(GemmArgs g) {
  constexpr int BM = 64 * WM, BN = 64 * WN, BK = 16, PAD = 2;
  constexpr int NACC = FORM == kForm3M ? 3 : 2;
  __shared__ float2 As[BK][BM + PAD];
  __shared__ float2 Bs[BK][BN + PAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int q = blockIdx.y;
  const float2 *A = (const float2 *)g.A + q * g.abs;
  const float2 *B = (const float2 *)g.B + q * g.bbs;
  float2 *C = g.C + q * g.cbs;
  const Slot *sa = g.sa + q * g.sabs;
  const Slot *sb = g.sb + q * g.sbbs;
  Slot *sc = g.sc + q * g.scbs;
  int ks;
  int64_t tile;
  gemm_block_tile(g, ks, tile);  // XCD-aware block -> (k chunk, tile)
  const int64_t m0 = (tile % g.tiles_m) * BM, n0 = (tile / g.tiles_m) * BN;
  const int64_t kbeg = (int64_t)ks * g.kchunk;
  const int64_t kend = g.K < kbeg + g.kchunk ? g.K : kbeg + g.kchunk;
  const int ea = tn_scale_exp(sa->maxbits), eb = tn_scale_exp(sb->maxbits);
  const float fa = ldexpf(1.0f, -ea), fb = ldexpf(1.0f, -eb);
  if (blockIdx.x == 0 && tid == 0) sc->log2s = sa->log2s + sb->log2s + (double)(ea + eb);

  v16f acc[WM][WN][NACC];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b)
#pragma unroll
      for (int c = 0; c < NACC; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][b][c][v] = 0.0f;

  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int i = 0; i < BM * BK / 256; ++i) {
      const int e = tid + 256 * i;
      int m, k;
      if (g.opA == 0) {
        m = e / BK;
        k = e % BK;
      } else {
        k = e / BM;
        m = e % BM;
      }
      const int64_t gm = m0 + m, gk = k0 + k;
      float2 v = make_float2(0.0f, 0.0f);
      if (gm < g.M && gk < kend) v = g.opA == 0 ? A[gm * g.lda + gk] : A[gk * g.lda + gm];
      As[k][m] = make_float2(v.x * fa, v.y * fa);
    }
#pragma unroll
    for (int i = 0; i < BN * BK / 256; ++i) {
      const int e = tid + 256 * i;
      int n, k;
      if (g.opB == 0) {
        k = e / BN;
        n = e % BN;
      } else {
        n = e / BK;
        k = e % BK;
      }
      const int64_t gn = n0 + n, gk = k0 + k;
      float2 v = make_float2(0.0f, 0.0f);
      if (gn < g.N && gk < kend) v = g.opB == 0 ? B[gk * g.ldb + gn] : B[gn * g.ldb + gk];
      Bs[k][n] = make_float2(v.x * fb, v.y * fb);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const int kr = kk + (lane >> 5);
      float2 a[WM], b[WN];
#pragma unroll
      for (int mb = 0; mb < WM; ++mb) a[mb] = As[kr][wm * 32 * WM + mb * 32 + (lane & 31)];
#pragma unroll
      for (int nb = 0; nb < WN; ++nb) b[nb] = Bs[kr][wn * 32 * WN + nb * 32 + (lane & 31)];
#pragma unroll
      for (int mb = 0; mb < WM; ++mb)
#pragma unroll
        for (int nb = 0; nb < WN; ++nb) {
          if (FORM == kForm4M) {
            acc[mb][nb][0] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(a[mb].x, b[nb].x, acc[mb][nb][0], 0, 0, 0);
            acc[mb][nb][0] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(-a[mb].y, b[nb].y, acc[mb][nb][0], 0, 0, 0);
            acc[mb][nb][1] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(a[mb].x, b[nb].y, acc[mb][nb][1], 0, 0, 0);
            acc[mb][nb][1] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(a[mb].y, b[nb].x, acc[mb][nb][1], 0, 0, 0);
          } else {
            acc[mb][nb][0] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(a[mb].x, b[nb].x, acc[mb][nb][0], 0, 0, 0);
            acc[mb][nb][1] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(a[mb].y, b[nb].y, acc[mb][nb][1], 0, 0, 0);
            acc[mb][nb][NACC - 1] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                a[mb].x + a[mb].y, b[nb].x + b[nb].y, acc[mb][nb][NACC - 1], 0, 0, 0);
          }
        }
    }
    __syncthreads();
  }

  // C (and the max for the scale record), or a split-k partial
  const bool partial = g.ksplit > 1;
  if (partial) C = g.part + q * g.partbs + (int64_t)ks * g.M * g.N;
  const int64_t ldc = partial ? g.N : g.ldc;
  float mx = 0.0f;
#pragma unroll
  for (int mb = 0; mb < WM; ++mb)
#pragma unroll
    for (int nb = 0; nb < WN; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * 32 * WM + mb * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        const int col = wn * 32 * WN + nb * 32 + (lane & 31);
        const int64_t gm = m0 + row, gn = n0 + col;
        float re, im;
        if (FORM == kForm4M) {
          re = acc[mb][nb][0][v];
          im = acc[mb][nb][1][v];
        } else {
          const float t1 = acc[mb][nb][0][v], t2 = acc[mb][nb][1][v], t3 = acc[mb][nb][NACC - 1][v];
          re = t1 - t2;
          im = t3 - t1 - t2;
        }
        if (gm < g.M && gn < g.N) {
          C[gm * ldc + gn] = make_float2(re, im);
          mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
      }
  if (!partial) wave_atomic_max(&sc->maxbits, mx);
}

// Split-k reduction: C[m][n] = sum over chunks s (in order) of the partials,
// and the max for C's scale record.
__global__ __launch_bounds__(256) void k_splitk_reduce(GemmArgs g) {
  const int q = blockIdx.y;
  const int64_t mn = g.M * g.N;
  const float2 *P = g.part + q * g.partbs;
  float2 *C = g.C + q * g.cbs;
  float mx = 0.0f;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < mn; e += (int64_t)gridDim.x * 256) {
    float2 s = P[e];
    for (int c = 1; c < g.ksplit; ++c) {
      const float2 v = P[(int64_t)c * mn + e];
      s.x += v.x;
      s.y += v.y;
    }
    C[(e / g.N) * g.ldc + e % g.N] = s;
    mx = fmaxf(mx, fmaxf(fabsf(s.x), fabsf(s.y)));
  }
  wave_atomic_max(&(g.sc + q * g.scbs)->maxbits, mx);
}

hipError_t launch_splitk_reduce(hipStream_t st, const GemmArgs &g, int nbatch) {
  const dim3 grid(grid_for(g.M * g.N, 256, 4096), nbatch);
  hipLaunchKernelGGL(k_splitk_reduce, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

// Split k when the output tiles alone cannot fill the chip: aim at about 512
// blocks, each chunk at least 1024 deep and a multiple of 32.
int gemm_ksplit(int64_t M, int64_t N, int64_t K, int tile_m, int tile_n, int64_t *kchunk) {
  const int64_t tiles = ((M + tile_m - 1) / tile_m) * ((N + tile_n - 1) / tile_n);
  int s = 1;
  while (tiles * s * 2 <= 512 && K / (s * 2) >= 1024 && s < 64) s *= 2;
  int64_t kc = (K + s - 1) / s;
  kc = (kc + 31) / 32 * 32;
  if (kchunk) *kchunk = kc;
  return (int)((K + kc - 1) / kc);
}

struct GemmVariant {
  int tm, tn;
};
static const GemmVariant kVariants[] = {{128, 128}, {64, 64}};

int gemm_num_variants() { return 2; }
int gemm_variant_tile_m(int v) { return kVariants[v].tm; }
int gemm_variant_tile_n(int v) { return kVariants[v].tn; }

hipError_t launch_gemm(hipStream_t st, const GemmArgs &g0, int prec, int form, int variant,
                       int nbatch) {
  if (prec == kPrecBF16x3) return launch_gemm_bf16x3(st, g0, form, nbatch);
  if (prec != kPrecFP32) return hipErrorInvalidValue;
  if (g0.planes == 2) return launch_gemm_f32_planes(st, g0, form, nbatch);
  if (g0.planes != 0) return hipErrorInvalidValue;
  GemmArgs g = g0;
  const int tm = kVariants[variant].tm, tn = kVariants[variant].tn;
  g.tiles_m = (int)((g.M + tm - 1) / tm);
  g.tiles_n = (int)((g.N + tn - 1) / tn);
  if (g.ksplit < 1) g.ksplit = 1;
  if (g.ksplit == 1) g.kchunk = g.K;
  if (g.kchunk < 1 || (int64_t)g.ksplit * g.kchunk < g.K || (g.ksplit > 1 && !g.part))
    return hipErrorInvalidValue;
  const int64_t tiles = (int64_t)g.tiles_m * g.tiles_n * g.ksplit;
  if (tiles <= 0 || tiles > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tiles, nbatch);
  if (variant == 0) {
    if (form == kForm4M)
      hipLaunchKernelGGL((k_cgemm_f32<2, 2, kForm4M>), grid, dim3(256), 0, st, g);
    else
      hipLaunchKernelGGL((k_cgemm_f32<2, 2, kForm3M>), grid, dim3(256), 0, st, g);
  } else {
    if (form == kForm4M)
      hipLaunchKernelGGL((k_cgemm_f32<1, 1, kForm4M>), grid, dim3(256), 0, st, g);
    else
      hipLaunchKernelGGL((k_cgemm_f32<1, 1, kForm3M>), grid, dim3(256), 0, st, g);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.ksplit == 1) return e;
  return launch_splitk_reduce(st, g, nbatch);
}

// ------------------------------------------------------------------- dot
// Partial sums per block in FP64, then one block per query adds the partials
// in a fixed order (deterministic), normalises the FP64 value to a mantissa in
// [0.5, 1) and writes both the FP64 result and a complex64 copy.
__global__ __launch_bounds__(256) void k_dot_partial(const DotDesc *__restrict__ d, Operand A,
                                                     Operand B, double2 *partials, int nblocks) {
  __shared__ SegLds L;
  __shared__ double red_re[256], red_im[256];
  const int tid = threadIdx.x;
  const int q = blockIdx.y;
  const float2 *ap = A.p + q * A.bs;
  const float2 *bp = B.p + q * B.bs;
  seg_stage(L, d->map, tid);
  __syncthreads();
  const int nseg = d->map.nseg;
  const bool p2 = d->map.pow2 != 0;
  double re = 0.0, im = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < d->nelem; i += (int64_t)nblocks * 256) {
    int64_t ao, bo;
    seg_decode(L, nseg, p2, i, ao, bo);
    const float2 a = ap[ao], b = bp[bo];
    re += (double)a.x * (double)b.x - (double)a.y * (double)b.y;
    im += (double)a.x * (double)b.y + (double)a.y * (double)b.x;
  }
  red_re[tid] = re;
  red_im[tid] = im;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      red_re[tid] += red_re[tid + s];
      red_im[tid] += red_im[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) partials[(int64_t)q * nblocks + blockIdx.x] = make_double2(red_re[0], red_im[0]);
}

__global__ __launch_bounds__(256) void k_dot_final(const double2 *partials, int nblocks, Operand A,
                                                   Operand B, OutOperand C, Result *res,
                                                   int64_t rbs) {
  __shared__ double red_re[256], red_im[256];
  const int tid = threadIdx.x;
  const int q = blockIdx.x;
  double re = 0.0, im = 0.0;
  for (int i = tid; i < nblocks; i += 256) {
    const double2 p = partials[(int64_t)q * nblocks + i];
    re += p.x;
    im += p.y;
  }
  red_re[tid] = re;
  red_im[tid] = im;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      red_re[tid] += red_re[tid + s];
      red_im[tid] += red_im[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const Slot *sa = A.slot + q * A.sbs;
    const Slot *sb = B.slot + q * B.sbs;
    double log2s = sa->log2s + sb->log2s;
    double vr = red_re[0], vi = red_im[0];
    const double m = fmax(fabs(vr), fabs(vi));
    if (m > 0.0 && isfinite(m)) {
      int e;
      frexp(m, &e);
      vr = ldexp(vr, -e);
      vi = ldexp(vi, -e);
      log2s += (double)e;
    }
    if (res) {
      Result *r = res + q * rbs;
      r->re = vr;
      r->im = vi;
      r->log2s = log2s;
      r->pad = 0.0;
    }
    const float2 c = make_float2((float)vr, (float)vi);
    C.p[q * C.bs] = c;
    Slot *sc = C.slot + q * C.sbs;
    sc->log2s = log2s;
    sc->maxbits = __float_as_uint(fmaxf(fabsf(c.x), fabsf(c.y)));
  }
}

int dot_blocks_for(int64_t nelem) { return grid_for(nelem, 256 * 8, 512); }

hipError_t launch_dot(hipStream_t st, const DotDesc *d_desc, int64_t nelem, Operand A, Operand B,
                      OutOperand C, Result *res, int64_t rbs, double2 *partials, int nblocks,
                      int nbatch) {
  hipLaunchKernelGGL(k_dot_partial, dim3(nblocks, nbatch), dim3(256), 0, st, d_desc, A, B, partials,
                     nblocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dot_final, dim3(nbatch), dim3(256), 0, st, partials, nblocks, A, B, C, res,
                     rbs);
  return hipGetLastError();
}

// ------------------------------------------------------- static scratch
// The workspace of tn_contract_strided_noalloc: a fixed array in device
// memory that every GPU the library runs on holds until the process ends, so
// that the call needs no allocation.  Host code never names it directly (in
// host code the name is a host-side stand-in, not a device address): its
// address on each device comes from hipGetSymbolAddress, taken once per
// device with that device current (at context creation) and kept.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void **ptr) {
  static std::mutex mu;
  static void *per_device[kScratchMaxDevices] = {};
  if (device < 0 || device >= kScratchMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!per_device[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    per_device[device] = p;
  }
  *ptr = per_device[device];
  return hipSuccess;
}

// Closed-root result records to complex128 values with the scale folded in
// (as the host does for tn_contract): out[q * stride] = (re, im) * 2^log2s.
__global__ void k_results_to_c128(const Result *res, int64_t rbs, int nq, double2 *out,
                                  int64_t stride) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const Result r = res[q * rbs];
  const int e = (int)r.log2s;
  out[(int64_t)q * stride] = make_double2(ldexp(r.re, e), ldexp(r.im, e));
}

hipError_t launch_results_to_c128(hipStream_t st, const Result *res, int64_t rbs, int nq,
                                  double2 *out, int64_t stride) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_results_to_c128, dim3((nq + 255) / 256), dim3(256), 0, st, res, rbs, nq, out,
                     stride);
  return hipGetLastError();
}

// ----------------------------------------------------------- slice sums
// Slicing: the full contraction is the sum of its slices' (Section 2.2, a sum
// over every bound index in any grouping).  The slice results carry scales
// of their own; the sum aligns them to the largest and adds in FP64, in
// slice order (deterministic).

// Closed roots: nq records (query q's at res[q * rbs]) into one record.
__global__ void k_slice_sum_records(const Result *res, int64_t rbs, int nq, Result *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double emax = -1e300;
  bool any = false;
  for (int q = 0; q < nq; ++q) {
    const Result r = res[q * rbs];
    if (r.re != 0.0 || r.im != 0.0) {
      emax = any ? fmax(emax, r.log2s) : r.log2s;
      any = true;
    }
  }
  double vr = 0.0, vi = 0.0;
  if (any)
    for (int q = 0; q < nq; ++q) {
      const Result r = res[q * rbs];
      const int sh = (int)(r.log2s - emax);
      vr += ldexp(r.re, sh);
      vi += ldexp(r.im, sh);
    }
  double log2s = any ? emax : 0.0;
  const double m = fmax(fabs(vr), fabs(vi));
  if (m > 0.0 && isfinite(m)) {
    int e;
    frexp(m, &e);
    vr = ldexp(vr, -e);
    vi = ldexp(vi, -e);
    log2s += (double)e;
  }
  out->re = vr;
  out->im = vi;
  out->log2s = log2s;
  out->pad = 0.0;
}

// Open results: nq tensors of n complex64 entries (query q's values at
// R.p + q * R.bs with scale record R.slot + q * R.sbs) into out[i] =
// sum_q v_q[i] 2^(l_q - lmax), with lmax (the largest l_q) in *out_log2.
__global__ __launch_bounds__(256) void k_slice_sum_tensors(Operand R, int nq, int64_t n, double2 *out,
                                                           double *out_log2) {
  double lmax = R.slot[0].log2s;
  for (int q = 1; q < nq; ++q) lmax = fmax(lmax, R.slot[q * R.sbs].log2s);
  if (blockIdx.x == 0 && threadIdx.x == 0) *out_log2 = lmax;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double vr = 0.0, vi = 0.0;
    for (int q = 0; q < nq; ++q) {
      const float2 v = R.p[q * R.bs + i];
      const int sh = (int)(R.slot[q * R.sbs].log2s - lmax);
      vr += ldexp((double)v.x, sh);
      vi += ldexp((double)v.y, sh);
    }
    out[i] = make_double2(vr, vi);
  }
}

hipError_t launch_slice_sum_records(hipStream_t st, const Result *res, int64_t rbs, int nq, Result *out) {
  hipLaunchKernelGGL(k_slice_sum_records, dim3(1), dim3(64), 0, st, res, rbs, nq, out);
  return hipGetLastError();
}

hipError_t launch_slice_sum_tensors(hipStream_t st, Operand R, int nq, int64_t n, double2 *out,
                                    double *out_log2) {
  hipLaunchKernelGGL(k_slice_sum_tensors, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, R, nq, n, out,
                     out_log2);
  return hipGetLastError();
}

}  // namespace tn

namespace tn {

// Matrix-core rate probe: every wave runs four independent accumulation
// chains of one MFMA instruction with no memory traffic in the loop (one
// store per lane at the end keeps the chains live), four waves per SIMD.
// RANDOM: each lane holds four A and four B operands of pseudo-random values
// in [-1, 1) (a hash of lane, block and index) and consecutive products
// take different pairs of them.  A matrix unit fed the same operands over
// and over switches few bits and draws little power, so the device holds
// its top clock; on data that changes from product to product, as in a GEMM,
// it may not.  The random rate is the ceiling a GEMM kernel on real data can
// approach; the constant one shows the clock's share of the gap.
template <int PREC, bool RANDOM>
__global__ __launch_bounds__(256) void k_probe_mfma(float *out, int iters, float seed) {
  v16f acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[c][v] = 0.0f;
  auto rnd = [&](uint32_t k) {
    uint32_t h = (blockIdx.x * 256u + threadIdx.x) * 0x9E3779B1u + k * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    // constant operands: per-lane values, fixed for the whole run
    return RANDOM ? ((float)(h >> 8) * (2.0f / 16777216.0f) - 1.0f) * seed
                  : seed + (float)((threadIdx.x + k) & 7) * 0.125f;
  };
  // loop of iters / 4 rounds of 16 products (iters a multiple of 4)
  if (PREC == kPrecFP32) {
    float a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = rnd(j);
      b[j] = rnd(4 + j);
    }
    for (int i = 0; i < iters; i += 4) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[(c + r) & 3], b[c], acc[c], 0, 0, 0);
    }
  } else {
    typedef __bf16 v8b __attribute__((ext_vector_type(8)));
    v8b a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        a[j][e] = (__bf16)rnd(8 * j + e);
        b[j][e] = (__bf16)rnd(32 + 8 * j + e);
      }
    for (int i = 0; i < iters; i += 4) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[(c + r) & 3], b[c], acc[c], 0, 0, 0);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) s += acc[c][v];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// `out` holds blocks * 256 floats; flops per launch returned in *flops.
hipError_t launch_probe_mfma(hipStream_t st, int prec, bool random, float *out, int blocks, int iters,
                             double *flops) {
  if (blocks < 1 || iters < 4 || iters % 4 != 0) return hipErrorInvalidValue;
  const double per = prec == kPrecFP32 ? 2.0 * 32 * 32 * 2 : 2.0 * 32 * 32 * 16;
  *flops = per * 4.0 * iters * (double)blocks * 4.0;
#define TN_PROBE(P, R) hipLaunchKernelGGL((k_probe_mfma<P, R>), dim3(blocks), dim3(256), 0, st, out, iters, 1.0f)
  if (prec == kPrecFP32) {
    if (random) TN_PROBE(kPrecFP32, true);
    else TN_PROBE(kPrecFP32, false);
  } else {
    if (random) TN_PROBE(kPrecBF16x3, true);
    else TN_PROBE(kPrecBF16x3, false);
  }
#undef TN_PROBE
  return hipGetLastError();
}

}  // namespace tn
