// Complex GEMM on the BF16 matrix cores with a three-term split.
//
// Every FP32 value x is split as x = h + l with h = bf16(x) and l = bf16(x - h)
// (round to nearest even both times), so that h + l carries 16 significant
// bits; a product is then a*b ~ ha*hb + ha*lb + la*hb, the la*lb term (relative
// size 2^-16) dropped, accumulated in FP32 (Henry, Tang and Heinecke, 2019).
// The complex product takes the 4M form (Re = ArBr - AiBi, Im = ArBi + AiBr:
// 12 BF16 products per complex one) or the 3M form (T1 = ArBr, T2 = AiBi,
// T3 = (Ar + Ai)(Br + Bi), Re = T1 - T2, Im = T3 - T1 - T2: 9 products).
//
// The operands arrive already split, as bf16 planes with k contiguous
// (A: [M][K], B: [N][K]; planes re-hi, re-lo, im-hi, im-lo [, sum-hi,
// sum-lo]), written by the permutation kernel that puts them in GEMM order,
// so the split costs one pass over each operand instead of one per tile.
// That kernel also divides each operand by 2^e of its scale record, so the
// planes hold values below 2 in magnitude and the products cannot overflow.
//
// Block = 4 waves in a 2 x 2 grid over a 128 x 128 output tile; each wave owns
// 64 x 64 outputs as 2 x 2 tiles of v_mfma_f32_32x32x16_bf16 (lane l supplies
// eight consecutive k of row l%32 of A and of column l%32 of B; A and B use
// the same k mapping, so the sum over k is the same whatever order the
// hardware assigns).  A stage covers 32 k: each plane row is 64 bytes of LDS,
// its four 16-byte chunks stored in the order chunk ^ ((row / 2) % 4) so that
// the eight rows a group of lanes reads fall on distinct banks.  Global loads
// of the next stage are issued before the current stage's products; the 4M
// form double-buffers LDS (one barrier a stage), the 3M form, with six planes,
// has room for one buffer.  Consecutive products go to different accumulators
// so that no MFMA waits on the previous one.
#include "tn_device.h"

namespace tn {

typedef float v16f_b __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int slot_exp_b(uint32_t bits) {
  if (bits == 0u) return 0;
  const int e = (int)((bits >> 23) & 0xffu);
  if (e == 0xff) return 0;
  if (e == 0) return -126;
  return e - 127;
}

constexpr int BT = 128;     // tile rows (M) and columns (N)
constexpr int BKS = 32;     // k per stage
constexpr int ROWE = BKS;   // bf16 per LDS row (no padding: swizzled chunks)

__device__ __forceinline__ v8bf as_bf(v4u u) { return *(v8bf *)&u; }

__device__ __forceinline__ v4u neg4(v4u u) { return u ^ 0x80008000u; }

// 8 consecutive k of one plane row: a 16-byte load when aligned and in range,
// else entry by entry with zeros past the end of the chunk
__device__ __forceinline__ v4u load8(const uint16_t *row, int64_t k, int64_t kend, bool vec_ok) {
  if (vec_ok && k + 8 <= kend) return *(const v4u *)(row + k);
  uint16_t e[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) e[i] = (k + i < kend) ? row[k + i] : (uint16_t)0;
  v4u w;
  w.x = e[0] | ((uint32_t)e[1] << 16);
  w.y = e[2] | ((uint32_t)e[3] << 16);
  w.z = e[4] | ((uint32_t)e[5] << 16);
  w.w = e[6] | ((uint32_t)e[7] << 16);
  return w;
}

// Product table: (accumulator, A plane, B plane, negate A).  Entries
// alternate accumulators so that consecutive MFMAs are independent.
__device__ constexpr int prod_4m(int i, int f) {
  constexpr int t[12][4] = {{0, 0, 0, 0}, {1, 0, 2, 0}, {0, 0, 1, 0}, {1, 0, 3, 0},
                            {0, 1, 0, 0}, {1, 1, 2, 0}, {0, 2, 2, 1}, {1, 2, 0, 0},
                            {0, 2, 3, 1}, {1, 2, 1, 0}, {0, 3, 2, 1}, {1, 3, 0, 0}};
  return t[i][f];
}
__device__ constexpr int prod_3m(int i, int f) {
  constexpr int t[9][4] = {{0, 0, 0, 0}, {1, 2, 2, 0}, {2, 4, 4, 0}, {0, 0, 1, 0}, {1, 2, 3, 0},
                           {2, 4, 5, 0}, {0, 1, 0, 0}, {1, 3, 2, 0}, {2, 5, 4, 0}};
  return t[i][f];
}

template <int FORM>
__global__ __launch_bounds__(256) void k_cgemm_bf16x3(GemmArgs g) {
  constexpr int NP = FORM == kForm3M ? 6 : 4;
  constexpr int NACC = FORM == kForm3M ? 3 : 2;
  constexpr int NPROD = FORM == kForm3M ? 9 : 12;
  constexpr int NBUF = FORM == kForm3M ? 1 : 2;
  constexpr int PLANE = BT * ROWE;              // bf16 per plane tile
  constexpr int OPER = NP * PLANE;              // one operand's stage
  __shared__ __align__(16) uint16_t lds[NBUF * 2 * OPER];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int q = blockIdx.y;
  const uint16_t *A = (const uint16_t *)g.A + q * g.abs;
  const uint16_t *B = (const uint16_t *)g.B + q * g.bbs;
  const Slot *sa = g.sa + q * g.sabs;
  const Slot *sb = g.sb + q * g.sbbs;
  Slot *sc = g.sc + q * g.scbs;
  // block -> (k chunk, tile); XCD-aware tile order: blocks land on the 8 XCDs
  // round-robin, so give each XCD a contiguous run of tiles, M-tiles fastest,
  // and the tiles that share a B panel run together on one XCD's L2
  const int64_t ntiles = (int64_t)g.tiles_m * g.tiles_n;
  const int ks = (int)(blockIdx.x / ntiles);
  int64_t t = blockIdx.x - (int64_t)ks * ntiles;
  if (ntiles % 8 == 0 && ntiles >= 64) t = (t % 8) * (ntiles / 8) + t / 8;
  const int64_t m0 = (t % g.tiles_m) * BT, n0 = (t / g.tiles_m) * BT;
  const int64_t kbeg = (int64_t)ks * g.kchunk;
  const int64_t kend = g.K < kbeg + g.kchunk ? g.K : kbeg + g.kchunk;
  const int ea = slot_exp_b(sa->maxbits), eb = slot_exp_b(sb->maxbits);
  if (blockIdx.x == 0 && tid == 0) sc->log2s = sa->log2s + sb->log2s + (double)(ea + eb);

  v16f_b acc[2][2][NACC];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < NACC; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][b][c][v] = 0.0f;

  // staging: thread -> rows tid/4 and tid/4 + 64 of every plane, chunk tid%4
  const int srow = tid >> 2, sch = tid & 3;
  const bool vec_ok = (g.K % 8) == 0 && (kbeg % 8) == 0;
  const uint16_t *arow[2], *brow[2];
  bool rowA[2], rowB[2];
  int spos[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int r = srow + 64 * i;
    rowA[i] = m0 + r < g.M;
    rowB[i] = n0 + r < g.N;
    arow[i] = A + (m0 + r) * g.lda;
    brow[i] = B + (n0 + r) * g.ldb;
    spos[i] = r * ROWE + ((sch ^ ((r >> 1) & 3)) * 8);
  }
  v4u ra[NP][2], rb[NP][2];
  const v4u zero = {0u, 0u, 0u, 0u};
  auto gload = [&](int64_t k0) {
    const int64_t k = k0 + sch * 8;
#pragma unroll
    for (int pl = 0; pl < NP; ++pl)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ra[pl][i] = rowA[i] ? load8(arow[i] + pl * g.pa, k, kend, vec_ok) : zero;
        rb[pl][i] = rowB[i] ? load8(brow[i] + pl * g.pb, k, kend, vec_ok) : zero;
      }
  };
  auto lstore = [&](int buf) {
    uint16_t *la = lds + buf * 2 * OPER, *lb = la + OPER;
#pragma unroll
    for (int pl = 0; pl < NP; ++pl)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        *(v4u *)&la[pl * PLANE + spos[i]] = ra[pl][i];
        *(v4u *)&lb[pl * PLANE + spos[i]] = rb[pl][i];
      }
  };
  // fragment rows: (wm|wn)*64 + mb*32 + lane%32; the swizzle term depends on
  // lane%32 alone since the rest is a multiple of 8
  const int fr = lane & 31, fsw = (fr >> 1) & 3, fhalf = lane >> 5;

  const int64_t nk = (kend - kbeg + BKS - 1) / BKS;
  gload(kbeg);
  lstore(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = NBUF == 2 ? (int)(kt & 1) : 0;
    const bool more = kt + 1 < nk;
    if (more) gload(kbeg + (kt + 1) * BKS);
    const uint16_t *la = lds + cur * 2 * OPER, *lb = la + OPER;
#pragma unroll
    for (int ss = 0; ss < 2; ++ss) {
      const int cpos = ((2 * ss + fhalf) ^ fsw) * 8;
      v4u a[2][NP], b[2][NP];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int pl = 0; pl < NP; ++pl)
          a[mb][pl] = *(const v4u *)&la[pl * PLANE + (wm * 64 + mb * 32 + fr) * ROWE + cpos];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int pl = 0; pl < NP; ++pl)
          b[nb][pl] = *(const v4u *)&lb[pl * PLANE + (wn * 64 + nb * 32 + fr) * ROWE + cpos];
#pragma unroll
      for (int pi = 0; pi < NPROD; ++pi) {
        const int c = FORM == kForm3M ? prod_3m(pi, 0) : prod_4m(pi, 0);
        const int ap = FORM == kForm3M ? prod_3m(pi, 1) : prod_4m(pi, 1);
        const int bp = FORM == kForm3M ? prod_3m(pi, 2) : prod_4m(pi, 2);
        const int ng = FORM == kForm3M ? prod_3m(pi, 3) : prod_4m(pi, 3);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          const v8bf av = as_bf(ng ? neg4(a[mb][ap]) : a[mb][ap]);
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb][c] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, as_bf(b[nb][bp]), acc[mb][nb][c], 0, 0, 0);
        }
      }
    }
    if (more) {
      if (NBUF == 1) __syncthreads();
      lstore(NBUF == 2 ? (int)((kt + 1) & 1) : 0);
      __syncthreads();
    }
  }

  // epilogue: C (and the max for the scale record), or a split-k partial
  const bool partial = g.ksplit > 1;
  float2 *C = partial ? g.part + q * g.partbs + (int64_t)ks * g.M * g.N : g.C + q * g.cbs;
  const int64_t ldc = partial ? g.N : g.ldc;
  float mx = 0.0f;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * 64 + mb * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        const int col = wn * 64 + nb * 32 + (lane & 31);
        const int64_t cm = m0 + row, cn = n0 + col;
        float re, im;
        if (FORM == kForm4M) {
          re = acc[mb][nb][0][v];
          im = acc[mb][nb][1][v];
        } else {
          const float t1 = acc[mb][nb][0][v], t2 = acc[mb][nb][1][v], t3 = acc[mb][nb][NACC - 1][v];
          re = t1 - t2;
          im = t3 - t1 - t2;
        }
        if (cm < g.M && cn < g.N) {
          C[cm * ldc + cn] = make_float2(re, im);
          mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
      }
  if (!partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) atomicMax(&sc->maxbits, __float_as_uint(mx));
  }
}

hipError_t launch_gemm_bf16x3(hipStream_t st, const GemmArgs &g0, int form, int nbatch) {
  GemmArgs g = g0;
  if (g.opA != 0 || g.opB != 1 || g.planes != (form == kForm3M ? 6 : 4)) return hipErrorInvalidValue;
  g.tiles_m = (int)((g.M + BT - 1) / BT);
  g.tiles_n = (int)((g.N + BT - 1) / BT);
  if (g.ksplit < 1) g.ksplit = 1;
  if (g.ksplit == 1) g.kchunk = g.K;
  if (g.kchunk < 1 || (int64_t)g.ksplit * g.kchunk < g.K || (g.ksplit > 1 && !g.part))
    return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)g.tiles_m * g.tiles_n * g.ksplit;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks, nbatch);
  if (form == kForm4M)
    hipLaunchKernelGGL(k_cgemm_bf16x3<kForm4M>, grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL(k_cgemm_bf16x3<kForm3M>, grid, dim3(256), 0, st, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.ksplit == 1) return e;
  return launch_splitk_reduce(st, g, nbatch);
}

}  // namespace tn
