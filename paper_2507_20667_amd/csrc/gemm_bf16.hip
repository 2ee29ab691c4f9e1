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
// Block = 4 waves in a 2 x 2 grid; each wave owns 64 x 64 outputs as 2 x 2
// tiles of v_mfma_f32_32x32x16_bf16 (lane l supplies eight consecutive k of
// row l%32 of A and of column l%32 of B; A and B use the same k mapping, so
// the sum over k is the same whatever order the hardware assigns).  Each
// stage moves 16-byte plane vectors into LDS rows padded to 48 bytes (16
// lanes of a fragment read hit distinct banks); the next stage's global loads
// are in flight while the current one multiplies.
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

constexpr int BK16 = 16;   // complex k per stage (one MFMA k-step)
constexpr int ROWH = 24;   // bf16 per LDS row (16 used, 8 of padding)

__device__ __forceinline__ v8bf ld8(const uint16_t *p) { return *(const v8bf *)p; }

__device__ __forceinline__ v8bf neg8(v8bf v) {
  v4u u = *(v4u *)&v;
  u ^= 0x80008000u;
  return *(v8bf *)&u;
}

// 8 consecutive k of one plane row: a 16-byte load when aligned and in range,
// else entry by entry with zeros past the edge
__device__ __forceinline__ v4u load8(const uint16_t *row, int64_t k, int64_t K, bool vec_ok) {
  if (vec_ok && k + 8 <= K) return *(const v4u *)(row + k);
  uint16_t e[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) e[i] = (k + i < K) ? row[k + i] : (uint16_t)0;
  v4u w;
  w.x = e[0] | ((uint32_t)e[1] << 16);
  w.y = e[2] | ((uint32_t)e[3] << 16);
  w.z = e[4] | ((uint32_t)e[5] << 16);
  w.w = e[6] | ((uint32_t)e[7] << 16);
  return w;
}

template <int FORM>
__global__ __launch_bounds__(256) void k_cgemm_bf16x3(GemmArgs g) {
  constexpr int BM = 128, BN = 128, NP = FORM == kForm3M ? 6 : 4;
  constexpr int NACC = FORM == kForm3M ? 3 : 2;
  __shared__ __align__(16) uint16_t As[NP][BM * ROWH];
  __shared__ __align__(16) uint16_t Bs[NP][BN * ROWH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int q = blockIdx.y;
  const uint16_t *A = (const uint16_t *)g.A + q * g.abs;
  const uint16_t *B = (const uint16_t *)g.B + q * g.bbs;
  float2 *C = g.C + q * g.cbs;
  const Slot *sa = g.sa + q * g.sabs;
  const Slot *sb = g.sb + q * g.sbbs;
  Slot *sc = g.sc + q * g.scbs;
  // XCD-aware order: blocks land on the 8 XCDs round-robin; give each XCD a
  // contiguous run of tiles, M-tiles fastest, so that the tiles sharing a B
  // panel run together on one XCD's L2
  const int64_t ntiles = (int64_t)g.tiles_m * g.tiles_n;
  int64_t t = blockIdx.x;
  if (ntiles % 8 == 0 && ntiles >= 64) t = (t % 8) * (ntiles / 8) + t / 8;
  const int64_t m0 = (t % g.tiles_m) * BM, n0 = (t / g.tiles_m) * BN;
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

  // staging: thread -> (row tid/2, k offset 0 or 8) of each plane
  const int srow = tid >> 1, sk = (tid & 1) * 8;
  const bool vec_ok = (g.K % 8) == 0;
  const int64_t gm = m0 + srow, gn = n0 + srow;
  const bool rowA = gm < g.M, rowB = gn < g.N;
  const uint16_t *arow = A + gm * g.lda;
  const uint16_t *brow = B + gn * g.ldb;
  v4u ra[NP], rb[NP];
  const v4u zero = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int pl = 0; pl < NP; ++pl) {
    ra[pl] = rowA ? load8(arow + pl * g.pa, sk, g.K, vec_ok) : zero;
    rb[pl] = rowB ? load8(brow + pl * g.pb, sk, g.K, vec_ok) : zero;
  }
  const int fr = lane & 31, fk = (lane >> 5) * 8;
  for (int64_t k0 = 0; k0 < g.K; k0 += BK16) {
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) {
      *(v4u *)&As[pl][srow * ROWH + sk] = ra[pl];
      *(v4u *)&Bs[pl][srow * ROWH + sk] = rb[pl];
    }
    __syncthreads();
    if (k0 + BK16 < g.K) {
      const int64_t kn = k0 + BK16 + sk;
#pragma unroll
      for (int pl = 0; pl < NP; ++pl) {
        ra[pl] = rowA ? load8(arow + pl * g.pa, kn, g.K, vec_ok) : zero;
        rb[pl] = rowB ? load8(brow + pl * g.pb, kn, g.K, vec_ok) : zero;
      }
    }
    v8bf a[2][NP], b[2][NP];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int pl = 0; pl < NP; ++pl) a[mb][pl] = ld8(&As[pl][(wm * 64 + mb * 32 + fr) * ROWH + fk]);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int pl = 0; pl < NP; ++pl) b[nb][pl] = ld8(&Bs[pl][(wn * 64 + nb * 32 + fr) * ROWH + fk]);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const v8bf arh = a[mb][0], arl = a[mb][1], aih = a[mb][2], ail = a[mb][3];
        const v8bf brh = b[nb][0], brl = b[nb][1], bih = b[nb][2], bil = b[nb][3];
        v16f_b *ac = acc[mb][nb];
        if (FORM == kForm4M) {
          const v8bf naih = neg8(aih), nail = neg8(ail);
          ac[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brh, ac[0], 0, 0, 0);
          ac[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brl, ac[0], 0, 0, 0);
          ac[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, brh, ac[0], 0, 0, 0);
          ac[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(naih, bih, ac[0], 0, 0, 0);
          ac[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(naih, bil, ac[0], 0, 0, 0);
          ac[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nail, bih, ac[0], 0, 0, 0);
          ac[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bih, ac[1], 0, 0, 0);
          ac[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bil, ac[1], 0, 0, 0);
          ac[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, bih, ac[1], 0, 0, 0);
          ac[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, brh, ac[1], 0, 0, 0);
          ac[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, brl, ac[1], 0, 0, 0);
          ac[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, brh, ac[1], 0, 0, 0);
        } else {
          const v8bf ash = a[mb][NP - 2], asl = a[mb][NP - 1];
          const v8bf bsh = b[nb][NP - 2], bsl = b[nb][NP - 1];
          ac[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brh, ac[0], 0, 0, 0);
          ac[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brl, ac[0], 0, 0, 0);
          ac[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, brh, ac[0], 0, 0, 0);
          ac[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, bih, ac[1], 0, 0, 0);
          ac[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, bil, ac[1], 0, 0, 0);
          ac[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, bih, ac[1], 0, 0, 0);
          ac[NACC - 1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ash, bsh, ac[NACC - 1], 0, 0, 0);
          ac[NACC - 1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ash, bsl, ac[NACC - 1], 0, 0, 0);
          ac[NACC - 1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(asl, bsh, ac[NACC - 1], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

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
          C[cm * g.ldc + cn] = make_float2(re, im);
          mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
      }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) atomicMax(&sc->maxbits, __float_as_uint(mx));
}

hipError_t launch_gemm_bf16x3(hipStream_t st, const GemmArgs &g0, int form, int nbatch) {
  GemmArgs g = g0;
  if (g.opA != 0 || g.opB != 1 || g.planes != (form == kForm3M ? 6 : 4)) return hipErrorInvalidValue;
  g.tiles_m = (int)((g.M + 127) / 128);
  g.tiles_n = (int)((g.N + 127) / 128);
  const int64_t tiles = (int64_t)g.tiles_m * g.tiles_n;
  if (tiles <= 0 || tiles > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tiles, nbatch);
  if (form == kForm4M)
    hipLaunchKernelGGL(k_cgemm_bf16x3<kForm4M>, grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL(k_cgemm_bf16x3<kForm3M>, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

}  // namespace tn
