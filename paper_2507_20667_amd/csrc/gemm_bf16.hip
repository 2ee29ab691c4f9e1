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
// Block = 4 waves in a 2 x 2 grid; each wave owns 64 x 64 outputs as 2 x 2
// tiles of v_mfma_f32_32x32x16_bf16 (lane l supplies eight consecutive k of
// row l%32 of A and of column l%32 of B; A and B use the same k mapping, so
// the sum over k is the same whatever order the hardware assigns).  Tiles
// are split while staged into LDS as bf16 planes [row][k], rows padded to 48
// bytes so that the 16-byte fragment reads of 16 lanes hit distinct banks.
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

// bf16 bits of x rounded to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void split(float x, uint16_t &h, uint16_t &l) {
  const uint32_t hb = bf16_rne(x);
  h = (uint16_t)hb;
  l = (uint16_t)bf16_rne(x - __uint_as_float(hb << 16));
}

constexpr int BK16 = 16;   // complex k per stage (one MFMA k-step)
constexpr int ROWH = 24;   // bf16 per LDS row (16 used, 8 of padding)

template <int FORM>
struct Planes {
  static constexpr int N = FORM == kForm3M ? 6 : 4;  // rh rl ih il [sh sl]
};

__device__ __forceinline__ v8bf ld8(const uint16_t *p) { return *(const v8bf *)p; }

__device__ __forceinline__ v8bf neg8(v8bf v) {
  v4u u = *(v4u *)&v;
  u ^= 0x80008000u;
  return *(v8bf *)&u;
}

template <int FORM>
__global__ __launch_bounds__(256) void k_cgemm_bf16x3(GemmArgs g) {
  constexpr int BM = 128, BN = 128, NP = Planes<FORM>::N;
  constexpr int NACC = FORM == kForm3M ? 3 : 2;
  __shared__ __align__(16) uint16_t As[NP][BM * ROWH];
  __shared__ __align__(16) uint16_t Bs[NP][BN * ROWH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int q = blockIdx.y;
  const float2 *A = g.A + q * g.abs;
  const float2 *B = g.B + q * g.bbs;
  float2 *C = g.C + q * g.cbs;
  const Slot *sa = g.sa + q * g.sabs;
  const Slot *sb = g.sb + q * g.sbbs;
  Slot *sc = g.sc + q * g.scbs;
  const int64_t tile = blockIdx.x;
  const int64_t m0 = (tile / g.tiles_n) * BM, n0 = (tile % g.tiles_n) * BN;
  const int ea = slot_exp_b(sa->maxbits), eb = slot_exp_b(sb->maxbits);
  const float fa = ldexpf(1.0f, -ea), fb = ldexpf(1.0f, -eb);
  if (tile == 0 && tid == 0) sc->log2s = sa->log2s + sb->log2s + (double)(ea + eb);

  v16f_b acc[2][2][NACC];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < NACC; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][b][c][v] = 0.0f;

  // staging: each thread handles 8 complex values of A and 8 of B per stage
  // as (row, 8 consecutive k) when the operand is k-contiguous, otherwise
  // element by element
  const int srow = tid >> 1, sk = (tid & 1) * 8;
  for (int64_t k0 = 0; k0 < g.K; k0 += BK16) {
    // ---- A tile
    {
      float2 v[8];
      const int64_t gm = m0 + srow;
      if (g.opA == 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t gk = k0 + sk + e;
          v[e] = (gm < g.M && gk < g.K) ? A[gm * g.lda + gk] : make_float2(0.f, 0.f);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t gk = k0 + sk + e;
          v[e] = (gm < g.M && gk < g.K) ? A[gk * g.lda + gm] : make_float2(0.f, 0.f);
        }
      }
      uint16_t p[NP][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float re = v[e].x * fa, im = v[e].y * fa;
        split(re, p[0][e], p[1][e]);
        split(im, p[2][e], p[3][e]);
        if (FORM == kForm3M) split(re + im, p[NP - 2][e], p[NP - 1][e]);
      }
#pragma unroll
      for (int pl = 0; pl < NP; ++pl) {
        v4u w;
        w.x = p[pl][0] | ((uint32_t)p[pl][1] << 16);
        w.y = p[pl][2] | ((uint32_t)p[pl][3] << 16);
        w.z = p[pl][4] | ((uint32_t)p[pl][5] << 16);
        w.w = p[pl][6] | ((uint32_t)p[pl][7] << 16);
        *(v4u *)&As[pl][srow * ROWH + sk] = w;
      }
    }
    // ---- B tile, stored [n][k]
    {
      float2 v[8];
      const int64_t gn = n0 + srow;
      if (g.opB == 1) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t gk = k0 + sk + e;
          v[e] = (gn < g.N && gk < g.K) ? B[gn * g.ldb + gk] : make_float2(0.f, 0.f);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t gk = k0 + sk + e;
          v[e] = (gn < g.N && gk < g.K) ? B[gk * g.ldb + gn] : make_float2(0.f, 0.f);
        }
      }
      uint16_t p[NP][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float re = v[e].x * fb, im = v[e].y * fb;
        split(re, p[0][e], p[1][e]);
        split(im, p[2][e], p[3][e]);
        if (FORM == kForm3M) split(re + im, p[NP - 2][e], p[NP - 1][e]);
      }
#pragma unroll
      for (int pl = 0; pl < NP; ++pl) {
        v4u w;
        w.x = p[pl][0] | ((uint32_t)p[pl][1] << 16);
        w.y = p[pl][2] | ((uint32_t)p[pl][3] << 16);
        w.z = p[pl][4] | ((uint32_t)p[pl][5] << 16);
        w.w = p[pl][6] | ((uint32_t)p[pl][7] << 16);
        *(v4u *)&Bs[pl][srow * ROWH + sk] = w;
      }
    }
    __syncthreads();
    // ---- MFMA: lane reads row l%32, k = 8*(l/32) .. +7 of each plane
    const int fr = lane & 31, fk = (lane >> 5) * 8;
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
          C[gm * g.ldc + gn] = make_float2(re, im);
          mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
      }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) atomicMax(&sc->maxbits, __float_as_uint(mx));
}

hipError_t launch_gemm_bf16x3(hipStream_t st, const GemmArgs &g0, int form, int nbatch) {
  GemmArgs g = g0;
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
