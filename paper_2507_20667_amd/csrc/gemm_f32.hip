// FP32 complex GEMM on v_mfma_f32_32x32x2_f32 from k-tiled float planes.
//
// The permutation that puts a vertex's operands in GEMM order writes them as
// two float planes (re, im), divided by 2^e of the operand's scale record and
// k-tiled: row r, k sits at ((k / 16) * rows + r) * 16 + k % 16, so that one
// 16-deep stage of a 128-row tile is a contiguous 8 KB block of each plane.
// Stages stream straight from global memory into a ring of LDS slots
// (global_load_lds_dwordx4, no staging registers): two slots, one stage
// ahead, when two blocks share a CU (see TWO below), else four slots, three
// stages ahead.  The wait for a stage is a vmcnt on the wave's own loads
// followed by a barrier.  Past the last stage the requests repeat the last
// stage into the free slot, so the number of loads in flight, and the wait,
// never change.  The slots are distinct arrays named statically (the loop is
// unrolled by the slot count), which lets the compiler see that a read of one
// slot does not wait on loads into another.
//
// Block = 4 waves in a 2 x 2 grid over a 128 x 128 output tile, each wave
// 64 x 64 outputs as 2 x 2 MFMA tiles.  For that instruction lane l supplies
// A[l%32][kk] and B[kk][l%32] with kk = l/32 of a 2-deep step and holds
// C[8(v/4) + 4(l/32) + v%4][l%32] in accumulator v.  Within a stage, step s
// gives lane half h the k value 8h + s (A and B alike, so the sum over k is
// unchanged): a lane's eight k of a row are two 16-byte LDS reads.  Rows are
// 64 bytes; row r's chunk c sits at position c ^ swz(r), so the rows one LDS
// access touches fall on distinct banks.  A stage is 128 MFMAs per wave (4M).
// FORM = 4M: Re = ArBr - AiBi, Im = ArBi + AiBr (four products per complex
// one).  FORM = 3M (Gauss): T1 = ArBr, T2 = AiBi, T3 = (Ar + Ai)(Br + Bi),
// Re = T1 - T2, Im = T3 - T1 - T2; the sums are formed in registers from the
// fragments (one add per value), so the planes and the LDS traffic are the
// same as 4M's and the MFMA work is three quarters of it.
#include <type_traits>

#include "tn_device.h"

namespace tn {

typedef float v16f_c __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void_f;

constexpr int FBK = 16;               // k per stage

// s_waitcnt immediate: vmcnt(v) expcnt(7) lgkmcnt(0)
__host__ __device__ constexpr int f_wait_imm(int v) { return (v & 15) | ((v >> 4) << 14) | (7 << 4); }

// (b3 ^ b1, b2) of the row index: rows r..r+15 cover every (r % 4, chunk)
// pair and rows r..r+7 every (r % 2, chunk) pair once
__device__ __forceinline__ int fswz(int r) {
  return ((((r >> 3) ^ (r >> 1)) & 1) << 1) | ((r >> 2) & 1);
}

// WMW = waves along M (the four waves form a WMW x 4/WMW grid, 64 x 64
// outputs each): 2 gives a 128 x 128 tile, 1 a 64 x 256 tile (for M <= 64),
// 4 a 256 x 64 tile (for N <= 64).
//
// TWO: two blocks share a CU.  The ring then has two slots (64 KB of LDS for
// the 128 x 128 tile) and a wave reads a stage's fragments in two halves of
// eight k (32 fragment registers), so that a block fits in 256 registers;
// one block's barrier and fragment reads overlap the other's products
// (1.04-1.14 x on the 30-qubit shapes against one block with four slots).
// The 3M form of the 64 x 256 and 256 x 64 tiles would not fit and keeps one
// block per CU with the four-slot ring.
template <int FORM, int WMW>
__device__ __forceinline__ constexpr bool planes_two() { return FORM == kForm4M || WMW == 2; }

template <int FORM, int WMW>
__global__ __launch_bounds__(256, (FORM == kForm4M || WMW == 2) ? 2 : 1) void k_cgemm_f32_planes(GemmArgs g) {
  constexpr bool TWO = planes_two<FORM, WMW>();
  constexpr int NSLOT = TWO ? 2 : 4;
  constexpr int NACC = FORM == kForm3M ? 3 : 2;
  constexpr int WNW = 4 / WMW;
  constexpr int BM = 64 * WMW, BN = 64 * WNW;          // tile rows of A and of B
  constexpr int APL = BM * FBK, BPL = BN * FBK;        // floats per plane tile
  constexpr int FSTAGE = 2 * (APL + BPL);              // A re, A im, B re, B im
  constexpr int JA = BM / 64, JB = BN / 64;            // load instructions per wave and plane
  __shared__ __align__(16) float ring0[FSTAGE], ring1[FSTAGE], ring2[TWO ? 4 : FSTAGE], ring3[TWO ? 4 : FSTAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WNW, wn = wave % WNW;
  const int q = blockIdx.y;
  const float *A = (const float *)g.A + q * g.abs;
  const float *B = (const float *)g.B + q * g.bbs;
  const Slot *sa = g.sa + q * g.sabs;
  const Slot *sb = g.sb + q * g.sbbs;
  Slot *sc = g.sc + q * g.scbs;
  int ks;
  int64_t t;
  gemm_block_tile(g, ks, t);  // XCD-aware block -> (k chunk, tile)
  const int64_t m0 = (t % g.tiles_m) * BM, n0 = (t / g.tiles_m) * BN;
  const int64_t kbeg = (int64_t)ks * g.kchunk;
  const int64_t kend = g.K < kbeg + g.kchunk ? g.K : kbeg + g.kchunk;
  const int ea = tn_scale_exp(sa->maxbits), eb = tn_scale_exp(sb->maxbits);
  if (blockIdx.x == 0 && tid == 0) sc->log2s = sa->log2s + sb->log2s + (double)(ea + eb);

  v16f_c acc[2][2][NACC];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < NACC; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][b][c][v] = 0.0f;

  // this lane's loads: instruction j covers rows (R / 4) * wave + 16 * j +
  // lane / 4 of an R-row plane tile; position lane % 4 of the row holds
  // logical chunk (lane % 4) ^ fswz(row) (rows past M or N clamped to the
  // last one)
  const uint8_t *abase = (const uint8_t *)(A + m0 * FBK);
  const uint8_t *bbase = (const uint8_t *)(B + n0 * FBK);
  uint32_t aoff[JA], boff[JB];
#pragma unroll
  for (int j = 0; j < JA; ++j) {
    const int r = (BM / 4) * wave + 16 * j + (lane >> 2);
    const int c = (lane & 3) ^ fswz(r);
    const int64_t ra_ = m0 + r < g.M ? r : g.M - 1 - m0;
    aoff[j] = (uint32_t)((ra_ * FBK + c * 4) * 4);
  }
#pragma unroll
  for (int j = 0; j < JB; ++j) {
    const int r = (BN / 4) * wave + 16 * j + (lane >> 2);
    const int c = (lane & 3) ^ fswz(r);
    const int64_t rb_ = n0 + r < g.N ? r : g.N - 1 - n0;
    boff[j] = (uint32_t)((rb_ * FBK + c * 4) * 4);
  }
  const int64_t nk = (kend - kbeg) / FBK;
#define TN_FRING(S) ((S) == 0 ? ring0 : (S) == 1 ? ring1 : (S) == 2 ? ring2 : ring3)
  auto issue = [&](auto slot, int64_t stg) {
    constexpr int S = decltype(slot)::value;
    float *rb = TN_FRING(S);
    const int64_t kb = kbeg / FBK + (stg < nk ? stg : nk - 1);
    const uint8_t *ak = abase + kb * g.M * FBK * 4, *bk = bbase + kb * g.N * FBK * 4;
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
#pragma unroll
      for (int j = 0; j < JA; ++j)
        __builtin_amdgcn_global_load_lds((const void *)(ak + pl * g.pa * 4 + aoff[j]),
                                         (lds_void_f *)(rb + pl * APL + ((BM / 4) * wave + 16 * j) * FBK),
                                         16, 0, 0);
#pragma unroll
      for (int j = 0; j < JB; ++j)
        __builtin_amdgcn_global_load_lds(
            (const void *)(bk + pl * g.pb * 4 + boff[j]),
            (lds_void_f *)(rb + 2 * APL + pl * BPL + ((BN / 4) * wave + 16 * j) * FBK), 16, 0, 0);
    }
  };
  // fragments: lane half h reads k 8h .. 8h+7 of its row (logical chunks 2h
  // and 2h + 1) from each plane
  const int fr = lane & 31, fh = lane >> 5;
  const int fp0 = ((2 * fh) ^ fswz(fr)) * 4, fp1 = ((2 * fh + 1) ^ fswz(fr)) * 4;
  auto fread = [&](auto slot, int h, v4f (&a)[2][2], v4f (&b)[2][2]) {
    constexpr int S = decltype(slot)::value;
    const float *rb = TN_FRING(S);
    const int fp = h ? fp1 : fp0;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int pl = 0; pl < 2; ++pl)
        a[mb][pl] = *(const v4f *)(rb + pl * APL + (wm * 64 + mb * 32 + fr) * FBK + fp);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int pl = 0; pl < 2; ++pl)
        b[nb][pl] = *(const v4f *)(rb + 2 * APL + pl * BPL + (wn * 64 + nb * 32 + fr) * FBK + fp);
  };
#undef TN_FRING
  // the four k of one fragment half (k 8h + 4c + s of lane half c), in order
  auto mma = [&](const v4f (&a)[2][2], const v4f (&b)[2][2]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      float ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        ar[x] = a[x][0][s];
        ai[x] = a[x][1][s];
        br[x] = b[x][0][s];
        bi[x] = b[x][1][s];
      }
      if (FORM == kForm4M) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[mb], br[nb], acc[mb][nb][0], 0, 0, 0);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[mb], bi[nb], acc[mb][nb][1], 0, 0, 0);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai[mb], bi[nb], acc[mb][nb][0], 0, 0, 0);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[mb], br[nb], acc[mb][nb][1], 0, 0, 0);
      } else {
        float as[2], bs[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          as[x] = ar[x] + ai[x];
          bs[x] = br[x] + bi[x];
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[mb], br[nb], acc[mb][nb][0], 0, 0, 0);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[mb], bi[nb], acc[mb][nb][1], 0, 0, 0);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb][2] = __builtin_amdgcn_mfma_f32_32x32x2f32(as[mb], bs[nb], acc[mb][nb][NACC - 1], 0, 0, 0);
      }
    }
  };
  // one stage: wait for it (the loads of the NSLOT - 2 stages after it may
  // stay in flight), barrier, request stage kt + NSLOT - 1 into the slot
  // stage kt - 1 used, then the stage's products.  TWO: the two halves of the
  // stage's k one after the other (read, multiply); otherwise both halves'
  // fragments first (one set of 64 registers), then the products.
  v4f fa[2][2], fb[2][2], ga[2][2], gb[2][2];
  auto stage = [&](auto slot, int64_t kt) {
    constexpr int S = decltype(slot)::value;
    __builtin_amdgcn_s_waitcnt(f_wait_imm((NSLOT - 2) * 2 * (JA + JB)));
    __builtin_amdgcn_s_barrier();
    issue(std::integral_constant<int, (S + NSLOT - 1) % NSLOT>(), kt + NSLOT - 1);
    if constexpr (TWO) {
      fread(slot, 0, fa, fb);
      mma(fa, fb);
      fread(slot, 1, fa, fb);
      mma(fa, fb);
    } else {
      fread(slot, 0, fa, fb);
      fread(slot, 1, ga, gb);
      mma(fa, fb);
      mma(ga, gb);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  const std::integral_constant<int, 0> s0;
  const std::integral_constant<int, 1> s1;
  const std::integral_constant<int, 2> s2;
  const std::integral_constant<int, 3> s3;
  __builtin_amdgcn_s_waitcnt(0);  // nothing else in flight when the ring starts
  issue(s0, 0);
  if constexpr (NSLOT == 4) {
    issue(s1, 1);
    issue(s2, 2);
  }
  int64_t kt = 0;
  for (; kt + NSLOT <= nk; kt += NSLOT) {
    stage(s0, kt);
    stage(s1, kt + 1);
    if constexpr (NSLOT == 4) {
      stage(s2, kt + 2);
      stage(s3, kt + 3);
    }
  }
  if (kt < nk) stage(s0, kt);
  if (NSLOT == 4 && kt + 1 < nk) stage(s1, kt + 1);
  if (NSLOT == 4 && kt + 2 < nk) stage(s2, kt + 2);
  __builtin_amdgcn_s_waitcnt(0);  // no load may still write LDS when the block ends

  const bool partial = g.ksplit > 1;
  float2 *C = partial ? g.part + q * g.partbs + (int64_t)ks * g.M * g.N : g.C + q * g.cbs;
  const int64_t ldc = partial ? g.N : g.ldc;
  // an operand read as it is (raw) scales the result instead: exact
  const float post = (g.raw_a | g.raw_b) ? ldexpf(1.0f, -(g.raw_a ? ea : 0) - (g.raw_b ? eb : 0)) : 1.0f;
  // or the result as its parent's operand planes
  const bool fo = g.fo_on != 0;
  uint8_t *P = (uint8_t *)(g.C + q * g.cbs), *P1 = P + g.fo_plane * 4;
  PlaneOut<4> po;
  if (fo) po.init(g, m0 + wm * 64 + (lane >> 5) * 4, n0 + wn * 64 + (lane & 31));
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
        re *= post;
        im *= post;
        if (cm < g.M && cn < g.N) {
          if (fo) {
            const uint32_t d = po.at(mb, nb, v);
            *(float *)(P + d) = re;
            *(float *)(P1 + d) = im;
          } else {
            C[cm * ldc + cn] = make_float2(re, im);
          }
          mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
      }
  if (!partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) atomicMax(&sc->maxbits, __float_as_uint(mx));
  }
}

// Tile shape of variant v: 0 = 128 x 128, 1 = 64 x 256, 2 = 256 x 64.
int gemm_planes_tile_m(int v) { return v == 1 ? 64 : v == 2 ? 256 : 128; }
int gemm_planes_tile_n(int v) { return v == 1 ? 256 : v == 2 ? 64 : 128; }

hipError_t launch_gemm_f32_planes(hipStream_t st, const GemmArgs &g0, int form, int nbatch) {
  GemmArgs g = g0;
  if (g.opA != 0 || g.opB != 1 || g.planes != 2 || !g.ktile || g.K % FBK != 0 ||
      (form != kForm4M && form != kForm3M) || g.tile < 0 || g.tile > 2 || (g.fo_on && g.ksplit > 1))
    return hipErrorInvalidValue;
  const int tm = gemm_planes_tile_m(g.tile), tn = gemm_planes_tile_n(g.tile);
  g.tiles_m = (int)((g.M + tm - 1) / tm);
  g.tiles_n = (int)((g.N + tn - 1) / tn);
  if (g.ksplit < 1) g.ksplit = 1;
  if (g.ksplit == 1) g.kchunk = g.K;
  if (g.kchunk < 1 || g.kchunk % FBK != 0 || (int64_t)g.ksplit * g.kchunk < g.K ||
      (g.ksplit > 1 && !g.part))
    return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)g.tiles_m * g.tiles_n * g.ksplit;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks, nbatch);
#define TN_F32P(F, W) hipLaunchKernelGGL((k_cgemm_f32_planes<F, W>), grid, dim3(256), 0, st, g)
  if (form == kForm4M) {
    if (g.tile == 0) TN_F32P(kForm4M, 2);
    else if (g.tile == 1) TN_F32P(kForm4M, 1);
    else TN_F32P(kForm4M, 4);
  } else {
    if (g.tile == 0) TN_F32P(kForm3M, 2);
    else if (g.tile == 1) TN_F32P(kForm3M, 1);
    else TN_F32P(kForm3M, 4);
  }
#undef TN_F32P
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.ksplit == 1) return e;
  return launch_splitk_reduce(st, g, nbatch);
}

}  // namespace tn
