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
// its four 16-byte chunks stored in the order chunk ^ swz(row), chosen so that
// the rows read together by one 16-byte-per-lane LDS access (8 rows on 32
// banks, 16 rows on 64 banks) fall on distinct banks.  Global loads
// of the next stage are issued before the current stage's products; the 4M
// form double-buffers LDS (one barrier a stage), the 3M form, with six planes,
// has room for one buffer.  Consecutive products go to different accumulators
// so that no MFMA waits on the previous one.
#include <type_traits>

#include "tn_device.h"

namespace tn {

typedef float v16f_b __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

constexpr int BT = 128;     // tile rows (M) and columns (N)
constexpr int BKS = 32;     // k per stage
constexpr int ROWE = BKS;   // bf16 per LDS row (no padding: swizzled chunks)

__device__ __forceinline__ v8bf as_bf(v4u u) { return *(v8bf *)&u; }

// Chunk swizzle of LDS row r (rows are 64 bytes, 4 chunks): (b3 ^ b1, b2) of
// r's bits.  Rows r..r+15 then cover every (r % 4, chunk slot) pair once, and
// rows r..r+7 every (r % 2, chunk slot) pair once.
__device__ __forceinline__ int swz(int r) {
  return ((((r >> 3) ^ (r >> 1)) & 1) << 1) | ((r >> 2) & 1);
}

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
// 3M products grouped by plane pair (re, im, sum), for the direct-to-LDS
// kernel, which reads one group's fragments while the previous group's
// products run
__device__ constexpr int prod_3m_g(int i, int f) {
  constexpr int t[9][4] = {{0, 0, 0, 0}, {0, 0, 1, 0}, {0, 1, 0, 0}, {1, 2, 2, 0}, {1, 2, 3, 0},
                           {1, 3, 2, 0}, {2, 4, 4, 0}, {2, 4, 5, 0}, {2, 5, 4, 0}};
  return t[i][f];
}
__device__ constexpr int prod_3m(int i, int f) {
  constexpr int t[9][4] = {{0, 0, 0, 0}, {1, 2, 2, 0}, {2, 4, 4, 0}, {0, 0, 1, 0}, {1, 2, 3, 0},
                           {2, 4, 5, 0}, {0, 1, 0, 0}, {1, 3, 2, 0}, {2, 5, 4, 0}};
  return t[i][f];
}

// EXACT: every k chunk is a whole number of stages (K % 32 == 0), so the main
// loop has no bounds checks and forms one basic block the scheduler can
// interleave.  Rows past M or N are clamped to the last row: they only feed
// outputs that the epilogue discards.
template <int FORM, bool EXACT>
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
  int ks;
  int64_t t;
  gemm_block_tile(g, ks, t);  // XCD-aware block -> (k chunk, tile)
  const int64_t m0 = (t % g.tiles_m) * BT, n0 = (t / g.tiles_m) * BT;
  const int64_t kbeg = (int64_t)ks * g.kchunk;
  const int64_t kend = g.K < kbeg + g.kchunk ? g.K : kbeg + g.kchunk;
  const int ea = tn_scale_exp(sa->maxbits), eb = tn_scale_exp(sb->maxbits);
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
  // loads address a block-uniform base (scalar registers) plus a 32-bit byte
  // offset per thread and row (rows past M or N clamped to the last one)
  const uint8_t *abase = (const uint8_t *)(A + m0 * g.lda);
  const uint8_t *bbase = (const uint8_t *)(B + n0 * g.ldb);
  uint32_t aoff[2], boff[2];
  int spos[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int r = srow + 64 * i;
    const int64_t ra_ = m0 + r < g.M ? r : g.M - 1 - m0;
    const int64_t rb_ = n0 + r < g.N ? r : g.N - 1 - n0;
    aoff[i] = (uint32_t)((ra_ * g.lda + sch * 8) * 2);
    boff[i] = (uint32_t)((rb_ * g.ldb + sch * 8) * 2);
    spos[i] = r * ROWE + ((sch ^ swz(r)) * 8);
  }
  // register staging: two sets, so that a stage's loads can be issued two
  // stages before they are stored to LDS
  v4u ra[2][NP][2], rb[2][NP][2];
  auto gload = [&](int set, int64_t k0) {
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) {
      const uint8_t *pa_ = abase + (pl * g.pa + k0) * 2;
      const uint8_t *pb_ = bbase + (pl * g.pb + k0) * 2;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (EXACT) {
          ra[set][pl][i] = *(const v4u *)(pa_ + aoff[i]);
          rb[set][pl][i] = *(const v4u *)(pb_ + boff[i]);
        } else {
          const int64_t kk = k0 + sch * 8;
          ra[set][pl][i] = load8((const uint16_t *)(pa_ + aoff[i]) - kk, kk, kend, vec_ok);
          rb[set][pl][i] = load8((const uint16_t *)(pb_ + boff[i]) - kk, kk, kend, vec_ok);
        }
      }
    }
  };
  auto lstore = [&](int set, int buf) {
    uint16_t *la = lds + buf * 2 * OPER, *lb = la + OPER;
#pragma unroll
    for (int pl = 0; pl < NP; ++pl)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        *(v4u *)&la[pl * PLANE + spos[i]] = ra[set][pl][i];
        *(v4u *)&lb[pl * PLANE + spos[i]] = rb[set][pl][i];
      }
  };
  // fragment rows: (wm|wn)*64 + mb*32 + lane%32; the swizzle term depends on
  // lane%32 alone since the rest is a multiple of 16
  const int fr = lane & 31, fsw = swz(fr), fhalf = lane >> 5;

  auto frag_read = [&](int buf, int ss, v4u (&a)[2][NP], v4u (&b)[2][NP]) {
    const uint16_t *la = lds + buf * 2 * OPER, *lb = la + OPER;
    const int cpos = ((2 * ss + fhalf) ^ fsw) * 8;
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
  };
  // products p0 .. p1-1 of the table on one 16-deep k step
  auto mma = [&](const v4u (&a)[2][NP], const v4u (&b)[2][NP], int p0, int p1) {
#pragma unroll
    for (int pi = 0; pi < NPROD; ++pi) {
      if (pi < p0 || pi >= p1) continue;
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
  };

  const int64_t nk = (kend - kbeg + BKS - 1) / BKS;
  // (fence between the two 16-deep steps: one fragment set live at a time)
  auto compute = [&](int buf) {
#pragma unroll
    for (int ss = 0; ss < 2; ++ss) {
      v4u a[2][NP], b[2][NP];
      frag_read(buf, ss, a, b);
      mma(a, b, 0, NPROD);
      if (EXACT && NBUF == 2 && ss == 0) __builtin_amdgcn_sched_barrier(0);
    }
  };
  if (EXACT && NBUF == 2) {
    // Stage kt sits in LDS buffer kt % 2 while it is multiplied; stage kt + 1
    // is in register set (kt + 1) % 2 (loaded or in flight) and goes to the
    // other buffer at the end; stage kt + 2 is requested into set kt % 2 at
    // the start.  Scheduling fences keep the requests at the top: left free,
    // the compiler sinks them next to the stores that wait on them.
    auto body = [&](auto sc, int64_t kt, bool load, bool store) {
      constexpr int S = decltype(sc)::value;
      if (load) gload(S, kbeg + (kt + 2) * BKS);
      __builtin_amdgcn_sched_barrier(0);
      compute(S);
      __builtin_amdgcn_sched_barrier(0);
      if (store) lstore(S ^ 1, S ^ 1);
      __syncthreads();
    };
    const std::integral_constant<int, 0> s0;
    const std::integral_constant<int, 1> s1;
    gload(0, kbeg);
    lstore(0, 0);
    if (nk > 1) gload(1, kbeg + BKS);
    __syncthreads();
    int64_t kt = 0;
    for (; kt + 3 < nk; kt += 2) {
      body(s0, kt, true, true);
      body(s1, kt + 1, true, true);
    }
    for (; kt < nk; ++kt) {
      if (kt & 1)
        body(s1, kt, kt + 2 < nk, kt + 1 < nk);
      else
        body(s0, kt, kt + 2 < nk, kt + 1 < nk);
    }
  } else {
    gload(0, kbeg);
    lstore(0, 0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
      const int cur = NBUF == 2 ? (int)(kt & 1) : 0;
      const bool more = kt + 1 < nk;
      if (more) gload(0, kbeg + (kt + 1) * BKS);
      compute(cur);
      if (more) {
        if (NBUF == 1) __syncthreads();
        lstore(0, NBUF == 2 ? (int)((kt + 1) & 1) : 0);
        __syncthreads();
      }
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

// ------------------------------------------------------- direct-to-LDS form
// For k a multiple of 16 the permutation writes the planes k-tiled (16
// consecutive k of consecutive rows contiguous), so one stage of a tile is a
// contiguous 4 KB block of each plane, streamed straight from global memory
// into LDS (global_load_lds_dwordx4: each lane's 16 bytes land at the wave's
// LDS segment base + 16 * lane), with no staging registers and no LDS
// stores.  The stages form a ring of NSLOT slots, filled NSLOT - 1 stages
// ahead.  A bf16 stage is 48 MFMAs of 32 cycles per wave (4M), a sixth of an
// FP32 stage's matrix work for the same fragment reads, so the barrier and
// the fragment reads of a stage are not hidden behind its products when one
// block holds the CU.  4M (four planes, 32 KB a stage) therefore keeps two
// slots and one fragment set (64 KB of LDS, at most 256 registers), so that
// two blocks share a CU and one block's barrier and fragment reads overlap
// the other's products (measured 1.12-1.21 x on the 30-qubit shapes against
// one block with four slots and two fragment sets).  3M (six planes, 48 KB a
// stage) keeps three slots, one block per CU.  A wave waits for its own loads
// of a stage (vmcnt, the later stages' loads may stay in flight) and the
// barrier that follows publishes everyone's.  Past the last stage the
// requests repeat the last stage into the free slot, so the count of loads in
// flight, and the wait, are the same in every iteration.  The slots are
// distinct arrays named statically (the loop is unrolled by NSLOT), which
// lets the compiler see that a read of one slot does not depend on loads
// into another.
//
// LDS layout of a slot: [A planes][B planes], each 128 rows x 32 bytes; row
// r's 16-byte chunk c sits at position c ^ dswz(r), so the 16 rows read
// together fall on distinct banks.
constexpr int DBK = 16;               // k per stage
constexpr int DPLANE = BT * DBK;      // bf16 per plane tile (4 KB)
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ int dswz(int r) { return ((r >> 2) ^ (r >> 3)) & 1; }

// One result entry as its parent's k-tiled bf16 operand planes (re hi, re
// lo, im hi, im lo at P[0..3] + d bytes, and for a 3M parent (re+im) hi and
// lo at P[4], P[5]; the split of the operand permutation).
template <int NPL>
__device__ __forceinline__ void store_planes(uint8_t *const (&P)[6], uint32_t d, float re, float im) {
  uint32_t h, l;
  tn_split_bf16x2(re, im, h, l);
  *(uint16_t *)(P[0] + d) = (uint16_t)h;
  *(uint16_t *)(P[1] + d) = (uint16_t)l;
  *(uint16_t *)(P[2] + d) = (uint16_t)(h >> 16);
  *(uint16_t *)(P[3] + d) = (uint16_t)(l >> 16);
  if (NPL == 6) {
    uint16_t sh, sl;
    tn_split_bf16(re + im, sh, sl);
    *(uint16_t *)(P[4] + d) = sh;
    *(uint16_t *)(P[5] + d) = sl;
  }
}

// s_waitcnt immediate: vmcnt(v) expcnt(7) lgkmcnt(0)
__host__ __device__ constexpr int dma_wait_imm(int v) { return (v & 15) | ((v >> 4) << 14) | (7 << 4); }

template <int FORM>
__global__ __launch_bounds__(256, FORM == kForm3M ? 1 : 2) void k_cgemm_bf16x3_dma(GemmArgs g) {
  constexpr int NP = FORM == kForm3M ? 6 : 4;        // planes per operand
  constexpr int NSLOT = FORM == kForm3M ? 3 : 2;     // ring slots
  constexpr int NACC = FORM == kForm3M ? 3 : 2;
  constexpr int NPROD = FORM == kForm3M ? 9 : 12;
  constexpr int STAGE = 2 * NP * DPLANE;
  // loads of a wave per stage: one 1 KB instruction per plane of A and of B
  constexpr int LOADS = 2 * NP;
  __shared__ __align__(16) uint16_t ring0[STAGE], ring1[STAGE], ring2[NSLOT == 3 ? STAGE : 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int q = blockIdx.y;
  const uint16_t *A = (const uint16_t *)g.A + q * g.abs;
  const uint16_t *B = (const uint16_t *)g.B + q * g.bbs;
  const Slot *sa = g.sa + q * g.sabs;
  const Slot *sb = g.sb + q * g.sbbs;
  Slot *sc = g.sc + q * g.scbs;
  int ks;
  int64_t t;
  gemm_block_tile(g, ks, t);  // XCD-aware block -> (k chunk, tile)
  const int64_t m0 = (t % g.tiles_m) * BT, n0 = (t / g.tiles_m) * BT;
  const int64_t kbeg = (int64_t)ks * g.kchunk;
  const int64_t kend = g.K < kbeg + g.kchunk ? g.K : kbeg + g.kchunk;
  const int ea = tn_scale_exp(sa->maxbits), eb = tn_scale_exp(sb->maxbits);
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

  // this lane's load: row 32 * wave + lane / 2 of every plane tile, logical
  // chunk (lane % 2) ^ dswz(row) (rows past M or N clamped to the last one);
  // in the k-tiled planes row r of k block kb starts at (kb * rows + r) * 16
  const uint8_t *abase = (const uint8_t *)(A + m0 * DBK);
  const uint8_t *bbase = (const uint8_t *)(B + n0 * DBK);
  uint32_t aoff, boff;
  {
    const int r = 32 * wave + (lane >> 1);
    const int c = (lane & 1) ^ dswz(r);
    const int64_t ra_ = m0 + r < g.M ? r : g.M - 1 - m0;
    const int64_t rb_ = n0 + r < g.N ? r : g.N - 1 - n0;
    aoff = (uint32_t)((ra_ * DBK + c * 8) * 2);
    boff = (uint32_t)((rb_ * DBK + c * 8) * 2);
  }
  const int64_t nk = (kend - kbeg) / DBK;
#define TN_RING(S) ((S) == 0 ? ring0 : (S) == 1 ? ring1 : ring2)
  auto issue = [&](auto slot, int64_t stg) {
    constexpr int S = decltype(slot)::value;
    uint16_t *rb = TN_RING(S) + wave * (DPLANE / 4);
    const int64_t kb = kbeg / DBK + (stg < nk ? stg : nk - 1);
    const uint8_t *ak = abase + kb * g.M * DBK * 2, *bk = bbase + kb * g.N * DBK * 2;
#pragma unroll
    for (int pl = 0; pl < NP; ++pl) {
      __builtin_amdgcn_global_load_lds((const void *)(ak + pl * g.pa * 2 + aoff),
                                       (lds_void *)(rb + pl * DPLANE), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void *)(bk + pl * g.pb * 2 + boff),
                                       (lds_void *)(rb + (NP + pl) * DPLANE), 16, 0, 0);
    }
  };
  const int fr = lane & 31, fpos = ((lane >> 5) ^ dswz(fr)) * 8;
  // fragments in plane-pair order (A and B of pair 0, then pair 1, ...), so
  // that the products of one pair can start while the next pair is read
  auto fread = [&](auto slot, v4u (&a)[2][NP], v4u (&b)[2][NP]) {
    constexpr int S = decltype(slot)::value;
    const uint16_t *rb = TN_RING(S);
#pragma unroll
    for (int pp = 0; pp < NP; pp += 2) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int pl = pp; pl < pp + 2; ++pl)
          a[mb][pl] = *(const v4u *)(rb + pl * DPLANE + (wm * 64 + mb * 32 + fr) * DBK + fpos);
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int pl = pp; pl < pp + 2; ++pl)
          b[nb][pl] = *(const v4u *)(rb + (NP + pl) * DPLANE + (wn * 64 + nb * 32 + fr) * DBK + fpos);
    }
  };
#undef TN_RING
  auto mma = [&](const v4u (&a)[2][NP], const v4u (&b)[2][NP]) {
#pragma unroll
    for (int pi = 0; pi < NPROD; ++pi) {
      const int c = FORM == kForm3M ? prod_3m_g(pi, 0) : prod_4m(pi, 0);
      const int ap = FORM == kForm3M ? prod_3m_g(pi, 1) : prod_4m(pi, 1);
      const int bp = FORM == kForm3M ? prod_3m_g(pi, 2) : prod_4m(pi, 2);
      const int ng = FORM == kForm3M ? prod_3m_g(pi, 3) : prod_4m(pi, 3);
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const v8bf av = as_bf(ng ? neg4(a[mb][ap]) : a[mb][ap]);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          acc[mb][nb][c] =
              __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, as_bf(b[nb][bp]), acc[mb][nb][c], 0, 0, 0);
      }
    }
  };
  v4u fa[2][NP], fb[2][NP];
  // one stage (ring slot S): wait for it (the loads of the NSLOT - 2 stages
  // after it may stay in flight), barrier (every wave has read the fragments
  // of stage kt - 1), request stage kt + NSLOT - 1 into the slot stage kt - 1
  // used, read stage kt's fragments pair by pair and run its products
  auto run_stage = [&](auto slot, int64_t kt) {
    constexpr int S = decltype(slot)::value;
    __builtin_amdgcn_s_waitcnt(dma_wait_imm((NSLOT - 2) * LOADS));
    __builtin_amdgcn_s_barrier();
    issue(std::integral_constant<int, (S + NSLOT - 1) % NSLOT>(), kt + NSLOT - 1);
    fread(slot, fa, fb);
    mma(fa, fb);
    __builtin_amdgcn_sched_barrier(0);
  };
  __builtin_amdgcn_s_waitcnt(0);  // nothing else in flight when the ring starts
  issue(std::integral_constant<int, 0>(), 0);
  if constexpr (NSLOT == 3) issue(std::integral_constant<int, 1>(), 1);
  int64_t kt = 0;
  for (; kt + NSLOT <= nk; kt += NSLOT) {
    run_stage(std::integral_constant<int, 0>(), kt);
    run_stage(std::integral_constant<int, 1>(), kt + 1);
    if constexpr (NSLOT == 3) run_stage(std::integral_constant<int, 2>(), kt + 2);
  }
  if (kt < nk) run_stage(std::integral_constant<int, 0>(), kt);
  if (NSLOT == 3 && kt + 1 < nk) run_stage(std::integral_constant<int, 1>(), kt + 1);
  __builtin_amdgcn_s_waitcnt(0);  // no load may still write LDS when the block ends

  const bool partial = g.ksplit > 1;
  float2 *C = partial ? g.part + q * g.partbs + (int64_t)ks * g.M * g.N : g.C + q * g.cbs;
  const int64_t ldc = partial ? g.N : g.ldc;
  // an operand read as it is (raw) scales the result instead: exact; the
  // result may go out as its parent's operand planes (four, six for 3M)
  const float post = (g.raw_a | g.raw_b) ? ldexpf(1.0f, -(g.raw_a ? ea : 0) - (g.raw_b ? eb : 0)) : 1.0f;
  const bool fo = g.fo_on != 0;
  uint8_t *const P0 = (uint8_t *)(g.C + q * g.cbs);
  uint8_t *const P[6] = {P0, P0 + g.fo_plane * 2, P0 + g.fo_plane * 4, P0 + g.fo_plane * 6, P0 + g.fo_plane * 8,
                         P0 + g.fo_plane * 10};
  PlaneOut<2> po;
  if (fo) po.init(g, m0 + wm * 64 + (lane >> 5) * 4, n0 + wn * 64 + (lane & 31));
  float mx = 0.0f;
  auto value = [&](int mb, int nb, int v, float &re, float &im) {
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
  };
  if (fo && m0 + BT <= g.M && n0 + BT <= g.N) {
    // a whole tile of planes: no entry to test
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          float re, im;
          value(mb, nb, v, re, im);
          store_planes<NP>(P, po.at(mb, nb, v), re, im);
          mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
  } else {
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
          value(mb, nb, v, re, im);
          if (cm < g.M && cn < g.N) {
            if (fo)
              store_planes<NP>(P, po.at(mb, nb, v), re, im);
            else
              C[cm * ldc + cn] = make_float2(re, im);
            mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
          }
        }
  }
  if (!partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) atomicMax(&sc->maxbits, __float_as_uint(mx));
  }
}

// ------------------------------------------------ two wave groups (4M form)
// One block of eight waves owns a 256 x 128 output tile (WIDE_A: 256 rows of
// A) or 128 x 256 (256 rows of B), as two groups of four waves, each group a
// 128 x 128 half laid out like the four-wave kernel above.  Waves w and w + 4
// share a SIMD, and the two groups take turns: while one group's waves run
// the 48 products of a stage, the other group's waves read the next
// fragments, and a barrier between the halves keeps them in opposite phases,
// so the matrix pipe of each SIMD has one wave feeding it at every moment
// (with one group per block, or two independent blocks per CU, the fragment
// reads and the barrier of a stage left the pipe idle a third of the time).
// A stage of both operands is 48 KB (4 planes x 384 rows x 16 k); the ring
// has three slots, filled two stages ahead, which spans four half-stages of
// products for the load latency.
//
// Iteration j, slot j % 3: wait for this wave's loads of stage j (stage
// j + 1's may stay in flight; the wait also drains this wave's LDS reads);
// barrier (stage j is in LDS, every wave is done with stage j - 1's slot);
// request stage j + 2 into that slot; group 0 reads stage j while group 1
// multiplies stage j - 1; barrier; group 0 multiplies stage j while group 1
// reads stage j.  After the last iteration group 1 multiplies the last stage.
// Each wave issues the same number of loads per stage: every plane of the
// 256-row operand at rows 32 w .. 32 w + 31, and half the planes of the
// 128-row operand at rows 32 (w % 4) ...
constexpr int PPW = 256;  // rows of the wide operand's tile

int gemm_bf16_tile_m(int tile) { return tile == 2 ? PPW : BT; }
int gemm_bf16_tile_n(int tile) { return tile == 1 ? PPW : BT; }

template <bool WIDE_A>
__global__ __launch_bounds__(512, 1) void k_cgemm_bf16x3_pp(GemmArgs g) {
  constexpr int NP = 4, NACC = 2, NPROD = 12;
  constexpr int RA = WIDE_A ? PPW : BT, RB = WIDE_A ? BT : PPW;
  constexpr int DPA = RA * DBK, DPB = RB * DBK;  // bf16 per plane tile
  constexpr int STAGE = NP * (DPA + DPB);
  constexpr int LW = NP + NP / 2;                // loads of a wave per stage
  __shared__ __align__(16) uint16_t ring0[STAGE], ring1[STAGE], ring2[STAGE];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int grp = wave >> 2, wm = (wave >> 1) & 1, wn = wave & 1;
  const int q = blockIdx.y;
  const uint16_t *A = (const uint16_t *)g.A + q * g.abs;
  const uint16_t *B = (const uint16_t *)g.B + q * g.bbs;
  const Slot *sa = g.sa + q * g.sabs;
  const Slot *sb = g.sb + q * g.sbbs;
  Slot *sc = g.sc + q * g.scbs;
  int ks;
  int64_t t;
  gemm_block_tile(g, ks, t);  // XCD-aware block -> (k chunk, tile)
  const int64_t m0 = (t % g.tiles_m) * RA, n0 = (t / g.tiles_m) * RB;
  const int64_t kbeg = (int64_t)ks * g.kchunk;
  const int64_t kend = g.K < kbeg + g.kchunk ? g.K : kbeg + g.kchunk;
  const int ea = tn_scale_exp(sa->maxbits), eb = tn_scale_exp(sb->maxbits);
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

  // this wave's loads: rows ra0 / rb0 .. + 31 of the planes from pa0 / pb0
  // on (all of the wide operand's, half of the other's); this lane's row is
  // lane / 2 of those, logical chunk (lane % 2) ^ dswz(row), rows past M or
  // N clamped to the last one
  const int ra0 = WIDE_A ? 32 * wave : 32 * (wave & 3), rb0 = WIDE_A ? 32 * (wave & 3) : 32 * wave;
  const int pa0 = WIDE_A ? 0 : (wave >> 2) * (NP / 2), pb0 = WIDE_A ? (wave >> 2) * (NP / 2) : 0;
  constexpr int NLA = WIDE_A ? NP : NP / 2, NLB = WIDE_A ? NP / 2 : NP;
  const uint8_t *abase = (const uint8_t *)(A + m0 * DBK);
  const uint8_t *bbase = (const uint8_t *)(B + n0 * DBK);
  uint32_t aoff, boff;  // per lane, below 16 KB; the rest of an address is uniform
  {
    const int ra = ra0 + (lane >> 1), rb = rb0 + (lane >> 1);
    const int64_t ra_ = m0 + ra < g.M ? ra : g.M - 1 - m0;
    const int64_t rb_ = n0 + rb < g.N ? rb : g.N - 1 - n0;
    aoff = (uint32_t)((ra_ * DBK + ((lane & 1) ^ dswz(ra)) * 8) * 2);
    boff = (uint32_t)((rb_ * DBK + ((lane & 1) ^ dswz(rb)) * 8) * 2);
  }
  const int64_t nk = (kend - kbeg) / DBK;
#define TN_RING(S) ((S) == 0 ? ring0 : (S) == 1 ? ring1 : ring2)
  auto issue = [&](auto slot, int64_t stg) {
    constexpr int S = decltype(slot)::value;
    uint16_t *rs = TN_RING(S);
    const int64_t kb = kbeg / DBK + (stg < nk ? stg : nk - 1);
    const uint8_t *ak = abase + kb * g.M * DBK * 2, *bk = bbase + kb * g.N * DBK * 2;
#pragma unroll
    for (int i = 0; i < NLA; ++i)
      __builtin_amdgcn_global_load_lds((const void *)(ak + (pa0 + i) * g.pa * 2 + aoff),
                                       (lds_void *)(rs + (pa0 + i) * DPA + ra0 * DBK), 16, 0, 0);
#pragma unroll
    for (int i = 0; i < NLB; ++i)
      __builtin_amdgcn_global_load_lds((const void *)(bk + (pb0 + i) * g.pb * 2 + boff),
                                       (lds_void *)(rs + NP * DPA + (pb0 + i) * DPB + rb0 * DBK), 16, 0, 0);
  };
  // fragment rows of this wave's 64 x 64 part of its group's half
  const int fr = lane & 31, fpos = ((lane >> 5) ^ dswz(fr)) * 8;
  const int arow = (WIDE_A ? grp * BT : 0) + wm * 64 + fr;
  const int brow = (WIDE_A ? 0 : grp * BT) + wn * 64 + fr;
  auto fread = [&](auto slot, v4u (&a)[2][NP], v4u (&b)[2][NP]) {
    constexpr int S = decltype(slot)::value;
    const uint16_t *rs = TN_RING(S);
#pragma unroll
    for (int pp = 0; pp < NP; pp += 2) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int pl = pp; pl < pp + 2; ++pl)
          a[mb][pl] = *(const v4u *)(rs + pl * DPA + (arow + mb * 32) * DBK + fpos);
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int pl = pp; pl < pp + 2; ++pl)
          b[nb][pl] = *(const v4u *)(rs + NP * DPA + pl * DPB + (brow + nb * 32) * DBK + fpos);
    }
  };
#undef TN_RING
  auto mma = [&](const v4u (&a)[2][NP], const v4u (&b)[2][NP]) {
#pragma unroll
    for (int pi = 0; pi < NPROD; ++pi) {
      const int c = prod_4m(pi, 0), ap = prod_4m(pi, 1), bp = prod_4m(pi, 2), ng = prod_4m(pi, 3);
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const v8bf av = as_bf(ng ? neg4(a[mb][ap]) : a[mb][ap]);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          acc[mb][nb][c] =
              __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, as_bf(b[nb][bp]), acc[mb][nb][c], 0, 0, 0);
      }
    }
  };
  v4u fa[2][NP], fb[2][NP];
  // wait for stage j, barrier, request stage j + 2 into the slot of j - 1
  auto head = [&](auto slot, int64_t j) {
    constexpr int S = decltype(slot)::value;
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(dma_wait_imm(LW));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    issue(std::integral_constant<int, (S + 2) % 3>(), j + 2);
  };
  auto half = [&]() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  __builtin_amdgcn_s_waitcnt(0);  // nothing else in flight when the ring starts
  if (nk > 0) {
    issue(S0(), 0);
    issue(S1(), 1);
  }
  // each group runs its own loop (no branch inside, so the accumulators stay
  // in place); both pass the same barriers in the same order, two an
  // iteration
  if (grp == 0) {
    auto it = [&](auto slot, int64_t j) {
      head(slot, j);
      fread(slot, fa, fb);
      half();
      mma(fa, fb);
    };
    int64_t j = 0;
    for (; j + 3 <= nk; j += 3) {
      it(S0(), j);
      it(S1(), j + 1);
      it(S2(), j + 2);
    }
    if (j < nk) it(S0(), j);
    if (j + 1 < nk) it(S1(), j + 1);
  } else if (nk > 0) {
    // the loop turned so that a body reads its fragments and uses them
    // (nothing carried across the back edge): barrier, read stage j, wait and
    // barrier of stage j + 1 (with its request; none after the last stage),
    // products of stage j
    auto it = [&](auto slot, int64_t j) {
      constexpr int S = decltype(slot)::value;
      half();
      fread(slot, fa, fb);
      if (j + 1 < nk) head(std::integral_constant<int, (S + 1) % 3>(), j + 1);
      __builtin_amdgcn_sched_barrier(0);
      mma(fa, fb);
    };
    head(S0(), 0);
    int64_t j = 0;
    for (; j + 3 <= nk; j += 3) {
      it(S0(), j);
      it(S1(), j + 1);
      it(S2(), j + 2);
    }
    if (j < nk) it(S0(), j);
    if (j + 1 < nk) it(S1(), j + 1);
  }
  __builtin_amdgcn_s_waitcnt(0);  // no load may still write LDS when the block ends

  const bool partial = g.ksplit > 1;
  float2 *C = partial ? g.part + q * g.partbs + (int64_t)ks * g.M * g.N : g.C + q * g.cbs;
  const int64_t ldc = partial ? g.N : g.ldc;
  const int rbase = (WIDE_A ? grp * BT : 0) + wm * 64, cbase = (WIDE_A ? 0 : grp * BT) + wn * 64;
  // raw operands and the result as its parent's planes, as in the one-group
  // kernel
  const float post = (g.raw_a | g.raw_b) ? ldexpf(1.0f, -(g.raw_a ? ea : 0) - (g.raw_b ? eb : 0)) : 1.0f;
  const bool fo = g.fo_on != 0;
  uint8_t *const P0 = (uint8_t *)(g.C + q * g.cbs);
  uint8_t *const P[6] = {P0, P0 + g.fo_plane * 2, P0 + g.fo_plane * 4, P0 + g.fo_plane * 6, P0, P0};
  PlaneOut<2> po;
  if (fo) po.init(g, m0 + rbase + (lane >> 5) * 4, n0 + cbase + (lane & 31));
  float mx = 0.0f;
  if (fo && m0 + RA <= g.M && n0 + RB <= g.N) {
    // a whole tile of planes: no entry to test
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const float re = acc[mb][nb][0][v] * post, im = acc[mb][nb][1][v] * post;
          store_planes<4>(P, po.at(mb, nb, v), re, im);
          mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
  } else {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = rbase + mb * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
          const int col = cbase + nb * 32 + (lane & 31);
          const int64_t cm = m0 + row, cn = n0 + col;
          const float re = acc[mb][nb][0][v] * post, im = acc[mb][nb][1][v] * post;
          if (cm < g.M && cn < g.N) {
            if (fo)
              store_planes<4>(P, po.at(mb, nb, v), re, im);
            else
              C[cm * ldc + cn] = make_float2(re, im);
            mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
          }
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
  if (g.tile < 0 || g.tile > 2) return hipErrorInvalidValue;
  if ((g.raw_a || g.raw_b || g.fo_on) && !g.ktile) return hipErrorInvalidValue;
  if (g.fo_on && g.ksplit > 1) return hipErrorInvalidValue;
  // the two-group kernel: 4M from k-tiled planes with a wide tile
  const bool pp = g.ktile && form == kForm4M && g.tile != 0;
  g.tiles_m = (int)((g.M + (pp ? gemm_bf16_tile_m(g.tile) : BT) - 1) / (pp ? gemm_bf16_tile_m(g.tile) : BT));
  g.tiles_n = (int)((g.N + (pp ? gemm_bf16_tile_n(g.tile) : BT) - 1) / (pp ? gemm_bf16_tile_n(g.tile) : BT));
  if (g.ksplit < 1) g.ksplit = 1;
  if (g.ksplit == 1) g.kchunk = g.K;
  if (g.kchunk < 1 || (int64_t)g.ksplit * g.kchunk < g.K || (g.ksplit > 1 && !g.part))
    return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)g.tiles_m * g.tiles_n * g.ksplit;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks, nbatch);
  const bool exact = g.K % BKS == 0 && g.kchunk % BKS == 0;
  if (g.ktile) {
    if (g.K % DBK != 0 || g.kchunk % DBK != 0) return hipErrorInvalidValue;
    if (pp && g.tile == 2)
      hipLaunchKernelGGL(k_cgemm_bf16x3_pp<true>, grid, dim3(512), 0, st, g);
    else if (pp)
      hipLaunchKernelGGL(k_cgemm_bf16x3_pp<false>, grid, dim3(512), 0, st, g);
    else if (form == kForm4M)
      hipLaunchKernelGGL(k_cgemm_bf16x3_dma<kForm4M>, grid, dim3(256), 0, st, g);
    else
      hipLaunchKernelGGL(k_cgemm_bf16x3_dma<kForm3M>, grid, dim3(256), 0, st, g);
  } else if (form == kForm4M) {
    if (exact)
      hipLaunchKernelGGL((k_cgemm_bf16x3<kForm4M, true>), grid, dim3(256), 0, st, g);
    else
      hipLaunchKernelGGL((k_cgemm_bf16x3<kForm4M, false>), grid, dim3(256), 0, st, g);
  } else {
    if (exact)
      hipLaunchKernelGGL((k_cgemm_bf16x3<kForm3M, true>), grid, dim3(256), 0, st, g);
    else
      hipLaunchKernelGGL((k_cgemm_bf16x3<kForm3M, false>), grid, dim3(256), 0, st, g);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.ksplit == 1) return e;
  return launch_splitk_reduce(st, g, nbatch);
}

}  // namespace tn
