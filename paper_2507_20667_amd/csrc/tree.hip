// Subtree kernels: a whole subtree of small contractions in one workgroup.
//
// The many small contractions near the leaves of a circuit network (gate
// tensors of 2-16 entries meeting intermediates of up to a few thousand
// entries) would each be a launch of their own.  Here one workgroup takes one
// subtree for `qw` queries at once: it copies the subtree's leaves into LDS (a
// shared copy of the leaves no query overrides and of the shared
// intermediates it reads, a per-query copy of the overridden leaves, read in
// place from the caller's buffers), then runs the subtree's program with every
// operand and result in LDS, and finally writes the subtree's result and its
// scale record to device memory or, when the subtree ends in the network's
// closed root, the FP64 inner product.
//
// Two ways to run the program:
//  * k_tree (one query per launch: the shared subtrees, single queries): the
//    four waves share the query.  The program runs level by level; the
//    contractions of one level are independent, so up to kTreeChunk of them
//    share one barrier.  The descriptors of the next chunk are fetched while
//    the current one computes.
//  * k_tree_wave (a batch of queries): every wave takes its own queries
//    through the whole program, one step after the other, with no barrier
//    after the leaves are in LDS: a wave's LDS accesses complete in order, so
//    a step reads what the wave's earlier steps wrote.  The descriptors are
//    uniform across the wave and are read with scalar loads.  A chain of
//    small contractions (a gate sequence) then costs one wave's latency per
//    step instead of a workgroup barrier and a descriptor round trip, and the
//    other waves of the CU fill the gaps.
//
// Scales: every intermediate keeps a running integer log2 scale and the IEEE
// bits of its max |re|/|im|; a consumer multiplies its operands by 2^-e
// (e = floor(log2 max)), exactly as the one-contraction kernels do.
#include "tn_device.h"

namespace tn {

extern __shared__ __align__(16) unsigned char tree_lds[];

typedef const TreeLaunch __attribute__((address_space(4))) *KernargLaunch;
// step descriptors through the scalar cache (read only, uniform per wave)
typedef const TreeStep __attribute__((address_space(4))) *CStep;

// Index arithmetic: every offset, stride and index of a subtree is far below
// 2^24, so the full-rate 24-bit multiply-add serves (the 32-bit integer
// multiply runs at a quarter of the rate).
__device__ __forceinline__ int mad24(int a, int b, int c) {
  __builtin_assume((unsigned)a < (1u << 24));
  __builtin_assume((unsigned)b < (1u << 24));
  return (int)__umul24((unsigned)a, (unsigned)b) + c;
}

// entry at a byte offset from p
__device__ __forceinline__ const float2 &at_bytes(const float2 *p, int bytes) {
  return *(const float2 *)((const char *)p + bytes);
}

// Decode with the map held in registers (unrolled over kTreeSeg); P2: every
// extent a power of two, and `ext` holds the masks (extent - 1).
template <bool P2>
__device__ __forceinline__ void seg2r(const int32_t (&ext)[kTreeSeg], const int32_t (&s0)[kTreeSeg],
                                      const int32_t (&s1)[kTreeSeg], const int32_t (&lg)[kTreeSeg],
                                      int nseg, int idx, int &o0, int &o1) {
  o0 = 0;
  o1 = 0;
#pragma unroll
  for (int i = 0; i < kTreeSeg; ++i) {
    // power-of-two maps run every segment: an unused one has mask, shift and
    // strides 0 and adds nothing, which spares the scalar unit a test per
    // segment
    if (P2 || i < nseg) {
      int v;
      if (P2) {
        v = idx & ext[i];
        idx >>= lg[i];
      } else {
        v = idx % ext[i];
        idx /= ext[i];
      }
      o0 = mad24(v, s0[i], o0);
      o1 = mad24(v, s1[i], o1);
    }
  }
}

// A step's result entries are dealt to threads (an item: one result entry, or
// one fiber, of one query).  Every load of an item (the operands' scale
// records, the operand entries) is issued before anything is stored: a store
// to LDS ahead of a load keeps the compiler from moving the load up, and each
// LDS round trip then costs its full latency.  The results, the result's log2
// scale and the running max |re|/|im| (folded into the scale record with an
// LDS atomic) follow.  ONE: the group holds a single query, so its pointers
// and operand scales are the same for every item (uniform, computed once).
struct ItemScale {
  int2 za, zb;
  __device__ __forceinline__ int e() const { return tn_scale_exp((uint32_t)za.y) + tn_scale_exp((uint32_t)zb.y); }
};

__device__ __forceinline__ ItemScale item_scale(const int2 *sc, int asl, int bsl) {
  ItemScale z;
  z.za = asl >= 0 ? sc[asl] : make_int2(0, 0);
  z.zb = bsl >= 0 ? sc[bsl] : make_int2(0, 0);
  return z;
}

// The operand scales of a single-query step, read once and made uniform.
__device__ __forceinline__ ItemScale uniform_scale(const int2 *sc, int asl, int bsl) {
  ItemScale z = item_scale(sc, asl, bsl);
  z.za.x = __builtin_amdgcn_readfirstlane(z.za.x);
  z.za.y = __builtin_amdgcn_readfirstlane(z.za.y);
  z.zb.x = __builtin_amdgcn_readfirstlane(z.zb.x);
  z.zb.y = __builtin_amdgcn_readfirstlane(z.zb.y);
  return z;
}

__device__ __forceinline__ void fold_max(int2 *scl, int nscale, int csl, int q, int &qprev, float &mx,
                                         float m) {
  if (q != qprev) {
    if (qprev >= 0) atomicMax((unsigned int *)&scl[mad24(qprev, nscale, csl)].y, __float_as_uint(mx));
    qprev = q;
    mx = 0.f;
  }
  mx = fmaxf(mx, m);
}

// Kind 2: one thread per fiber of the large operand X (and query) reads the
// fiber's ns entries once and writes nfy results; the small operand Y sits in
// registers.
template <bool ONE, bool P2, int NS, int NFY, class SP>
__device__ __forceinline__ void tree_stream_impl(SP Sp, int lane, int nthr, int nqw, float2 *pq,
                                                 int perq, const float2 *shr, int2 *scl,
                                                 int nscale) {
  const int a = Sp->a, b = Sp->b, c = Sp->c, asl = Sp->asl, bsl = Sp->bsl, csl = Sp->csl;
  const int nfib = Sp->nc / NFY, ncs = Sp->ncs;
  const int lgf = P2 ? __builtin_ctz((unsigned)nfib) : 0;
  int32_t fext[kTreeSeg], fx[kTreeSeg], fc[kTreeSeg], flg[kTreeSeg];
#pragma unroll
  for (int i = 0; i < kTreeSeg; ++i) {
    fext[i] = Sp->cext[i];
    fx[i] = Sp->ca[i];
    fc[i] = Sp->cb[i];
    flg[i] = Sp->clg[i];
  }
  int xs[NS], cy[NFY], ym[NS * NFY];
#pragma unroll
  for (int v = 0; v < NS; ++v) xs[v] = Sp->xs[v];
#pragma unroll
  for (int v = 0; v < NFY; ++v) cy[v] = Sp->cy[v];
#pragma unroll
  for (int v = 0; v < NS * NFY; ++v) ym[v] = Sp->ymap[v];
  if constexpr (ONE) {
    const float2 *X = (a & kPerQuery) ? pq + (a & ~kPerQuery) : shr + a;
    const float2 *Y = (b & kPerQuery) ? pq + (b & ~kPerQuery) : shr + b;
    float2 *C = pq + (c & ~kPerQuery);
    if (NFY > 1 && nfib * NFY <= nthr) {
      // one result per thread, thread (fiber, j): a quarter (half) of the
      // multiply-adds, loads and stores per thread of a fiber's nfy results.
      // Y's shared and free legs are apart, so ymap[s * nfy + j] =
      // ymap[s * nfy] + (ymap[j] - ymap[0]).
      if (lane >= nfib * NFY) return;
      const int j = lane & (NFY - 1), fi = lane >> (NFY == 4 ? 2 : 1);
      int dj = 0, cj = cy[0];
#pragma unroll
      for (int v = 1; v < NFY; ++v)
        if (j == v) {
          dj = ym[v] - ym[0];
          cj = cy[v];
        }
      int xo, co;
      seg2r<P2>(fext, fx, fc, flg, ncs, fi, xo, co);
      float2 x[NS], yv[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        x[s] = at_bytes(X + xo, xs[s]);
        yv[s] = at_bytes(Y, ym[s * NFY] + dj);
      }
      const ItemScale z = uniform_scale(scl, asl, bsl);
      const int e = z.e();
      const float f = ldexpf(1.0f, -e);
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        re = fmaf(x[s].x, yv[s].x, re);
        re = fmaf(-x[s].y, yv[s].y, re);
        im = fmaf(x[s].x, yv[s].y, im);
        im = fmaf(x[s].y, yv[s].x, im);
      }
      re *= f;
      im *= f;
      *(float2 *)((char *)(C + co) + cj) = make_float2(re, im);
      if (lane == 0) scl[csl].x = z.za.x + z.zb.x + e;
      atomicMax((unsigned int *)&scl[csl].y, __float_as_uint(fmaxf(fabsf(re), fabsf(im))));
      return;
    }
    if (lane >= nfib) return;
    float2 y[NS * NFY];
#pragma unroll
    for (int v = 0; v < NS * NFY; ++v) y[v] = at_bytes(Y, ym[v]);
    const ItemScale z = uniform_scale(scl, asl, bsl);
    const int e = z.e();
    const float f = ldexpf(1.0f, -e);
    float mx = 0.f;
    for (int fi = lane; fi < nfib; fi += nthr) {
      int xo, co;
      seg2r<P2>(fext, fx, fc, flg, ncs, fi, xo, co);
      float2 x[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) x[s] = at_bytes(X + xo, xs[s]);
#pragma unroll
      for (int j = 0; j < NFY; ++j) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const float2 yv = y[s * NFY + j];
          re = fmaf(x[s].x, yv.x, re);
          re = fmaf(-x[s].y, yv.y, re);
          im = fmaf(x[s].x, yv.y, im);
          im = fmaf(x[s].y, yv.x, im);
        }
        re *= f;
        im *= f;
        *(float2 *)((char *)(C + co) + cy[j]) = make_float2(re, im);
        mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
      }
    }
    if (lane == 0) scl[csl].x = z.za.x + z.zb.x + e;
    atomicMax((unsigned int *)&scl[csl].y, __float_as_uint(mx));
  } else {
    const int total = nqw * nfib;
    int qprev = -1;
    float mx = 0.f;
    for (int w = lane; w < total; w += nthr) {
      const int q = P2 ? (w >> lgf) : w / nfib;
      const int fi = P2 ? (w & (nfib - 1)) : w - mad24(q, nfib, 0);
      float2 *base = pq + mad24(q, perq, 0);
      const float2 *X = (a & kPerQuery) ? base + (a & ~kPerQuery) : shr + a;
      const float2 *Y = (b & kPerQuery) ? base + (b & ~kPerQuery) : shr + b;
      const ItemScale z = item_scale(scl + mad24(q, nscale, 0), asl, bsl);
      int xo, co;
      seg2r<P2>(fext, fx, fc, flg, ncs, fi, xo, co);
      float2 x[NS], y[NS * NFY];
#pragma unroll
      for (int v = 0; v < NS * NFY; ++v) y[v] = at_bytes(Y, ym[v]);
#pragma unroll
      for (int s = 0; s < NS; ++s) x[s] = at_bytes(X + xo, xs[s]);
      const int e = z.e();
      const float f = ldexpf(1.0f, -e);
      float2 *C = base + (c & ~kPerQuery);
      float m = 0.f;
#pragma unroll
      for (int j = 0; j < NFY; ++j) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const float2 yv = y[s * NFY + j];
          re = fmaf(x[s].x, yv.x, re);
          re = fmaf(-x[s].y, yv.y, re);
          im = fmaf(x[s].x, yv.y, im);
          im = fmaf(x[s].y, yv.x, im);
        }
        re *= f;
        im *= f;
        *(float2 *)((char *)(C + co) + cy[j]) = make_float2(re, im);
        m = fmaxf(m, fmaxf(fabsf(re), fabsf(im)));
      }
      if (fi == 0) scl[mad24(q, nscale, csl)].x = z.za.x + z.zb.x + e;
      fold_max(scl, nscale, csl, q, qprev, mx, m);
    }
    if (qprev >= 0) atomicMax((unsigned int *)&scl[mad24(qprev, nscale, csl)].y, __float_as_uint(mx));
  }
}

// The shared index of a kind 0 item summed four terms at a time (offsets of
// term s in lane s of soa/sob when ns <= 64).
template <bool P2>
__device__ __forceinline__ float2 dot_terms(const float2 *A, const float2 *B, int ns, bool stab, int soa,
                                            int sob, const int32_t (&sext)[kTreeSeg],
                                            const int32_t (&sa)[kTreeSeg], const int32_t (&sb)[kTreeSeg],
                                            const int32_t (&slg)[kTreeSeg], int nss) {
  float re0 = 0.f, im0 = 0.f, re1 = 0.f, im1 = 0.f;
  if (stab) {
    int s = 0;
    for (; s + 4 <= ns; s += 4) {
      float2 x[4], y[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        x[t] = A[__builtin_amdgcn_readlane(soa, s + t)];
        y[t] = B[__builtin_amdgcn_readlane(sob, s + t)];
      }
#pragma unroll
      for (int t = 0; t < 4; t += 2) {
        re0 = fmaf(x[t].x, y[t].x, re0);
        re0 = fmaf(-x[t].y, y[t].y, re0);
        im0 = fmaf(x[t].x, y[t].y, im0);
        im0 = fmaf(x[t].y, y[t].x, im0);
        re1 = fmaf(x[t + 1].x, y[t + 1].x, re1);
        re1 = fmaf(-x[t + 1].y, y[t + 1].y, re1);
        im1 = fmaf(x[t + 1].x, y[t + 1].y, im1);
        im1 = fmaf(x[t + 1].y, y[t + 1].x, im1);
      }
    }
    for (; s < ns; ++s) {
      const float2 x = A[__builtin_amdgcn_readlane(soa, s)], y = B[__builtin_amdgcn_readlane(sob, s)];
      re0 = fmaf(x.x, y.x, re0);
      re0 = fmaf(-x.y, y.y, re0);
      im0 = fmaf(x.x, y.y, im0);
      im0 = fmaf(x.y, y.x, im0);
    }
  } else {
    for (int s = 0; s < ns; ++s) {
      int oa, ob;
      seg2r<P2>(sext, sa, sb, slg, nss, s, oa, ob);
      const float2 x = A[oa], y = B[ob];
      re0 = fmaf(x.x, y.x, re0);
      re0 = fmaf(-x.y, y.y, re0);
      im0 = fmaf(x.x, y.y, im0);
      im0 = fmaf(x.y, y.x, im0);
    }
  }
  return make_float2(re0 + re1, im0 + im1);
}

// Kind 0: one thread per result entry (and query).
template <bool ONE, bool P2, class SP>
__device__ __forceinline__ void tree_step_impl(SP Sp, int lane, int nthr, int nqw, float2 *pq,
                                               int perq, const float2 *shr, int2 *scl, int nscale) {
  const int a = Sp->a, b = Sp->b, c = Sp->c, asl = Sp->asl, bsl = Sp->bsl, csl = Sp->csl;
  const int nc = Sp->nc, ns = Sp->ns, ncs = Sp->ncs, nss = Sp->nss;
  const int lgnc = P2 ? __builtin_ctz((unsigned)nc) : 0;
  int32_t cext[kTreeSeg], ca[kTreeSeg], cb[kTreeSeg], clg[kTreeSeg];
  int32_t sext[kTreeSeg], sa[kTreeSeg], sb[kTreeSeg], slg[kTreeSeg];
#pragma unroll
  for (int i = 0; i < kTreeSeg; ++i) {
    cext[i] = Sp->cext[i];
    ca[i] = Sp->ca[i];
    cb[i] = Sp->cb[i];
    clg[i] = Sp->clg[i];
    sext[i] = Sp->sext[i];
    sa[i] = Sp->sa[i];
    sb[i] = Sp->sb[i];
    slg[i] = Sp->slg[i];
  }
  // shared-index offsets, computed once per wave: hardware lane l holds those
  // of s = l (ns <= 64), read back in the inner loop with readlane (s is the
  // same in every lane there); every lane of the wave is active here
  const int hl = threadIdx.x & 63;
  const bool stab = ns <= 64;
  int soa = 0, sob = 0;
  if (stab && hl < ns) seg2r<P2>(sext, sa, sb, slg, nss, hl, soa, sob);
  if constexpr (ONE) {
    const float2 *A0 = (a & kPerQuery) ? pq + (a & ~kPerQuery) : shr + a;
    const float2 *B0 = (b & kPerQuery) ? pq + (b & ~kPerQuery) : shr + b;
    float2 *C = pq + (c & ~kPerQuery);
    if (lane >= nc) return;
    const ItemScale z = uniform_scale(scl, asl, bsl);
    const int e = z.e();
    const float f = ldexpf(1.0f, -e);
    float mx = 0.f;
    for (int ci = lane; ci < nc; ci += nthr) {
      int ao, bo;
      seg2r<P2>(cext, ca, cb, clg, ncs, ci, ao, bo);
      const float2 r = dot_terms<P2>(A0 + ao, B0 + bo, ns, stab, soa, sob, sext, sa, sb, slg, nss);
      const float rr = r.x * f, ii = r.y * f;
      C[ci] = make_float2(rr, ii);
      mx = fmaxf(mx, fmaxf(fabsf(rr), fabsf(ii)));
    }
    if (lane == 0) scl[csl].x = z.za.x + z.zb.x + e;
    atomicMax((unsigned int *)&scl[csl].y, __float_as_uint(mx));
  } else {
    const int total = nqw * nc;
    int qprev = -1;
    float mx = 0.f;
    for (int w = lane; w < total; w += nthr) {
      const int q = P2 ? (w >> lgnc) : w / nc;
      const int ci = P2 ? (w & (nc - 1)) : w - mad24(q, nc, 0);
      float2 *base = pq + mad24(q, perq, 0);
      int ao, bo;
      seg2r<P2>(cext, ca, cb, clg, ncs, ci, ao, bo);
      const float2 *A = ((a & kPerQuery) ? base + (a & ~kPerQuery) : shr + a) + ao;
      const float2 *B = ((b & kPerQuery) ? base + (b & ~kPerQuery) : shr + b) + bo;
      const ItemScale z = item_scale(scl + mad24(q, nscale, 0), asl, bsl);
      const float2 r = dot_terms<P2>(A, B, ns, stab, soa, sob, sext, sa, sb, slg, nss);
      const int e = z.e();
      const float f = ldexpf(1.0f, -e);
      const float rr = r.x * f, ii = r.y * f;
      base[(c & ~kPerQuery) + ci] = make_float2(rr, ii);
      if (ci == 0) scl[mad24(q, nscale, csl)].x = z.za.x + z.zb.x + e;
      fold_max(scl, nscale, csl, q, qprev, mx, fmaxf(fabsf(rr), fabsf(ii)));
    }
    if (qprev >= 0) atomicMax((unsigned int *)&scl[mad24(qprev, nscale, csl)].y, __float_as_uint(mx));
  }
}

// One contraction for every query of the group, by `nthr` threads starting at
// `lane`.  The step's maps live in registers; each thread keeps the running
// max of its results per query and folds it into the scale record once per
// query.
template <bool ONE, class SP>
__device__ __forceinline__ void tree_step_q(SP Sp, int lane, int nthr, int nqw, float2 *pq, int perq,
                                            const float2 *shr, int2 *scl, int nscale) {
  if (Sp->kind == 2) {
    // a small operand along the fibers of a large one: ns, nfy in {1, 2, 4}
    const int sel = (Sp->ns >> 1) * 3 + (Sp->nss >> 1) + (Sp->pow2 ? 0 : 9);
#define TN_TS(P, A, B) tree_stream_impl<ONE, P, A, B>(Sp, lane, nthr, nqw, pq, perq, shr, scl, nscale)
    switch (sel) {
      case 0: TN_TS(true, 1, 1); break;
      case 1: TN_TS(true, 1, 2); break;
      case 2: TN_TS(true, 1, 4); break;
      case 3: TN_TS(true, 2, 1); break;
      case 4: TN_TS(true, 2, 2); break;
      case 5: TN_TS(true, 2, 4); break;
      case 6: TN_TS(true, 4, 1); break;
      case 7: TN_TS(true, 4, 2); break;
      case 8: TN_TS(true, 4, 4); break;
      case 9: TN_TS(false, 1, 1); break;
      case 10: TN_TS(false, 1, 2); break;
      case 11: TN_TS(false, 1, 4); break;
      case 12: TN_TS(false, 2, 1); break;
      case 13: TN_TS(false, 2, 2); break;
      case 14: TN_TS(false, 2, 4); break;
      case 15: TN_TS(false, 4, 1); break;
      case 16: TN_TS(false, 4, 2); break;
      default: TN_TS(false, 4, 4); break;
    }
#undef TN_TS
    return;
  }
  if (Sp->pow2)
    tree_step_impl<ONE, true>(Sp, lane, nthr, nqw, pq, perq, shr, scl, nscale);
  else
    tree_step_impl<ONE, false>(Sp, lane, nthr, nqw, pq, perq, shr, scl, nscale);
}

// Kind 3: the kind 0 form with some operands in the query's device workspace
// (a large intermediate of a per-query subtree), reached through generic
// pointers.  gq: the device workspace of the group's first query, gstride
// float2 apart.
template <bool P2, class SP>
__device__ __forceinline__ void tree_dev_impl(SP Sp, int lane, int nthr, int nqw, float2 *pq, int perq,
                              const float2 *shr, int2 *scl, int nscale, float2 *gq, int64_t gstride) {
  const int a = Sp->a, b = Sp->b, c = Sp->c, asl = Sp->asl, bsl = Sp->bsl, csl = Sp->csl;
  const int nc = Sp->nc, ns = Sp->ns, ncs = Sp->ncs, nss = Sp->nss, glob = Sp->glob;
  int32_t cext[kTreeSeg], ca[kTreeSeg], cb[kTreeSeg], clg[kTreeSeg];
  int32_t sext[kTreeSeg], sa[kTreeSeg], sb[kTreeSeg], slg[kTreeSeg];
#pragma unroll
  for (int i = 0; i < kTreeSeg; ++i) {
    cext[i] = Sp->cext[i];
    ca[i] = Sp->ca[i];
    cb[i] = Sp->cb[i];
    clg[i] = Sp->clg[i];
    sext[i] = Sp->sext[i];
    sa[i] = Sp->sa[i];
    sb[i] = Sp->sb[i];
    slg[i] = Sp->slg[i];
  }
  const int hl = threadIdx.x & 63;
  const bool stab = ns <= 64;
  int soa = 0, sob = 0;
  if (stab && hl < ns) seg2r<P2>(sext, sa, sb, slg, nss, hl, soa, sob);
  const int total = nqw * nc;
  int qprev = -1;
  float mx = 0.f;
  for (int w = lane; w < total; w += nthr) {
    const int q = w / nc;
    const int ci = w - q * nc;
    float2 *base = pq + mad24(q, perq, 0);
    float2 *dev = gq + (int64_t)q * gstride;
    const float2 *A = (glob & 1) ? dev + a : ((a & kPerQuery) ? base + (a & ~kPerQuery) : shr + a);
    const float2 *B = (glob & 2) ? dev + b : ((b & kPerQuery) ? base + (b & ~kPerQuery) : shr + b);
    float2 *C = (glob & 4) ? dev + c : base + (c & ~kPerQuery);
    int ao, bo;
    seg2r<P2>(cext, ca, cb, clg, ncs, ci, ao, bo);
    const ItemScale z = item_scale(scl + mad24(q, nscale, 0), asl, bsl);
    const float2 r = dot_terms<P2>(A + ao, B + bo, ns, stab, soa, sob, sext, sa, sb, slg, nss);
    const int e = z.e();
    const float f = ldexpf(1.0f, -e);
    const float rr = r.x * f, ii = r.y * f;
    C[ci] = make_float2(rr, ii);
    if (ci == 0) scl[mad24(q, nscale, csl)].x = z.za.x + z.zb.x + e;
    fold_max(scl, nscale, csl, q, qprev, mx, fmaxf(fabsf(rr), fabsf(ii)));
  }
  if (qprev >= 0) atomicMax((unsigned int *)&scl[mad24(qprev, nscale, csl)].y, __float_as_uint(mx));
}

// Kind 3 for a single query with power-of-two maps.  GLOB (bit 1: A, 2: B,
// 4: C in the device workspace) is a template argument here, so that every
// operand has one memory space the compiler knows: LDS operands are read with
// LDS instructions and the device workspace with global ones (a pointer that
// may point at either compiles to the slower flat instructions).  The items
// are dealt as in the single-query kind 0 form: operand scales read once,
// no division per item.
template <int GLOB, class SP>
__device__ __forceinline__ void tree_dev_one(SP Sp, int lane, int nthr, float2 *pq, const float2 *shr,
                                             int2 *scl, float2 *gq) {
  const int a = Sp->a, b = Sp->b, c = Sp->c, asl = Sp->asl, bsl = Sp->bsl, csl = Sp->csl;
  const int nc = Sp->nc, ns = Sp->ns, ncs = Sp->ncs, nss = Sp->nss;
  int32_t cext[kTreeSeg], ca[kTreeSeg], cb[kTreeSeg], clg[kTreeSeg];
  int32_t sext[kTreeSeg], sa[kTreeSeg], sb[kTreeSeg], slg[kTreeSeg];
#pragma unroll
  for (int i = 0; i < kTreeSeg; ++i) {
    cext[i] = Sp->cext[i];
    ca[i] = Sp->ca[i];
    cb[i] = Sp->cb[i];
    clg[i] = Sp->clg[i];
    sext[i] = Sp->sext[i];
    sa[i] = Sp->sa[i];
    sb[i] = Sp->sb[i];
    slg[i] = Sp->slg[i];
  }
  const int hl = threadIdx.x & 63;
  const bool stab = ns <= 64;
  int soa = 0, sob = 0;
  if (stab && hl < ns) seg2r<true>(sext, sa, sb, slg, nss, hl, soa, sob);
  const float2 *A0, *B0;
  float2 *C;
  if constexpr ((GLOB & 1) != 0)
    A0 = gq + a;
  else
    A0 = (a & kPerQuery) ? pq + (a & ~kPerQuery) : shr + a;
  if constexpr ((GLOB & 2) != 0)
    B0 = gq + b;
  else
    B0 = (b & kPerQuery) ? pq + (b & ~kPerQuery) : shr + b;
  if constexpr ((GLOB & 4) != 0)
    C = gq + c;
  else
    C = pq + (c & ~kPerQuery);
  const ItemScale z = uniform_scale(scl, asl, bsl);
  const int e = z.e();
  const float f = ldexpf(1.0f, -e);
  float mx = 0.f;
  for (int ci = lane; ci < nc; ci += nthr) {
    int ao, bo;
    seg2r<true>(cext, ca, cb, clg, ncs, ci, ao, bo);
    const float2 r = dot_terms<true>(A0 + ao, B0 + bo, ns, stab, soa, sob, sext, sa, sb, slg, nss);
    const float rr = r.x * f, ii = r.y * f;
    C[ci] = make_float2(rr, ii);
    mx = fmaxf(mx, fmaxf(fabsf(rr), fabsf(ii)));
  }
  if (lane == 0) scl[csl].x = z.za.x + z.zb.x + e;
  atomicMax((unsigned int *)&scl[csl].y, __float_as_uint(mx));
}

// Kind 4: up to 64 result entries of a level's small gate steps, one per
// lane.  A lane reads its addresses and scale records from its lane record
// (one global load of 16 bytes, two for ns = 4, from a table every wave of the
// launch reads) instead of decoding a step's maps, so several independent
// small steps cost one step of the wave.  Single-query groups only.
// r0, r1: the lane's record (r1 for ns = 4 only).
template <int NS>
__device__ __forceinline__ void tree_lane_exec(uint4 r0, uint4 r1, float2 *pq, const float2 *shr,
                                               int2 *scl) {
  // each operand's region once (bits 15 and 31 of w[3]), then byte offsets
  const char *xb = (const char *)((r0.w & 0x8000u) ? shr : pq);
  const char *yb = (const char *)((r0.w >> 31) ? shr : pq);
  auto at = [](const char *base, uint32_t off) -> float2 { return *(const float2 *)(base + off); };
  float2 x[NS], y[NS];
  x[0] = at(xb, r0.x & 0xffffu);
  y[0] = at(yb, r0.y & 0xffffu);
  if (NS >= 2) {
    x[1] = at(xb, r0.x >> 16);
    y[1] = at(yb, r0.y >> 16);
  }
  if (NS == 4) {
    x[2] = at(xb, r1.x & 0xffffu);
    x[3] = at(xb, r1.x >> 16);
    y[2] = at(yb, r1.y & 0xffffu);
    y[3] = at(yb, r1.y >> 16);
  }
  // a leaf operand's index is that of a record that stays zero
  const int2 za = scl[r0.w & 0x7fffu], zb = scl[(r0.w >> 16) & 0x7fffu];
  const int e = tn_scale_exp((uint32_t)za.y) + tn_scale_exp((uint32_t)zb.y);
  const float f = ldexpf(1.0f, -e);
  float re = 0.f, im = 0.f;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    re = fmaf(x[s].x, y[s].x, re);
    re = fmaf(-x[s].y, y[s].y, re);
    im = fmaf(x[s].x, y[s].y, im);
    im = fmaf(x[s].y, y[s].x, im);
  }
  re *= f;
  im *= f;
  *(float2 *)((char *)pq + (r0.z & 0xffffu)) = make_float2(re, im);
  const int csl = (int)((r0.z >> 16) & 0x7fffu);
  if (r0.z >> 31) scl[csl].x = za.x + zb.x + e;
  atomicMax((unsigned int *)&scl[csl].y, __float_as_uint(fmaxf(fabsf(re), fabsf(im))));
}

// The largest of v over the wave, in a scalar register (every lane of the
// wave active): a butterfly inside each row of 16 lanes by DPP moves, then the
// four rows' values read out.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // lane ^ 1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // lane ^ 2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // 7 - lane in 8
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // 15 - lane in 16
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
  const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(r0, r1), max(r2, r3));
}

// Kind 4 holding one whole kind 2 step (nss = 1), run by a whole wave (lanes
// past nc inactive in the arithmetic only): the operand scales are the same
// for every lane, and the wave writes the result's scale record with one
// store, its max reduced across the wave, instead of one LDS atomic per lane
// on one word.
template <int NS>
__device__ __forceinline__ void tree_lane_whole(uint4 r0, uint4 r1, bool act, int lane, float2 *pq,
                                                const float2 *shr, int2 *scl) {
  const uint32_t w3 = (uint32_t)__builtin_amdgcn_readfirstlane((int)r0.w);  // lane 0 is active
  const uint32_t wz = (uint32_t)__builtin_amdgcn_readfirstlane((int)r0.z);
  const int2 za = scl[w3 & 0x7fffu], zb = scl[(w3 >> 16) & 0x7fffu];
  const int zax = __builtin_amdgcn_readfirstlane(za.x), zay = __builtin_amdgcn_readfirstlane(za.y);
  const int zbx = __builtin_amdgcn_readfirstlane(zb.x), zby = __builtin_amdgcn_readfirstlane(zb.y);
  const int e = tn_scale_exp((uint32_t)zay) + tn_scale_exp((uint32_t)zby);
  float m = 0.f;
  if (act) {
    const char *xb = (const char *)((w3 & 0x8000u) ? shr : pq);
    const char *yb = (const char *)((w3 >> 31) ? shr : pq);
    auto at = [](const char *base, uint32_t off) -> float2 { return *(const float2 *)(base + off); };
    float2 x[NS], y[NS];
    x[0] = at(xb, r0.x & 0xffffu);
    y[0] = at(yb, r0.y & 0xffffu);
    if (NS >= 2) {
      x[1] = at(xb, r0.x >> 16);
      y[1] = at(yb, r0.y >> 16);
    }
    if (NS == 4) {
      x[2] = at(xb, r1.x & 0xffffu);
      x[3] = at(xb, r1.x >> 16);
      y[2] = at(yb, r1.y & 0xffffu);
      y[3] = at(yb, r1.y >> 16);
    }
    const float f = ldexpf(1.0f, -e);
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      re = fmaf(x[s].x, y[s].x, re);
      re = fmaf(-x[s].y, y[s].y, re);
      im = fmaf(x[s].x, y[s].y, im);
      im = fmaf(x[s].y, y[s].x, im);
    }
    re *= f;
    im *= f;
    *(float2 *)((char *)pq + (r0.z & 0xffffu)) = make_float2(re, im);
    m = fmaxf(fabsf(re), fabsf(im));
  }
  const unsigned mx = wave_max_u32(__float_as_uint(m));
  if (lane == 0) scl[(wz >> 16) & 0x7fffu] = make_int2(zax + zbx + e, (int)mx);
}

// Kind 5 (the batch kernel's program only): a chain of whole-vertex gate
// steps in which every step after the first takes the previous one's result
// as its X operand.  The running tensor stays in registers (lane l holds the
// entry its record names); a link reads its X terms from the lanes that hold
// them (ds_bpermute, the source lanes prepared on the host), its Y terms (the
// gate's entries) from LDS, and its X scale record from the link before (in
// scalar registers).  Only the last link writes its result and scale record
// to LDS: no other step reads the others (each vertex has one consumer).
// Term order, scaling and the wave-wide max are those of the kind 4 steps it
// replaces, so the results are the same bit for bit.  Link j's records are
// the 64 at rec + 64 j: w[0], w[4] the X terms (link 0: byte offsets in the
// X region; later links: source lane * 4), w[1], w[5] the Y byte offsets,
// w[2], w[3] as in kind 4, w[6] = ns | nc << 8 (lanes past nc are padding
// with valid offsets, inactive in the result).
template <int NS, bool FIRST, bool LAST>
__device__ __forceinline__ void chain_link(uint4 a0, uint4 a1, int lane, float2 *pq, const float2 *shr,
                                           int2 *scl, float &vre, float &vim, int &zx, int &zy) {
  const uint32_t w3 = (uint32_t)__builtin_amdgcn_readfirstlane((int)a0.w);
  const uint32_t wz = (uint32_t)__builtin_amdgcn_readfirstlane((int)a0.z);
  const int nc = (__builtin_amdgcn_readfirstlane((int)a1.z) >> 8) & 0xff;
  const bool act = lane < nc;
  const int2 zb = scl[(w3 >> 16) & 0x7fffu];
  int2 za = make_int2(0, 0);
  if (FIRST) za = scl[w3 & 0x7fffu];
  const char *yb = (const char *)((w3 >> 31) ? shr : pq);
  auto at = [](const char *base, uint32_t off) -> float2 { return *(const float2 *)(base + off); };
  float2 x[NS], y[NS];
  y[0] = at(yb, a0.y & 0xffffu);
  if (NS >= 2) y[1] = at(yb, a0.y >> 16);
  if (NS == 4) {
    y[2] = at(yb, a1.y & 0xffffu);
    y[3] = at(yb, a1.y >> 16);
  }
  if (FIRST) {
    const char *xb = (const char *)((w3 & 0x8000u) ? shr : pq);
    x[0] = at(xb, a0.x & 0xffffu);
    if (NS >= 2) x[1] = at(xb, a0.x >> 16);
    if (NS == 4) {
      x[2] = at(xb, a1.x & 0xffffu);
      x[3] = at(xb, a1.x >> 16);
    }
  } else {
    const int ir = __float_as_int(vre), ii = __float_as_int(vim);
    auto from = [&](uint32_t addr) {
      return make_float2(__int_as_float(__builtin_amdgcn_ds_bpermute((int)addr, ir)),
                         __int_as_float(__builtin_amdgcn_ds_bpermute((int)addr, ii)));
    };
    x[0] = from(a0.x & 0xffffu);
    if (NS >= 2) x[1] = from(a0.x >> 16);
    if (NS == 4) {
      x[2] = from(a1.x & 0xffffu);
      x[3] = from(a1.x >> 16);
    }
  }
  if (FIRST) {
    zx = __builtin_amdgcn_readfirstlane(za.x);
    zy = __builtin_amdgcn_readfirstlane(za.y);
  }
  const int zbx = __builtin_amdgcn_readfirstlane(zb.x), zby = __builtin_amdgcn_readfirstlane(zb.y);
  const int e = tn_scale_exp((uint32_t)zy) + tn_scale_exp((uint32_t)zby);
  const float f = ldexpf(1.0f, -e);
  float re = 0.f, im = 0.f;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    re = fmaf(x[s].x, y[s].x, re);
    re = fmaf(-x[s].y, y[s].y, re);
    im = fmaf(x[s].x, y[s].y, im);
    im = fmaf(x[s].y, y[s].x, im);
  }
  re *= f;
  im *= f;
  const float m = act ? fmaxf(fabsf(re), fabsf(im)) : 0.f;
  const unsigned mx = wave_max_u32(__float_as_uint(m));
  zx = zx + zbx + e;
  zy = (int)mx;
  if (LAST) {
    if (act) *(float2 *)((char *)pq + (a0.z & 0xffffu)) = make_float2(re, im);
    if (lane == 0) scl[(wz >> 16) & 0x7fffu] = make_int2(zx, zy);
  }
  vre = re;
  vim = im;
}

template <bool FIRST, bool LAST>
__device__ __forceinline__ void chain_link_ns(int ns, uint4 a0, uint4 a1, int lane, float2 *pq,
                                              const float2 *shr, int2 *scl, float &vre, float &vim, int &zx,
                                              int &zy) {
  if (ns == 1)
    chain_link<1, FIRST, LAST>(a0, a1, lane, pq, shr, scl, vre, vim, zx, zy);
  else if (ns == 2)
    chain_link<2, FIRST, LAST>(a0, a1, lane, pq, shr, scl, vre, vim, zx, zy);
  else
    chain_link<4, FIRST, LAST>(a0, a1, lane, pq, shr, scl, vre, vim, zx, zy);
}

// A whole kind 5 step: `nlinks` links, link 0's record prefetched in r0, r1;
// each later link's record is loaded while the link before runs.
__device__ __forceinline__ void tree_chain(const TreeLaneRec *rec, int nlinks, uint4 r0, uint4 r1, int lane,
                                           float2 *pq, const float2 *shr, int2 *scl) {
  float vre = 0.f, vim = 0.f;
  int zx = 0, zy = 0;
  uint4 n0 = r0, n1 = r1;
  for (int j = 0; j < nlinks; ++j) {
    const uint4 a0 = n0, a1 = n1;
    if (j + 1 < nlinks) {
      const uint4 *nx = (const uint4 *)(rec + (j + 1) * 64 + lane);
      n0 = nx[0];
      n1 = nx[1];
    }
    const int ns = __builtin_amdgcn_readfirstlane((int)a1.z) & 0xff;
    if (j == 0)
      chain_link_ns<true, false>(ns, a0, a1, lane, pq, shr, scl, vre, vim, zx, zy);
    else if (j + 1 < nlinks)
      chain_link_ns<false, false>(ns, a0, a1, lane, pq, shr, scl, vre, vim, zx, zy);
    else
      chain_link_ns<false, true>(ns, a0, a1, lane, pq, shr, scl, vre, vim, zx, zy);
  }
}

template <int NS>
__device__ __forceinline__ void tree_lane_step(const TreeLaneRec *rec, int lane, int nl, float2 *pq,
                                               const float2 *shr, int2 *scl) {
  if (lane >= nl) return;
  const uint4 *r = (const uint4 *)(rec + lane);
  tree_lane_exec<NS>(r[0], NS == 4 ? r[1] : make_uint4(0u, 0u, 0u, 0u), pq, shr, scl);
}

// DEV: the program may hold kind 3 steps (per-query subtrees; a shared
// subtree never does, and its launch leaves that code out)
// A kind 3 step (operands in the query's device workspace), whatever its
// kind field says (a kind 6 pair runs as two of these when a wave holds more
// than one query).
template <class SP>
__device__ __forceinline__ void tree_kind3(SP Sp, int lane, int nthr, int nqw, float2 *pq, int perq,
                                           const float2 *shr, int2 *scl, int nscale, float2 *gq,
                                           int64_t gstride) {
  if (nqw == 1 && Sp->pow2) {
    switch (Sp->glob) {  // 1 .. 7 (checked on the host)
      case 1: tree_dev_one<1>(Sp, lane, nthr, pq, shr, scl, gq); break;
      case 2: tree_dev_one<2>(Sp, lane, nthr, pq, shr, scl, gq); break;
      case 3: tree_dev_one<3>(Sp, lane, nthr, pq, shr, scl, gq); break;
      case 4: tree_dev_one<4>(Sp, lane, nthr, pq, shr, scl, gq); break;
      case 5: tree_dev_one<5>(Sp, lane, nthr, pq, shr, scl, gq); break;
      case 6: tree_dev_one<6>(Sp, lane, nthr, pq, shr, scl, gq); break;
      default: tree_dev_one<7>(Sp, lane, nthr, pq, shr, scl, gq); break;
    }
  } else if (Sp->pow2) {
    tree_dev_impl<true>(Sp, lane, nthr, nqw, pq, perq, shr, scl, nscale, gq, gstride);
  } else {
    tree_dev_impl<false>(Sp, lane, nthr, nqw, pq, perq, shr, scl, nscale, gq, gstride);
  }
  // a later step of this wave reads what this one stored to device memory
  __builtin_amdgcn_s_waitcnt(0);
}

// Kind 6 (batch kernel, one query per wave): a kind 3 pair in one step.  P
// writes an intermediate T to the query's device workspace and Q contracts T
// with an operand B that has no free legs, so each entry of T enters exactly
// one of Q's products (checked on the host, which also moved Q up to P).
// Each lane computes the entries of T its own results need (result co = lane
// + 64 j takes T at ao(co) + oa(s) for its ns terms s), keeps them in
// registers, takes the wave-wide max |re|/|im| for T's scale record, and
// finishes Q: T never goes through device memory.  T's entries, its scale
// and Q's results come from the same operations in the same order as when
// the two steps run apart, so the results are bit-identical.  Q: nc <= 256,
// ns <= 4; P: ns <= 64; both power-of-two maps.
__device__ __forceinline__ void tree_pair(CStep P, CStep Q, int lane, float2 *pq, const float2 *shr,
                                          int2 *scl) {
  int32_t pcext[kTreeSeg], pca[kTreeSeg], pcb[kTreeSeg], pclg[kTreeSeg];
  int32_t psext[kTreeSeg], psa[kTreeSeg], psb[kTreeSeg], pslg[kTreeSeg];
  int32_t qcext[kTreeSeg], qca[kTreeSeg], qcb[kTreeSeg], qclg[kTreeSeg];
  int32_t qsext[kTreeSeg], qsa[kTreeSeg], qsb[kTreeSeg], qslg[kTreeSeg];
#pragma unroll
  for (int i = 0; i < kTreeSeg; ++i) {
    pcext[i] = P->cext[i];
    pca[i] = P->ca[i];
    pcb[i] = P->cb[i];
    pclg[i] = P->clg[i];
    psext[i] = P->sext[i];
    psa[i] = P->sa[i];
    psb[i] = P->sb[i];
    pslg[i] = P->slg[i];
    qcext[i] = Q->cext[i];
    qca[i] = Q->ca[i];
    qcb[i] = Q->cb[i];
    qclg[i] = Q->clg[i];
    qsext[i] = Q->sext[i];
    qsa[i] = Q->sa[i];
    qsb[i] = Q->sb[i];
    qslg[i] = Q->slg[i];
  }
  const int hl = threadIdx.x & 63;
  const int pns = P->ns, pnss = P->nss, pncs = P->ncs;
  const int qns = Q->ns, qnss = Q->nss, qncs = Q->ncs, qnc = Q->nc;
  // shared-index offsets, lane l holding those of term l (as in the kinds 0
  // and 3 forms): P's of X and Y, Q's of T and B
  int psoa = 0, psob = 0, qsoa = 0, qsob = 0;
  if (hl < pns) seg2r<true>(psext, psa, psb, pslg, pnss, hl, psoa, psob);
  if (hl < qns) seg2r<true>(qsext, qsa, qsb, qslg, qnss, hl, qsoa, qsob);
  // T's entry ao(co) + oa(s) has the bits of ao(co) and of oa(s) apart (a
  // bijection of power-of-two maps), and P's map of T's index is linear over
  // disjoint bits: P's offsets of the entry are those of ao(co) plus those of
  // oa(s), the latter held by lane s
  int pxs = 0, pys = 0;
  if (hl < qns) seg2r<true>(pcext, pca, pcb, pclg, pncs, qsoa, pxs, pys);
  const int pa = P->a, pb = P->b, qb = Q->b;
  const float2 *X0 = (pa & kPerQuery) ? pq + (pa & ~kPerQuery) : shr + pa;
  const float2 *Y0 = (pb & kPerQuery) ? pq + (pb & ~kPerQuery) : shr + pb;
  const float2 *B0 = (qb & kPerQuery) ? pq + (qb & ~kPerQuery) : shr + qb;
  float2 *C = pq + (Q->c & ~kPerQuery);
  const ItemScale zp = uniform_scale(scl, P->asl, P->bsl);
  const int ep = zp.e();
  const float fp = ldexpf(1.0f, -ep);
  // T's entries of this lane's results
  float2 tv[4][4];
  int bo[4];
  float mt = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int co = lane + 64 * j;
    bo[j] = 0;
#pragma unroll
    for (int sh = 0; sh < 4; ++sh) tv[j][sh] = make_float2(0.f, 0.f);
    if (co < qnc) {
      int ao, b_, xb, yb;
      seg2r<true>(qcext, qca, qcb, qclg, qncs, co, ao, b_);
      seg2r<true>(pcext, pca, pcb, pclg, pncs, ao, xb, yb);
      bo[j] = b_;
#pragma unroll
      for (int sh = 0; sh < 4; ++sh)
        if (sh < qns) {
          const int xo = xb + __builtin_amdgcn_readlane(pxs, sh), yo = yb + __builtin_amdgcn_readlane(pys, sh);
          const float2 r =
              dot_terms<true>(X0 + xo, Y0 + yo, pns, true, psoa, psob, psext, psa, psb, pslg, pnss);
          tv[j][sh] = make_float2(r.x * fp, r.y * fp);
          mt = fmaxf(mt, fmaxf(fabsf(tv[j][sh].x), fabsf(tv[j][sh].y)));
        }
    }
  }
  // T's scale record as P leaves it (max bits: non-negative floats order as
  // their bit patterns), and Q's operand scales
  const unsigned tbits = wave_max_u32(__float_as_uint(mt));
  const int tlog = zp.za.x + zp.zb.x + ep;
  int2 zb = Q->bsl >= 0 ? scl[Q->bsl] : make_int2(0, 0);
  zb.x = __builtin_amdgcn_readfirstlane(zb.x);
  zb.y = __builtin_amdgcn_readfirstlane(zb.y);
  const int eq = tn_scale_exp(tbits) + tn_scale_exp((uint32_t)zb.y);
  const float fq = ldexpf(1.0f, -eq);
  float mx = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int co = lane + 64 * j;
    if (co < qnc) {
      // the order of dot_terms: four terms at a time, the even ones into
      // (re0, im0) and the odd ones into (re1, im1), then the rest into
      // (re0, im0)
      float re0 = 0.f, im0 = 0.f, re1 = 0.f, im1 = 0.f;
      if (qns == 4) {
        float2 y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] = B0[bo[j] + __builtin_amdgcn_readlane(qsob, u)];
#pragma unroll
        for (int u = 0; u < 4; u += 2) {
          const float2 x0 = tv[j][u], x1 = tv[j][u + 1];
          re0 = fmaf(x0.x, y[u].x, re0);
          re0 = fmaf(-x0.y, y[u].y, re0);
          im0 = fmaf(x0.x, y[u].y, im0);
          im0 = fmaf(x0.y, y[u].x, im0);
          re1 = fmaf(x1.x, y[u + 1].x, re1);
          re1 = fmaf(-x1.y, y[u + 1].y, re1);
          im1 = fmaf(x1.x, y[u + 1].y, im1);
          im1 = fmaf(x1.y, y[u + 1].x, im1);
        }
      } else {
#pragma unroll
        for (int u = 0; u < 3; ++u)
          if (u < qns) {
            const float2 x = tv[j][u], y = B0[bo[j] + __builtin_amdgcn_readlane(qsob, u)];
            re0 = fmaf(x.x, y.x, re0);
            re0 = fmaf(-x.y, y.y, re0);
            im0 = fmaf(x.x, y.y, im0);
            im0 = fmaf(x.y, y.x, im0);
          }
      }
      const float rr = (re0 + re1) * fq, ii = (im0 + im1) * fq;
      C[co] = make_float2(rr, ii);
      mx = fmaxf(mx, fmaxf(fabsf(rr), fabsf(ii)));
    }
  }
  if (lane == 0) scl[Q->csl].x = tlog + zb.x + eq;
  atomicMax((unsigned int *)&scl[Q->csl].y, __float_as_uint(mx));
}

template <bool DEV, class SP>
__device__ __forceinline__ void tree_step(SP Sp, int lane, int nthr, int nqw, float2 *pq, int perq,
                                          const float2 *shr, int2 *scl, int nscale, float2 *gq,
                                          int64_t gstride, const TreeLaneRec *lanes, int lane0) {
  if (Sp->kind == 4) {
    // lanes: the launch's records (lane0 = 0) or the program's copy in LDS
    // (lane0 = its first record's index)
    const TreeLaneRec *rec = lanes + (Sp->tab - lane0);
    if (Sp->ns == 1)
      tree_lane_step<1>(rec, lane, Sp->nc, pq, shr, scl);
    else if (Sp->ns == 2)
      tree_lane_step<2>(rec, lane, Sp->nc, pq, shr, scl);
    else
      tree_lane_step<4>(rec, lane, Sp->nc, pq, shr, scl);
    return;
  }
  if (DEV && Sp->kind == 3) {
    tree_kind3(Sp, lane, nthr, nqw, pq, perq, shr, scl, nscale, gq, gstride);
    return;
  }
  if (nqw == 1)
    tree_step_q<true>(Sp, lane, nthr, 1, pq, perq, shr, scl, nscale);
  else
    tree_step_q<false>(Sp, lane, nthr, nqw, pq, perq, shr, scl, nscale);
}

// Closed root of one query: the FP64 inner product and its result record
// (mantissa pair normalised to [0.5, 1) in the larger part, exponent in log2s).
__device__ __forceinline__ void tree_write_result(Result *r, double vr, double vi, int2 za, int2 zb) {
  double log2s = (double)(za.x + zb.x);
  const double m = fmax(fabs(vr), fabs(vi));
  if (m > 0.0 && isfinite(m)) {
    int e;
    frexp(m, &e);
    vr = ldexp(vr, -e);
    vi = ldexp(vi, -e);
    log2s += (double)e;
  }
  r->re = vr;
  r->im = vi;
  r->log2s = log2s;
  r->pad = 0.0;
}

// Query q's closed root: its Result record, or (dres set) the value itself,
// the record's mantissas scaled by 2^log2s exactly as a reader of the record
// would.
__device__ __forceinline__ void tree_emit_result(const TreeLaunch &t, int q, double vr, double vi,
                                                 int2 za, int2 zb) {
  if (t.dres == nullptr) {
    tree_write_result(t.res + q, vr, vi, za, zb);
    return;
  }
  Result r;
  tree_write_result(&r, vr, vi, za, zb);
  const int e = (int)r.log2s;
  t.dres[(int64_t)q * t.dres_stride] = make_double2(ldexp(r.re, e), ldexp(r.im, e));
}

// The leaves into LDS, by the whole workgroup: the shared leaves from the
// image, the shared intermediates through the gather list, their scale
// records into every query's table, the per-query scale records cleared and
// the overridden leaves copied per query.  Loads are issued in groups of four
// per thread before any of them is stored, so each part costs about one
// round trip.  The caller places a barrier after it.
__device__ __forceinline__ void tree_prologue(const TreeLaunch &t, KernargLaunch ka, const TreeHdr &h,
                                              int tid, int qw, int nqw, int q0, int2 *scl,
                                              float2 *shr, float2 *pq, int perq) {
  // the shared intermediates' records (indices below nsloads) are written
  // below, every other record starts at zero
  for (int i = tid; i < qw * h.nscale; i += 256) {
    const int r = i % h.nscale;
    if (r >= h.nsloads) scl[i] = make_int2(0, 0);
  }
  const float2 *img = t.image + h.image_off;
  for (int i0 = 0; i0 < h.nimg; i0 += 1024) {
    float2 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = i0 + tid + 256 * j;
      if (i < h.nimg) v[j] = img[i];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = i0 + tid + 256 * j;
      if (i < h.nimg) shr[i] = v[j];
    }
  }
  const float2 *sbase = (const float2 *)t.shared_base;
  for (int e0 = 0; e0 < h.nsg; e0 += 1024) {
    int2 g[4];
    float2 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = e0 + tid + 256 * j;
      g[j] = e < h.nsg ? t.sgather[h.sg0 + e] : make_int2(-1, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (g[j].x >= 0) v[j] = sbase[g[j].y];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (g[j].x >= 0) shr[g[j].x] = v[j];
  }
  for (int e = tid; e < h.nsloads * nqw; e += 256) {
    const int k = e / nqw, q = e - k * nqw;
    const int slot = t.sloads[h.sload0 + k].slot;
    const Slot z = t.slots_sh[slot];
    scl[q * h.nscale + k] = make_int2((int)z.log2s, (int)z.maxbits);
  }
  for (int w = tid; w < h.nloads * nqw; w += 256) {
    const int li = w / nqw, q = w - li * nqw;
    const TreeLeafLoad L = t.loads[h.load0 + li];
    const float2 *op = ka->ovr[L.src].p;
    const int64_t ostride = ka->ovr[L.src].stride;
    const float2 *src = op + (int64_t)(q0 + q) * ostride;
    float2 *dst = pq + q * perq + (L.lds & ~kPerQuery);
    for (int i = 0; i < L.n; ++i) dst[i] = src[i];
  }
}

template <bool DEV>
__global__ __launch_bounds__(256) void k_tree(TreeLaunch t) {
  constexpr int W = kTreeStepWords;
  constexpr int CW = kTreeChunk * W;
  constexpr int PRE = (CW + 255) / 256;
  const int tid = threadIdx.x;
  const TreeHdr h = t.hdr[blockIdx.x];
  const int qw = t.qw;
  const int q0 = blockIdx.y * qw;
  const int nqw = min(qw, t.nq - q0);
  // the override table is indexed at run time: read it from the kernel
  // argument segment rather than from a private copy of the argument
  KernargLaunch ka = (KernargLaunch)__builtin_amdgcn_kernarg_segment_ptr();

  // LDS: [2 chunk buffers][reduction: 256 double2][scales: qw * nscale int2]
  //      [shared region][qw per-query regions]
  int32_t *sbuf = (int32_t *)tree_lds;
  double2 *red = (double2 *)(tree_lds + 2 * CW * 4);
  int2 *scl = (int2 *)(red + 256);
  float2 *shr = (float2 *)(scl + ((qw * h.nscale + 1) & ~1));
  float2 *pq = shr + ((h.shared_elems + 1) & ~1);
  const int perq = (h.perq_elems + 1) & ~1;
  const int32_t *gw = (const int32_t *)t.steps;
  // the queries' device workspaces (large per-query intermediates)
  float2 *gq = (float2 *)(t.perq_base + (int64_t)q0 * t.perq_stride);
  const int64_t gstride = t.perq_stride / 8;

  tree_prologue(t, ka, h, tid, qw, nqw, q0, scl, shr, pq, perq);
  // the program's kind 4 lane records: copied after the query regions
  // (16-byte aligned; the host sized the LDS for it) or read from device memory
  const TreeLaneRec *lrec = t.lanes;
  int lrec0 = 0;
  if (h.rec_lds) {
    const size_t off = ((size_t)((const unsigned char *)(pq + qw * perq) - tree_lds) + 15) & ~(size_t)15;
    uint4 *dst = (uint4 *)(tree_lds + off);
    const uint4 *src = (const uint4 *)(t.lanes + h.rec0);
    for (int i = tid; i < 2 * h.nrec; i += 256) dst[i] = src[i];
    lrec = (const TreeLaneRec *)dst;
    lrec0 = h.rec0;
  }
  // the chunks' steps are consecutive from step0: the next chunk's size is
  // fetched one chunk ahead, so no chunk waits on the chunk table
  // A program of at most 2 kTreeChunk steps is copied whole into the two
  // chunk buffers here, and no level waits on device memory for its steps.
  const bool whole = h.nsteps <= 2 * kTreeChunk;
  // (its chunk sizes too, one per lane of every wave: nchunks <= nsteps <= 32)
  const int csz = whole && (tid & 63) < h.nchunks ? t.chunks[h.chunk0 + (tid & 63)].nsteps : 0;
  int cur = 0, nxt = 0, s_cur = h.step0;
  if (h.nchunks > 0) {
    cur = t.chunks[h.chunk0].nsteps;
    if (h.nchunks > 1) nxt = t.chunks[h.chunk0 + 1].nsteps;
    const int n = (whole ? h.nsteps : cur) * W;
    for (int i = tid; i < n; i += 256) sbuf[i] = gw[(int64_t)s_cur * W + i];
  }
  __syncthreads();

  for (int k = 0; k < h.nchunks; ++k) {
    const TreeStep *S = (const TreeStep *)(sbuf + (whole ? (s_cur - h.step0) * W : (k & 1) * CW));
    int32_t pre[PRE];
    int nxt2 = 0;
    if (k + 1 < h.nchunks && whole) {
      if (k + 2 < h.nchunks) nxt2 = __builtin_amdgcn_readlane(csz, k + 2);
    } else if (k + 1 < h.nchunks) {
      const int64_t s_nxt = s_cur + cur;
#pragma unroll
      for (int j = 0; j < PRE; ++j) {
        const int i = tid + 256 * j;
        pre[j] = i < nxt * W ? gw[s_nxt * W + i] : 0;
      }
      if (k + 2 < h.nchunks) nxt2 = t.chunks[h.chunk0 + k + 2].nsteps;
    }
    if (S[0].kind == 1) {
      // closed root: FP64 inner product over ns entries for every query
      const TreeStep &st = S[0];
      const bool p2 = st.pow2 != 0;
      int32_t ext[kTreeSeg], s0[kTreeSeg], s1[kTreeSeg], lg[kTreeSeg];
#pragma unroll
      for (int i = 0; i < kTreeSeg; ++i) {
        ext[i] = st.sext[i];
        s0[i] = st.sa[i];
        s1[i] = st.sb[i];
        lg[i] = st.slg[i];
      }
      for (int q = 0; q < nqw; ++q) {
        float2 *base = pq + q * perq;
        const float2 *A = (st.a & kPerQuery) ? base + (st.a & ~kPerQuery) : shr + st.a;
        const float2 *B = (st.b & kPerQuery) ? base + (st.b & ~kPerQuery) : shr + st.b;
        double re = 0.0, im = 0.0;
        for (int s = tid; s < st.ns; s += 256) {
          int sa, sb;
          if (p2)
            seg2r<true>(ext, s0, s1, lg, st.nss, s, sa, sb);
          else
            seg2r<false>(ext, s0, s1, lg, st.nss, s, sa, sb);
          const float2 x = A[sa], y = B[sb];
          re += (double)x.x * y.x - (double)x.y * y.y;
          im += (double)x.x * y.y + (double)x.y * y.x;
        }
        red[tid] = make_double2(re, im);
        __syncthreads();
        for (int r = 128; r > 0; r >>= 1) {
          if (tid < r) {
            red[tid].x += red[tid + r].x;
            red[tid].y += red[tid + r].y;
          }
          __syncthreads();
        }
        if (tid == 0) {
          const int2 *sc = scl + q * h.nscale;
          const int2 za = st.asl >= 0 ? sc[st.asl] : make_int2(0, 0);
          const int2 zb = st.bsl >= 0 ? sc[st.bsl] : make_int2(0, 0);
          tree_emit_result(t, q0 + q, red[0].x, red[0].y, za, zb);
        }
        __syncthreads();
      }
    } else if (cur == 1) {
      // one step (a spine contraction): the whole workgroup on it
      tree_step<DEV>(S, tid, 256, nqw, pq, perq, shr, scl, h.nscale, gq, gstride, lrec, lrec0);
    } else {
      // several independent steps of one level (largest first): one wave per
      // step, round robin
      const int wave = tid >> 6, lane = tid & 63;
      for (int i = wave; i < cur; i += 4)
        tree_step<DEV>(S + i, lane, 64, nqw, pq, perq, shr, scl, h.nscale, gq, gstride, lrec, lrec0);
    }
    if (k + 1 < h.nchunks && !whole) {
      int32_t *dst = sbuf + ((k + 1) & 1) * CW;
#pragma unroll
      for (int j = 0; j < PRE; ++j) {
        const int i = tid + 256 * j;
        if (i < nxt * W) dst[i] = pre[j];
      }
    }
    s_cur += cur;
    cur = nxt;
    nxt = nxt2;
    __syncthreads();
  }

  // the subtree's result and its scale record to device memory
  if (!h.final_dot) {
    const int rl = h.root_loc & ~kPerQuery;
    for (int w = tid; w < nqw * h.root_elems; w += 256) {
      const int q = w / h.root_elems, i = w - q * h.root_elems;
      uint8_t *part = h.root_in_perq ? t.perq_base + (int64_t)(q0 + q) * t.perq_stride : t.shared_base;
      ((float2 *)(part + h.root_off))[i] = pq[q * perq + rl + i];
    }
    if (tid < nqw) {
      const int q = tid;
      const int2 z = scl[q * h.nscale + h.root_scale];
      Slot *s = h.root_in_perq ? t.slots_q + (int64_t)(q0 + q) * t.slot_stride + h.root_slot
                               : t.slots_sh + h.root_slot;
      s->log2s = (double)z.x;
      s->maxbits = (uint32_t)z.y;
      s->pad = 0u;
    }
  }
}

__global__ __launch_bounds__(256) void k_tree_wave(TreeLaunch t) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const TreeHdr *hp = t.hdr + blockIdx.x;
  const int qw = t.qw;
  const int qpw = (qw + 3) >> 2;
  const int q0 = blockIdx.y * qw;
  const int nqw = min(qw, t.nq - q0);
  KernargLaunch ka = (KernargLaunch)__builtin_amdgcn_kernarg_segment_ptr();

  int nscale, nsteps, step0, final_dot;
  int2 *scl;
  float2 *shr, *pq;
  int perq;
  {
    const TreeHdr h = *hp;
    nscale = h.nscale;
    nsteps = h.wnsteps;  // this kernel's form of the program (with kind 5 chains)
    step0 = h.wstep0;
    final_dot = h.final_dot;
    // LDS: [scales: qw * nscale int2][shared region][qw per-query regions]
    scl = (int2 *)tree_lds;
    shr = (float2 *)(scl + ((qw * h.nscale + 1) & ~1));
    pq = shr + ((h.shared_elems + 1) & ~1);
    perq = (h.perq_elems + 1) & ~1;
    tree_prologue(t, ka, h, tid, qw, nqw, q0, scl, shr, pq, perq);
  }
  __syncthreads();

  // this wave's queries: [wq0, wq0 + wn) of the workgroup's
  const int wq0 = wave * qpw;
  const int wn = min(qpw, nqw - wq0);
  if (wn <= 0) return;
  float2 *wpq = pq + wq0 * perq;
  int2 *wscl = scl + wq0 * nscale;
  const CStep prog = (CStep)t.steps + step0;
  // a closed root is the program's last step (checked on the host): it runs
  // after the loop
  const int nloop = nsteps - (final_dot ? 1 : 0);
  float2 *wgq = (float2 *)(t.perq_base + (int64_t)(q0 + wq0) * t.perq_stride);
  const int64_t gstride = t.perq_stride / 8;
  // a kind 4 step's lane record is loaded one step ahead, so that its
  // latency overlaps the step before
  uint4 n0 = make_uint4(0u, 0u, 0u, 0u), n1 = n0;
  auto fetch = [&](int k) {
    const CStep S = prog + k;
    if (S->kind == 5) {  // link 0 of a chain (64 records a link)
      const uint4 *r = (const uint4 *)(t.lanes + S->tab + lane);
      n0 = r[0];
      n1 = r[1];
    } else if (S->kind == 4 && lane < S->nc) {
      const uint4 *r = (const uint4 *)(t.lanes + S->tab + lane);
      n0 = r[0];
      if (S->ns == 4) n1 = r[1];
    }
  };
  if (nloop > 0) fetch(0);
  for (int k = 0; k < nloop; ++k) {
    const CStep S = prog + k;
    const uint4 c0 = n0, c1 = n1;
    if (k + 1 < nloop) fetch(k + 1);
    if (S->kind == 5) {
      tree_chain(t.lanes + S->tab, S->nc, c0, c1, lane, wpq, shr, wscl);
    } else if (S->kind == 6) {
      // a kind 3 pair: this step and the next
      if (wn == 1) {
        tree_pair(S, S + 1, lane, wpq, shr, wscl);
      } else {
        tree_kind3(S, lane, 64, wn, wpq, perq, shr, wscl, nscale, wgq, gstride);
        tree_kind3(S + 1, lane, 64, wn, wpq, perq, shr, wscl, nscale, wgq, gstride);
      }
      ++k;
      if (k + 1 < nloop) fetch(k + 1);
    } else if (S->kind == 4) {
      if (S->nss) {  // one whole step: the whole wave, one scale store
        const bool act = lane < S->nc;
        if (S->ns == 1)
          tree_lane_whole<1>(c0, c1, act, lane, wpq, shr, wscl);
        else if (S->ns == 2)
          tree_lane_whole<2>(c0, c1, act, lane, wpq, shr, wscl);
        else
          tree_lane_whole<4>(c0, c1, act, lane, wpq, shr, wscl);
      } else if (lane < S->nc) {
        if (S->ns == 1)
          tree_lane_exec<1>(c0, c1, wpq, shr, wscl);
        else if (S->ns == 2)
          tree_lane_exec<2>(c0, c1, wpq, shr, wscl);
        else
          tree_lane_exec<4>(c0, c1, wpq, shr, wscl);
      }
    } else {
      tree_step<true>(S, lane, 64, wn, wpq, perq, shr, wscl, nscale, wgq, gstride, t.lanes, 0);
    }
  }

  if (final_dot) {
    // closed root: FP64 inner product, reduced across the wave
    const CStep S = prog + nloop;
    const bool p2 = S->pow2 != 0;
    const int ns = S->ns, nss = S->nss, a = S->a, b = S->b;
    int32_t ext[kTreeSeg], s0[kTreeSeg], s1[kTreeSeg], lg[kTreeSeg];
#pragma unroll
    for (int i = 0; i < kTreeSeg; ++i) {
      ext[i] = S->sext[i];
      s0[i] = S->sa[i];
      s1[i] = S->sb[i];
      lg[i] = S->slg[i];
    }
    for (int q = 0; q < wn; ++q) {
      float2 *base = wpq + q * perq;
      const float2 *A = (a & kPerQuery) ? base + (a & ~kPerQuery) : shr + a;
      const float2 *B = (b & kPerQuery) ? base + (b & ~kPerQuery) : shr + b;
      double re = 0.0, im = 0.0;
      for (int s = lane; s < ns; s += 64) {
        int sa, sb;
        if (p2)
          seg2r<true>(ext, s0, s1, lg, nss, s, sa, sb);
        else
          seg2r<false>(ext, s0, s1, lg, nss, s, sa, sb);
        const float2 x = A[sa], y = B[sb];
        re += (double)x.x * y.x - (double)x.y * y.y;
        im += (double)x.x * y.y + (double)x.y * y.x;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
      }
      if (lane == 0) {
        const int2 *sc = wscl + q * nscale;
        const int2 za = S->asl >= 0 ? sc[S->asl] : make_int2(0, 0);
        const int2 zb = S->bsl >= 0 ? sc[S->bsl] : make_int2(0, 0);
        tree_emit_result(t, q0 + wq0 + q, re, im, za, zb);
      }
    }
    return;
  }
  // the subtree's result and its scale record to device memory (the header
  // fields read again here rather than kept through the loop)
  const volatile TreeHdr *vh = hp;
  const int root_elems = vh->root_elems, rl = vh->root_loc & ~kPerQuery, in_perq = vh->root_in_perq;
  const int64_t root_off = vh->root_off;
  const int root_scale = vh->root_scale, root_slot = vh->root_slot;
  for (int w = lane; w < wn * root_elems; w += 64) {
    const int q = w / root_elems, i = w - q * root_elems;
    uint8_t *part = in_perq ? t.perq_base + (int64_t)(q0 + wq0 + q) * t.perq_stride : t.shared_base;
    ((float2 *)(part + root_off))[i] = wpq[q * perq + rl + i];
  }
  if (lane < wn) {
    const int q = lane;
    const int2 z = wscl[q * nscale + root_scale];
    Slot *sl = in_perq ? t.slots_q + (int64_t)(q0 + wq0 + q) * t.slot_stride + root_slot
                       : t.slots_sh + root_slot;
    sl->log2s = (double)z.x;
    sl->maxbits = (uint32_t)z.y;
    sl->pad = 0u;
  }
}

// LDS a workgroup may use: the device's per-block limit (160 KiB on gfx950),
// raised for both subtree kernels once.
size_t tree_lds_limit() {
  static size_t limit = 0;
  if (limit == 0) {
    int dev = 0, v = 0;
    size_t l = 65536;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      l = (size_t)v;
    if (l > 163840) l = 163840;
    if (l > 65536 &&
        (hipFuncSetAttribute((const void *)k_tree<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)l) != hipSuccess ||
         hipFuncSetAttribute((const void *)k_tree<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)l) != hipSuccess ||
         hipFuncSetAttribute((const void *)k_tree_wave, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)l) != hipSuccess))
      l = 65536;
    limit = l;
  }
  return limit;
}

hipError_t launch_tree(hipStream_t st, const TreeLaunch &t, int nsub, size_t lds_bytes, bool dev) {
  if (nsub <= 0 || t.nq <= 0) return hipSuccess;
  if (lds_bytes > tree_lds_limit()) return hipErrorInvalidValue;
  const int groups = (t.nq + t.qw - 1) / t.qw;
  if (dev)
    hipLaunchKernelGGL(k_tree<true>, dim3(nsub, groups), dim3(256), lds_bytes, st, t);
  else
    hipLaunchKernelGGL(k_tree<false>, dim3(nsub, groups), dim3(256), lds_bytes, st, t);
  return hipGetLastError();
}

hipError_t launch_tree_wave(hipStream_t st, const TreeLaunch &t, int nsub, size_t lds_bytes) {
  if (nsub <= 0 || t.nq <= 0) return hipSuccess;
  if (lds_bytes > tree_lds_limit() || t.qw < 1 || t.qw > 16) return hipErrorInvalidValue;
  const int groups = (t.nq + t.qw - 1) / t.qw;
  hipLaunchKernelGGL(k_tree_wave, dim3(nsub, groups), dim3(256), lds_bytes, st, t);
  return hipGetLastError();
}

}  // namespace tn
