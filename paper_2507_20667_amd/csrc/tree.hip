// Subtree kernel: a whole subtree of small contractions in one workgroup.
//
// The many small contractions near the leaves of a circuit network (gate
// tensors of 2-16 entries meeting intermediates of up to a few thousand
// entries) would each be a launch of their own.  Here one workgroup takes one
// subtree for `qw` queries at once: it copies the subtree's leaves into LDS (a
// shared copy of the leaves no query overrides, a per-query copy of the
// overridden ones, read in place from the caller's buffers), then runs the
// subtree level by level: the contractions of one level are independent, so
// up to kTreeChunk of them share one barrier, with every operand and result in
// LDS.  Finally it writes the subtree's result and its scale record to device
// memory, or, when the subtree ends in the network's closed root, the FP64
// inner product.
//
// The descriptors of the next chunk are fetched into registers while the
// current chunk computes and stored to the second LDS buffer before the
// barrier.  Scales: every intermediate keeps a running integer log2 scale and
// the IEEE bits of its max |re|/|im|; a consumer multiplies its operands by
// 2^-e (e = floor(log2 max)), exactly as the one-contraction kernels do.
#include "tn_device.h"

namespace tn {

extern __shared__ __align__(16) unsigned char tree_lds[];

typedef const TreeLaunch __attribute__((address_space(4))) *KernargLaunch;

__device__ __forceinline__ int tree_exp(uint32_t bits) {
  if (bits == 0u) return 0;
  const int e = (int)((bits >> 23) & 0xffu);
  if (e == 0xff) return 0;
  if (e == 0) return -126;
  return e - 127;
}

__device__ __forceinline__ void seg2(const int32_t *ext, const int32_t *s0, const int32_t *s1,
                                     const int32_t *lg, int nseg, bool p2, int idx, int &o0,
                                     int &o1) {
  o0 = 0;
  o1 = 0;
  if (p2) {
    for (int i = 0; i < nseg; ++i) {
      const int v = idx & (ext[i] - 1);
      idx >>= lg[i];
      o0 += v * s0[i];
      o1 += v * s1[i];
    }
  } else {
    for (int i = 0; i < nseg; ++i) {
      const int v = idx % ext[i];
      idx /= ext[i];
      o0 += v * s0[i];
      o1 += v * s1[i];
    }
  }
}

// Decode with the map held in registers (unrolled over kTreeSeg); P2: every
// extent a power of two (shifts and masks instead of divisions).
template <bool P2>
__device__ __forceinline__ void seg2r(const int32_t (&ext)[kTreeSeg], const int32_t (&s0)[kTreeSeg],
                                      const int32_t (&s1)[kTreeSeg], const int32_t (&lg)[kTreeSeg],
                                      int nseg, int idx, int &o0, int &o1) {
  o0 = 0;
  o1 = 0;
#pragma unroll
  for (int i = 0; i < kTreeSeg; ++i) {
    if (i < nseg) {
      int v;
      if (P2) {
        v = idx & (ext[i] - 1);
        idx >>= lg[i];
      } else {
        v = idx % ext[i];
        idx /= ext[i];
      }
      o0 += v * s0[i];
      o1 += v * s1[i];
    }
  }
}

template <bool P2>
__device__ __forceinline__ void tree_step_impl(const TreeStep *Sp, int lane, int nthr, int nqw,
                                               float2 *pq, int perq, const float2 *shr, int2 *scl,
                                               int nscale);

template <bool P2, int NS, int NFY>
__device__ __forceinline__ void tree_stream_impl(const TreeStep *Sp, int lane, int nthr, int nqw,
                                                 float2 *pq, int perq, const float2 *shr,
                                                 int2 *scl, int nscale);

// One contraction for every query of the group, by `nthr` threads starting at
// `lane`.  The step's maps live in registers; each thread keeps the running
// max of its results per query and folds it into the scale record once per
// query.
__device__ __forceinline__ void tree_step(const TreeStep *Sp, int lane, int nthr, int nqw,
                                          float2 *pq, int perq, const float2 *shr, int2 *scl,
                                          int nscale) {
  if (Sp->kind == 2) {
    // a small operand along the fibers of a large one: ns, nfy in {1, 2, 4}
    const int sel = (Sp->ns >> 1) * 3 + (Sp->nss >> 1) + (Sp->pow2 ? 0 : 9);
#define TN_TS(P, A, B) tree_stream_impl<P, A, B>(Sp, lane, nthr, nqw, pq, perq, shr, scl, nscale)
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
    tree_step_impl<true>(Sp, lane, nthr, nqw, pq, perq, shr, scl, nscale);
  else
    tree_step_impl<false>(Sp, lane, nthr, nqw, pq, perq, shr, scl, nscale);
}

// Kind 2: one thread per fiber of the large operand X (and query) reads the
// fiber's ns entries once and writes nfy results; the small operand Y sits in
// registers, reloaded when a thread moves to another query.
template <bool P2, int NS, int NFY>
__device__ __forceinline__ void tree_stream_impl(const TreeStep *Sp, int lane, int nthr, int nqw,
                                                 float2 *pq, int perq, const float2 *shr,
                                                 int2 *scl, int nscale) {
  const int a = Sp->a, b = Sp->b, c = Sp->c;
  const int asl = Sp->asl, bsl = Sp->bsl, csl = Sp->csl;
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
  int qprev = -1;
  float mx = 0.f, f = 1.f;
  const float2 *X = nullptr;
  float2 *C = nullptr;
  int2 *sc = nullptr;
  float2 y[NS * NFY];
  for (int w = lane; w < nqw * nfib; w += nthr) {
    const int q = P2 ? (w >> lgf) : w / nfib;
    const int fi = w - q * nfib;
    if (q != qprev) {
      if (qprev >= 0) atomicMax((unsigned int *)&sc[csl].y, __float_as_uint(mx));
      qprev = q;
      mx = 0.f;
      float2 *base = pq + q * perq;
      X = (a & kPerQuery) ? base + (a & ~kPerQuery) : shr + a;
      const float2 *Y = (b & kPerQuery) ? base + (b & ~kPerQuery) : shr + b;
      C = base + (c & ~kPerQuery);
      sc = scl + q * nscale;
      const int2 za = asl >= 0 ? sc[asl] : make_int2(0, 0);
      const int2 zb = bsl >= 0 ? sc[bsl] : make_int2(0, 0);
      const int ea = tree_exp((uint32_t)za.y), eb = tree_exp((uint32_t)zb.y);
      f = ldexpf(1.0f, -(ea + eb));
      if (fi == 0) sc[csl].x = za.x + zb.x + ea + eb;
#pragma unroll
      for (int v = 0; v < NS * NFY; ++v) y[v] = Y[ym[v]];
    }
    int xo, co;
    seg2r<P2>(fext, fx, fc, flg, ncs, fi, xo, co);
    float2 x[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) x[s] = X[xo + xs[s]];
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
      C[co + cy[j]] = make_float2(re, im);
      mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
    }
  }
  if (qprev >= 0) atomicMax((unsigned int *)&sc[csl].y, __float_as_uint(mx));
}

template <bool P2>
__device__ __forceinline__ void tree_step_impl(const TreeStep *Sp, int lane, int nthr, int nqw,
                                               float2 *pq, int perq, const float2 *shr, int2 *scl,
                                               int nscale) {
  const int a = Sp->a, b = Sp->b, c = Sp->c;
  const int asl = Sp->asl, bsl = Sp->bsl, csl = Sp->csl;
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
  int qprev = -1;
  float mx = 0.f, f = 1.f;
  const float2 *A = nullptr, *B = nullptr;
  float2 *C = nullptr;
  int2 *sc = nullptr;
  for (int w = lane; w < nqw * nc; w += nthr) {
    const int q = P2 ? (w >> lgnc) : w / nc;
    const int ci = w - q * nc;
    if (q != qprev) {
      if (qprev >= 0) atomicMax((unsigned int *)&sc[csl].y, __float_as_uint(mx));
      qprev = q;
      mx = 0.f;
      float2 *base = pq + q * perq;
      A = (a & kPerQuery) ? base + (a & ~kPerQuery) : shr + a;
      B = (b & kPerQuery) ? base + (b & ~kPerQuery) : shr + b;
      C = base + (c & ~kPerQuery);
      sc = scl + q * nscale;
      const int2 za = asl >= 0 ? sc[asl] : make_int2(0, 0);
      const int2 zb = bsl >= 0 ? sc[bsl] : make_int2(0, 0);
      const int ea = tree_exp((uint32_t)za.y), eb = tree_exp((uint32_t)zb.y);
      f = ldexpf(1.0f, -(ea + eb));
      if (ci == 0) sc[csl].x = za.x + zb.x + ea + eb;
    }
    int ao, bo;
    seg2r<P2>(cext, ca, cb, clg, ncs, ci, ao, bo);
    float re = 0.f, im = 0.f;
    if (stab) {
      for (int s = 0; s < ns; ++s) {
        const int oa = __builtin_amdgcn_readlane(soa, s), ob = __builtin_amdgcn_readlane(sob, s);
        const float2 x = A[ao + oa], y = B[bo + ob];
        re = fmaf(x.x, y.x, re);
        re = fmaf(-x.y, y.y, re);
        im = fmaf(x.x, y.y, im);
        im = fmaf(x.y, y.x, im);
      }
    } else {
      for (int s = 0; s < ns; ++s) {
        int oa, ob;
        seg2r<P2>(sext, sa, sb, slg, nss, s, oa, ob);
        const float2 x = A[ao + oa], y = B[bo + ob];
        re = fmaf(x.x, y.x, re);
        re = fmaf(-x.y, y.y, re);
        im = fmaf(x.x, y.y, im);
        im = fmaf(x.y, y.x, im);
      }
    }
    re *= f;
    im *= f;
    C[ci] = make_float2(re, im);
    mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
  }
  if (qprev >= 0) atomicMax((unsigned int *)&sc[csl].y, __float_as_uint(mx));
}

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

  for (int i = tid; i < qw * h.nscale; i += 256) scl[i] = make_int2(0, 0);
  // shared leaves from the image; shared intermediates (computed by the shared
  // launch before this one) from the shared part, after them
  const int nimg = h.nsloads ? t.sloads[h.sload0].lds : h.shared_elems;
  for (int i = tid; i < nimg; i += 256) shr[i] = t.image[h.image_off + i];
  if (h.nsloads) {
    __syncthreads();  // the scale records are cleared
    for (int k = 0; k < h.nsloads; ++k) {
      const TreeSharedLoad S = t.sloads[h.sload0 + k];
      const float2 *src = (const float2 *)(t.shared_base + S.off);
      for (int i = tid; i < S.n; i += 256) shr[S.lds + i] = src[i];
      if (tid < nqw) {
        const Slot &z = t.slots_sh[S.slot];
        scl[tid * h.nscale + S.scale] = make_int2((int)z.log2s, (int)z.maxbits);
      }
    }
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
  int cur = 0;
  if (h.nchunks > 0) {
    const TreeChunk c0 = t.chunks[h.chunk0];
    cur = c0.nsteps;
    for (int i = tid; i < c0.nsteps * W; i += 256) sbuf[i] = gw[(int64_t)c0.step0 * W + i];
  }
  __syncthreads();

  for (int k = 0; k < h.nchunks; ++k) {
    const TreeStep *S = (const TreeStep *)(sbuf + (k & 1) * CW);
    int nxt = 0;
    int32_t pre[PRE];
    if (k + 1 < h.nchunks) {
      const TreeChunk cn = t.chunks[h.chunk0 + k + 1];
      nxt = cn.nsteps;
#pragma unroll
      for (int j = 0; j < PRE; ++j) {
        const int i = tid + 256 * j;
        pre[j] = i < nxt * W ? gw[(int64_t)cn.step0 * W + i] : 0;
      }
    }
    if (S[0].kind == 1) {
      // closed root: FP64 inner product over ns entries for every query
      const TreeStep &st = S[0];
      const bool p2 = st.pow2 != 0;
      for (int q = 0; q < nqw; ++q) {
        float2 *base = pq + q * perq;
        const float2 *A = (st.a & kPerQuery) ? base + (st.a & ~kPerQuery) : shr + st.a;
        const float2 *B = (st.b & kPerQuery) ? base + (st.b & ~kPerQuery) : shr + st.b;
        double re = 0.0, im = 0.0;
        for (int s = tid; s < st.ns; s += 256) {
          int sa, sb;
          seg2(st.sext, st.sa, st.sb, st.slg, st.nss, p2, s, sa, sb);
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
          double vr = red[0].x, vi = red[0].y;
          double log2s = (double)(za.x + zb.x);
          const double m = fmax(fabs(vr), fabs(vi));
          if (m > 0.0 && isfinite(m)) {
            int e;
            frexp(m, &e);
            vr = ldexp(vr, -e);
            vi = ldexp(vi, -e);
            log2s += (double)e;
          }
          Result *r = t.res + (q0 + q);
          r->re = vr;
          r->im = vi;
          r->log2s = log2s;
          r->pad = 0.0;
        }
        __syncthreads();
      }
    } else if (cur == 1) {
      // one step (a spine contraction): the whole workgroup on it
      tree_step(S, tid, 256, nqw, pq, perq, shr, scl, h.nscale);
    } else {
      // several independent steps of one level (largest first): one wave per
      // step, round robin
      const int wave = tid >> 6, lane = tid & 63;
      for (int i = wave; i < cur; i += 4) tree_step(S + i, lane, 64, nqw, pq, perq, shr, scl, h.nscale);
    }
    if (k + 1 < h.nchunks) {
      int32_t *dst = sbuf + ((k + 1) & 1) * CW;
#pragma unroll
      for (int j = 0; j < PRE; ++j) {
        const int i = tid + 256 * j;
        if (i < nxt * W) dst[i] = pre[j];
      }
    }
    cur = nxt;
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

// LDS a workgroup may use: the device's per-block limit (160 KiB on gfx950),
// raised for k_tree once.
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
        hipFuncSetAttribute((const void *)k_tree, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)l) != hipSuccess)
      l = 65536;
    limit = l;
  }
  return limit;
}

hipError_t launch_tree(hipStream_t st, const TreeLaunch &t, int nsub, size_t lds_bytes) {
  if (nsub <= 0 || t.nq <= 0) return hipSuccess;
  if (lds_bytes > tree_lds_limit()) return hipErrorInvalidValue;
  const int groups = (t.nq + t.qw - 1) / t.qw;
  hipLaunchKernelGGL(k_tree, dim3(nsub, groups), dim3(256), lds_bytes, st, t);
  return hipGetLastError();
}

}  // namespace tn
