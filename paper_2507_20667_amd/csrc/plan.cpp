// Plan loading: validation of the network, partitioning and tree (Sections
// 2.1-2.4), derived legs and vertex congestion, the cost integers of
// Section 3, the TTGT schedule of every contraction and the arena layout.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <map>
#include <set>
#include <unordered_map>

#include "tn_internal.h"

namespace tn {

static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char *last_error() { return g_err; }

static const int64_t kMaxElems = (int64_t)1 << 40;

static bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
static int ilog2(int64_t x) {
  int r = 0;
  while ((int64_t)1 << r < x) ++r;
  return r;
}

// ------------------------------------------------------------ index maps

// Segments of an index space given as a list of legs (outermost first), each
// leg with its extent and its strides into two tensors.  Adjacent legs fuse
// when both strides continue the inner leg's run.
struct LegMap {
  int64_t ext, s0, s1;
};

static bool fill_segmap(const std::vector<LegMap> &legs_outer_first, SegMap &m) {
  std::vector<LegMap> segs;  // innermost first
  for (int i = (int)legs_outer_first.size() - 1; i >= 0; --i) {
    const LegMap &l = legs_outer_first[i];
    if (l.ext == 1) continue;
    if (!segs.empty()) {
      LegMap &in = segs.back();
      if (l.s0 == in.s0 * in.ext && l.s1 == in.s1 * in.ext) {
        in.ext *= l.ext;
        continue;
      }
    }
    segs.push_back(l);
  }
  if ((int)segs.size() > kMaxSeg) return false;
  memset(&m, 0, sizeof(m));
  m.nseg = (int)segs.size();
  m.pow2 = 1;
  for (int i = 0; i < m.nseg; ++i) {
    m.ext[i] = segs[i].ext;
    m.s0[i] = segs[i].s0;
    m.s1[i] = segs[i].s1;
    if (!is_pow2(segs[i].ext)) m.pow2 = 0;
    m.lg[i] = ilog2(segs[i].ext);
  }
  return true;
}

// Permutation src -> dst (same leg set, dst order).
static bool make_perm(const Layout &src, const Layout &dst, PermDesc &h) {
  memset(&h, 0, sizeof(h));
  h.nelem = src.size();
  std::vector<int64_t> ss = src.strides(), ds = dst.strides();
  std::vector<LegMap> legs;
  for (int i = 0; i < dst.rank(); ++i) {
    int j = src.find(dst.lab[i]);
    legs.push_back({dst.dim[i], ss[j], ds[i]});
  }
  if (!fill_segmap(legs, h.map)) return false;
  // bit form when every extent is a power of two
  bool p2 = true;
  int bits = 0;
  for (int64_t d : src.dim) {
    if (!is_pow2(d)) p2 = false;
    bits += ilog2(d);
  }
  if (p2 && bits > 0 && bits <= 47) {
    // bit offset of each leg's least significant bit
    h.bits = bits;
    for (int i = 0; i < dst.rank(); ++i) {
      int j = src.find(dst.lab[i]);
      int k = ilog2(dst.dim[i]);
      int pd = ilog2(ds[i]), ps = ilog2(ss[j]);
      for (int t = 0; t < k; ++t) h.inbit[pd + t] = ps + t;
    }
  }
  return true;
}

static bool same_order(const Layout &a, const Layout &b) { return a.lab == b.lab; }

// ------------------------------------------------------------- blob helpers
template <typename T>
static size_t blob_put(std::vector<uint8_t> &blob, const T &v) {
  size_t off = (blob.size() + 255) & ~(size_t)255;
  blob.resize(off + sizeof(T));
  memcpy(blob.data() + off, &v, sizeof(T));
  return off;
}

// --------------------------------------------------------------- schedule

static tn_status schedule_stream(tn_plan *p, Node &n, const Layout &X, const Layout &Y, int xid,
                                 int yid) {
  n.kind = NK_STREAM;
  n.x = xid;
  n.y = yid;
  std::vector<int64_t> S, FY;
  for (int i = 0; i < Y.rank(); ++i) {
    if (X.find(Y.lab[i]) >= 0)
      S.push_back(Y.lab[i]);
    else
      FY.push_back(Y.lab[i]);
  }
  // C = X's legs with the shared legs removed and Y's free legs (Y order)
  // inserted where X's first shared leg was.
  Layout C;
  bool inserted = false;
  for (int i = 0; i < X.rank(); ++i) {
    bool shared = std::find(S.begin(), S.end(), X.lab[i]) != S.end();
    if (shared) {
      if (!inserted) {
        for (int64_t l : FY) {
          C.lab.push_back(l);
          C.dim.push_back(Y.dim[Y.find(l)]);
        }
        inserted = true;
      }
      continue;
    }
    C.lab.push_back(X.lab[i]);
    C.dim.push_back(X.dim[i]);
  }
  if (!inserted)
    for (int64_t l : FY) {
      C.lab.push_back(l);
      C.dim.push_back(Y.dim[Y.find(l)]);
    }
  n.out = C;
  std::vector<int64_t> xs = X.strides(), ys = Y.strides(), cs = C.strides();
  StreamDesc d;
  memset(&d, 0, sizeof(d));
  std::vector<LegMap> fib;
  int64_t nfib = 1;
  for (int i = 0; i < X.rank(); ++i) {
    if (std::find(S.begin(), S.end(), X.lab[i]) != S.end()) continue;
    fib.push_back({X.dim[i], xs[i], cs[C.find(X.lab[i])]});
    nfib *= X.dim[i];
  }
  if (!fill_segmap(fib, d.fib)) {
    set_error("tensor with too many index segments");
    return TN_E_INVALID_PLAN;
  }
  // enumerate S (Y order) and FY (Y order) row-major
  int64_t ns = 1, nfy = 1;
  for (int64_t l : S) ns *= Y.dim[Y.find(l)];
  for (int64_t l : FY) nfy *= Y.dim[Y.find(l)];
  d.nfib = nfib;
  d.ns = (int)ns;
  d.nfy = (int)nfy;
  for (int64_t s = 0; s < ns; ++s) {
    int64_t rem = s, xo = 0, yo = 0;
    for (int i = (int)S.size() - 1; i >= 0; --i) {
      int yi = Y.find(S[i]);
      int64_t v = rem % Y.dim[yi];
      rem /= Y.dim[yi];
      xo += v * xs[X.find(S[i])];
      yo += v * ys[yi];
    }
    d.xs[s] = xo;
    for (int64_t j = 0; j < nfy; ++j) {
      int64_t r2 = j, yo2 = 0;
      for (int i = (int)FY.size() - 1; i >= 0; --i) {
        int yi = Y.find(FY[i]);
        int64_t v = r2 % Y.dim[yi];
        r2 /= Y.dim[yi];
        yo2 += v * ys[yi];
      }
      d.ymap[s * nfy + j] = (int32_t)(yo + yo2);
    }
  }
  for (int64_t j = 0; j < nfy; ++j) {
    int64_t rem = j, co = 0;
    for (int i = (int)FY.size() - 1; i >= 0; --i) {
      int yi = Y.find(FY[i]);
      int64_t v = rem % Y.dim[yi];
      rem /= Y.dim[yi];
      co += v * cs[C.find(FY[i])];
    }
    d.cy[j] = co;
  }
  n.nfib = nfib;
  n.ns = (int)ns;
  n.nfy = (int)nfy;
  n.sdesc_off = blob_put(p->desc_blob, d);
  return TN_OK;
}

// S block at the end / start of a layout (any internal order).
static bool block_at_end(const Layout &L, const std::set<int64_t> &S) {
  int r = L.rank(), s = (int)S.size();
  for (int i = r - s; i < r; ++i)
    if (!S.count(L.lab[i])) return false;
  return true;
}
static bool block_at_start(const Layout &L, const std::set<int64_t> &S) {
  int s = (int)S.size();
  for (int i = 0; i < s; ++i)
    if (!S.count(L.lab[i])) return false;
  return true;
}

static std::vector<int64_t> select(const Layout &L, const std::set<int64_t> &S, bool in) {
  std::vector<int64_t> out;
  for (int64_t l : L.lab)
    if ((S.count(l) > 0) == in) out.push_back(l);
  return out;
}

static Layout make_layout(const std::vector<int64_t> &labs, const Layout &a, const Layout &b) {
  Layout L;
  for (int64_t l : labs) {
    int i = a.find(l);
    L.lab.push_back(l);
    L.dim.push_back(i >= 0 ? a.dim[i] : b.dim[b.find(l)]);
  }
  return L;
}

// FP32 plane GEMMs fused with a GEMM child (see Node::fuse_a, fo): the
// child's result index m N + n (its layout, row-major) maps to the k-tiled
// plane index of this GEMM's operand bit by bit when every dimension is a
// power of two.  Bits of a leg keep their order; the operand's row-major
// index o = r kdim + k becomes ((k / 16) rows + r) 16 + k % 16.  Fusion needs
// the four lowest bits to map to themselves, so that 16 consecutive results
// of a tile row land in 64 consecutive bytes of each plane.
static bool fuse_bits(const Layout &X, const Layout &D, int64_t rows, int64_t kdim, uint8_t *d, int &nbits) {
  auto lg = [](int64_t v) {
    int b = 0;
    while (((int64_t)1 << b) < v) ++b;
    return ((int64_t)1 << b) == v ? b : -1;
  };
  const int rb = lg(rows), kb = lg(kdim);
  if (rb < 0 || kb < 4 || X.rank() != D.rank()) return false;
  std::map<int64_t, int> spos, opos;
  int acc = 0;
  for (int i = X.rank() - 1; i >= 0; --i) {
    const int b = lg(X.dim[i]);
    if (b < 0) return false;
    spos[X.lab[i]] = acc;
    acc += b;
  }
  nbits = acc;
  if (acc > 48 || acc != rb + kb) return false;
  int oacc = 0;
  for (int i = D.rank() - 1; i >= 0; --i) {
    opos[D.lab[i]] = oacc;
    oacc += lg(D.dim[i]);
  }
  for (int i = 0; i < X.rank(); ++i) {
    const int64_t l = X.lab[i];
    if (!opos.count(l)) return false;
    for (int c = 0; c < lg(X.dim[i]); ++c) {
      const int ob = opos[l] + c;
      d[spos[l] + c] = (uint8_t)(ob < 4 ? ob : ob < kb ? ob + rb : ob - kb + 4);
    }
  }
  for (int b = 0; b < 4; ++b)
    if (d[b] != b) return false;
  return true;
}

// A GEMM whose result its parent may read as k-tiled planes written by this
// GEMM orders B's free legs [others..., contracted by the parent...] (the
// latter are the result's lowest bits, the parent's k).  The plane index of
// an entry has k % 16 in bits 0-3 and the parent operand's row in the bits
// above; when the result bits just above the lowest four are that row's
// lowest bits, a tile's 32 consecutive columns (a wave's store) land in 32
// consecutive plane entries instead of two runs of 16.  So move up to two
// bits' worth of free legs between the lowest four bits and the rest of the
// parent-contracted block: legs the parent keeps as its own lowest result
// bits (those the grandparent contracts, which the parent orders last), or
// any kept leg when the grandparent contracts none of them.  FB[0, npc) are
// the legs the parent keeps, FB[npc, end) those it contracts.
static void interleave_rows(std::vector<int64_t> &FB, int npc, const Layout &B, const Layout &A,
                            const std::set<int64_t> &pcon, const std::set<int64_t> &pcon2) {
  auto bits = [&](int64_t l) {
    const int64_t d = B.dim[B.find(l)];
    int b = 0;
    while (((int64_t)1 << b) < d) ++b;
    return ((int64_t)1 << b) == d ? b : -1;
  };
  // the parent-contracted legs that make the lowest four bits
  int low = (int)FB.size(), acc = 0;
  while (low > npc && acc < 4) {
    const int b = bits(FB[low - 1]);
    if (b < 0) return;
    acc += b;
    --low;
  }
  if (acc != 4 || low == npc) return;
  // does the grandparent contract any leg the parent keeps from this result?
  bool kept2 = false;
  for (int64_t l : A.lab)
    if (pcon.count(l) == 0 && pcon2.count(l)) kept2 = true;
  for (int i = 0; i < npc; ++i)
    if (pcon2.count(FB[i])) kept2 = true;
  std::vector<int64_t> rows;
  int rb = 0;
  for (int i = npc - 1; i >= 0 && rb < 2; --i) {
    const int b = bits(FB[i]);
    if (b < 1 || rb + b > 2 || (kept2 && !pcon2.count(FB[i]))) continue;
    rows.insert(rows.begin(), FB[i]);
    rb += b;
  }
  if (rows.empty()) return;
  std::vector<int64_t> out;
  for (int i = 0; i < npc; ++i)
    if (std::find(rows.begin(), rows.end(), FB[i]) == rows.end()) out.push_back(FB[i]);
  out.insert(out.end(), FB.begin() + npc, FB.begin() + low);
  out.insert(out.end(), rows.begin(), rows.end());
  out.insert(out.end(), FB.begin() + low, FB.end());
  FB = out;
}

static tn_status schedule_gemm(tn_plan *p, Node &n, const Layout &A, const Layout &B,
                               const std::set<int64_t> &pcon, const std::set<int64_t> &pcon2) {
  n.kind = NK_GEMM;
  n.ga = n.c1;
  n.gb = n.c2;
  std::set<int64_t> S;
  for (int64_t l : A.lab)
    if (B.find(l) >= 0) S.insert(l);
  std::vector<int64_t> FA = select(A, S, false), FB = select(B, S, false);
  std::vector<int64_t> sA = select(A, S, true), sB = select(B, S, true);
  // how each operand can enter the GEMM without a permutation
  int aMode = block_at_end(A, S) ? 0 : (block_at_start(A, S) ? 1 : -1);   // 0: N, 1: T
  int bMode = block_at_start(B, S) ? 0 : (block_at_end(B, S) ? 1 : -1);   // 0: N, 1: T
  std::vector<int64_t> sorder;
  bool permA = aMode < 0, permB = bMode < 0;
  // The split-BF16 GEMM, and the FP32 GEMM when k is a multiple of 16,
  // read both operands as planes that the permutation kernel writes (an
  // identity map where the order is right).
  int64_t k_all = 1;
  for (int64_t l : sA) k_all *= A.dim[A.find(l)];
  n.planes = 0;
  if (p->flags & TN_PREC_BF16X3)
    n.planes = (p->flags & TN_FORM_3M) ? 6 : 4;
  else if (k_all % 16 == 0)
    n.planes = 2;
  // a GEMM child whose result this GEMM may read as planes it writes itself
  // (both FP32, or both BF16x3 of one form; the child on k-tiled planes, not
  // split in k): the larger one
  const int nv = (int)p->leaf.size();
  const bool fuse_on = !getenv("TN_GEMM_FUSE") || atoi(getenv("TN_GEMM_FUSE")) != 0;
  const bool fuse_kind = n.planes > 0;
  auto fusable = [&](int c) {
    if (c < nv || !fuse_kind) return false;
    const Node &u = p->nodes[c - nv];
    return u.kind == NK_GEMM && u.planes == n.planes && u.ktile && u.ksplit == 1 && !u.fo;
  };
  int fx = 0;  // 1: A, 2: B
  if (fusable(n.c1)) fx = 1;
  if (fusable(n.c2) && (fx == 0 || B.size() > A.size())) fx = 2;
  if (n.planes > 0) {
    // k in the order of the fused operand, so that its child can write it
    sorder = fx == 2 ? sB : fx == 1 ? sA : (!permA || permB ? sA : sB);
    permA = permB = true;
    // the legs the parent contracts last among B's free legs: they are the
    // lowest bits of this GEMM's result, which the parent may read as its
    // k-tiled operand written by this GEMM
    if (fuse_kind && !pcon.empty()) {
      const auto mid = std::stable_partition(FB.begin(), FB.end(), [&](int64_t l) { return pcon.count(l) == 0; });
      interleave_rows(FB, (int)(mid - FB.begin()), B, A, pcon, pcon2);
    }
  } else if (!permA && !permB) {
    if (sA != sB) {
      if (A.size() <= B.size()) {
        permA = true;
        sorder = sB;
      } else {
        permB = true;
        sorder = sA;
      }
    } else {
      sorder = sA;
    }
  } else if (!permA) {
    sorder = sA;
  } else if (!permB) {
    sorder = sB;
  } else {
    sorder = sA;
  }
  n.M = n.N = n.K = 1;
  for (int64_t l : FA) n.M *= A.dim[A.find(l)];
  for (int64_t l : FB) n.N *= B.dim[B.find(l)];
  for (int64_t l : sorder) n.K *= A.dim[A.find(l)];
  if (permA) {
    std::vector<int64_t> lab = FA;
    lab.insert(lab.end(), sorder.begin(), sorder.end());
    n.pa.needed = true;
    n.pa.dst = make_layout(lab, A, B);
    if (!make_perm(A, n.pa.dst, n.pa.h)) {
      set_error("tensor with too many index segments");
      return TN_E_INVALID_PLAN;
    }
    n.pa.desc_off = blob_put(p->desc_blob, n.pa.h);
    n.opA = 0;
  } else {
    n.opA = aMode;
  }
  if (permB) {
    // a permuted B is written [FB, S] (N x K, k contiguous): both GEMM
    // operands then stream rows of consecutive k into the tile loaders
    std::vector<int64_t> lab = FB;
    lab.insert(lab.end(), sorder.begin(), sorder.end());
    n.pb.needed = true;
    n.pb.dst = make_layout(lab, A, B);
    if (!make_perm(B, n.pb.dst, n.pb.h)) {
      set_error("tensor with too many index segments");
      return TN_E_INVALID_PLAN;
    }
    n.pb.desc_off = blob_put(p->desc_blob, n.pb.h);
    n.opB = 1;
  } else {
    n.opB = bMode;
  }
  n.lda = n.opA == 0 ? n.K : n.M;
  n.ldb = n.opB == 0 ? n.N : n.K;
  n.ldc = n.N;
  std::vector<int64_t> out = FA;
  out.insert(out.end(), FB.begin(), FB.end());
  n.out = make_layout(out, A, B);
  n.variant = (n.M >= 128 && n.N >= 128) ? 0 : 1;
  // FP32 planes: a 64-row or 64-column tile when that side is that small
  // (a 128 x 128 tile would run half empty), unless the tuning table says
  // otherwise
  // BF16x3 4M: the two wave-group kernel's 256 x 128 (or 128 x 256) tile when
  // both sides fill it
  n.tile = 0;
  if (n.planes == 2) n.tile = n.M <= 64 && n.N > 64 ? 1 : n.N <= 64 && n.M > 64 ? 2 : 0;
  if (n.planes == 4) n.tile = n.M >= 256 && n.N >= 128 ? 2 : n.N >= 256 && n.M >= 128 ? 1 : 0;
  auto tile_m = [&](int tile) {
    return n.planes == 2 ? gemm_planes_tile_m(tile)
                         : n.planes > 0 ? gemm_bf16_tile_m(tile) : gemm_variant_tile_m(n.variant);
  };
  auto tile_n = [&](int tile) {
    return n.planes == 2 ? gemm_planes_tile_n(tile)
                         : n.planes > 0 ? gemm_bf16_tile_n(tile) : gemm_variant_tile_n(n.variant);
  };
  n.ksplit = gemm_ksplit(n.M, n.N, n.K, tile_m(n.tile), tile_n(n.tile), &n.kchunk);
  // the tuning table's choice for this shape, or TN_GEMM_FORCE="tile,ksplit"
  // (tuning runs): a tile shape for the FP32 planes or BF16x3 4M, k chunks
  // of a multiple of 32 entries
  {
    int tile = -1, ks = 0;
    if (const char *e = getenv("TN_GEMM_FORCE")) {
      if (sscanf(e, "%d,%d", &tile, &ks) != 2) tile = -1, ks = 0;
    } else if (n.planes > 0 && p->tuned) {
      if (const GemmRule *r = tune_gemm(n.planes > 2, (p->flags & TN_FORM_3M) != 0, n.M, n.N, n.K)) {
        tile = r->tile;
        ks = r->ksplit;
      }
    }
    if ((n.planes == 2 || n.planes == 4) && tile >= 0 && tile <= 2 && tile != n.tile) {
      n.tile = tile;
      if (ks < 1) n.ksplit = gemm_ksplit(n.M, n.N, n.K, tile_m(n.tile), tile_n(n.tile), &n.kchunk);
    }
    if (n.planes > 0 && ks >= 1) {
      int64_t kc = (n.K + ks - 1) / ks;
      kc = (kc + 31) / 32 * 32;
      n.kchunk = kc;
      n.ksplit = (int)((n.K + kc - 1) / kc);
    }
  }
  n.ktile = n.planes > 0 && n.K % 16 == 0 &&
            (n.ksplit == 1 || n.kchunk % 16 == 0);
  // fusion with the chosen child: its epilogue writes this GEMM's operand
  // planes (unscaled; this GEMM scales its result instead)
  if (fx && fuse_on && n.ktile) {
    const bool fa = fx == 1;
    const Layout &X = fa ? A : B;
    Node &u = p->nodes[(fa ? n.c1 : n.c2) - nv];
    uint8_t d[48];
    int nbits = 0;
    const Layout &D = fa ? n.pa.dst : n.pb.dst;
    // (both vertices too large for a subtree batch, which writes complex64;
    // at most 2^29 entries, so that 32-bit byte offsets from each plane's
    // base reach them)
    if (X.size() > kTreeMaxElems && X.size() <= ((int64_t)1 << 29) &&
        fuse_bits(X, D, fa ? n.M : n.N, n.K, d, nbits) && u.N >= 16 && u.M * u.N == X.size()) {
      u.fo = true;
      memcpy(u.fo_d, d, sizeof(d));
      // a BF16x3 4M producer on the two wave-group kernel where its shape
      // fills that tile: its 2-byte plane stores cost the one-group kernel a
      // third of its time on short k (the tuning table times GEMMs that
      // write complex64)
      if (u.planes == 4 && u.tile == 0 && u.ksplit == 1) {
        if (u.M >= 256 && u.N >= 128) u.tile = 2;
        else if (u.N >= 256 && u.M >= 128) u.tile = 1;
      }
      int nb = 0, mb = 0;
      while (((int64_t)1 << nb) < u.N) ++nb;
      while (((int64_t)1 << mb) < u.M) ++mb;
      u.fo_nbits = nb;
      u.fo_mbits = mb;
      u.fo_plane = X.size();
      // the operand as the planes kernel reads it: [rows][K], k-tiled
      if (fa) {
        n.fuse_a = true;
        n.pa.needed = false;
        n.opA = 0;
        n.lda = n.K;
        permA = false;
      } else {
        n.fuse_b = true;
        n.pb.needed = false;
        n.opB = 1;
        n.ldb = n.K;
        permB = false;
      }
    }
  }
  p->num_perm += (int)permA + (int)permB;
  return TN_OK;
}

static tn_status schedule_dot(tn_plan *p, Node &n, const Layout &A, const Layout &B) {
  n.kind = NK_DOT;
  n.out = Layout();
  DotDesc d;
  memset(&d, 0, sizeof(d));
  d.nelem = A.size();
  std::vector<int64_t> as = A.strides(), bs = B.strides();
  std::vector<LegMap> legs;
  for (int i = 0; i < A.rank(); ++i) legs.push_back({A.dim[i], as[i], bs[B.find(A.lab[i])]});
  if (!fill_segmap(legs, d.map)) {
    set_error("tensor with too many index segments");
    return TN_E_INVALID_PLAN;
  }
  n.nelem = d.nelem;
  n.dot_blocks = dot_blocks_for(d.nelem);
  n.ddesc_off = blob_put(p->desc_blob, d);
  return TN_OK;
}

// Largest offsets a segment map can produce (sum of (extent - 1) * stride).
static void seg_reach(const SegMap &m, int64_t &r0, int64_t &r1, int64_t &count) {
  r0 = r1 = 0;
  count = 1;
  for (int i = 0; i < m.nseg; ++i) {
    r0 += (m.ext[i] - 1) * m.s0[i];
    r1 += (m.ext[i] - 1) * m.s1[i];
    count *= m.ext[i];
  }
}

// Every kernel of a node must stay inside its operands: checked here on the
// host so that a scheduling mistake is a load error, never a device fault.
static bool node_in_bounds(const tn_plan *p, const Node &n, const std::vector<Layout> &lay) {
  const uint8_t *blob = p->desc_blob.data();
  int64_t r0, r1, cnt;
  if (n.kind == NK_STREAM) {
    const StreamDesc &d = *(const StreamDesc *)(blob + n.sdesc_off);
    seg_reach(d.fib, r0, r1, cnt);
    if (cnt != d.nfib || d.ns < 1 || d.nfy < 1 || d.ns * d.nfy > kStreamMax) return false;
    int64_t mx = 0, mc = 0;
    for (int s = 0; s < d.ns; ++s) mx = std::max(mx, d.xs[s]);
    for (int j = 0; j < d.nfy; ++j) mc = std::max(mc, d.cy[j]);
    for (int i = 0; i < d.ns * d.nfy; ++i)
      if (d.ymap[i] < 0 || d.ymap[i] >= lay[n.y].size()) return false;
    return r0 + mx < lay[n.x].size() && r1 + mc < std::max<int64_t>(n.out.size(), 1);
  }
  auto perm_ok = [&](const PermStep &ps, const Layout &src) {
    if (!ps.needed) return true;
    seg_reach(ps.h.map, r0, r1, cnt);
    if (ps.h.bits > 0 && ((int64_t)1 << ps.h.bits) != ps.h.nelem) return false;
    return cnt == ps.h.nelem && ps.h.nelem == src.size() && r0 < src.size() && r1 < ps.h.nelem;
  };
  if (n.kind == NK_GEMM) {
    if (!perm_ok(n.pa, lay[n.ga]) || !perm_ok(n.pb, lay[n.gb])) return false;
    const int64_t sa = lay[n.ga].size(), sb = lay[n.gb].size();
    const int64_t ea = n.opA == 0 ? (n.M - 1) * n.lda + n.K - 1 : (n.K - 1) * n.lda + n.M - 1;
    const int64_t eb = n.opB == 0 ? (n.K - 1) * n.ldb + n.N - 1 : (n.N - 1) * n.ldb + n.K - 1;
    const int64_t ec = (n.M - 1) * n.ldc + n.N - 1;
    // a result written as planes: every index bit to a distinct bit below
    // log2 of the result's size
    if (n.fo) {
      const int nb = n.fo_nbits + n.fo_mbits;
      if (nb > 29 || ((int64_t)1 << nb) != n.out.size() || n.fo_plane != n.out.size()) return false;
      int64_t seen = 0;
      for (int b = 0; b < nb; ++b) {
        if (n.fo_d[b] >= nb || ((seen >> n.fo_d[b]) & 1)) return false;
        seen |= (int64_t)1 << n.fo_d[b];
      }
    }
    return n.M * n.K == sa && n.K * n.N == sb && ea < sa && eb < sb && ec < n.out.size();
  }
  const DotDesc &d = *(const DotDesc *)(blob + n.ddesc_off);
  seg_reach(d.map, r0, r1, cnt);
  return cnt == d.nelem && d.nelem == lay[n.c1].size() && lay[n.c1].size() == lay[n.c2].size() &&
         r0 < lay[n.c1].size() && r1 < lay[n.c2].size();
}

static void select_trees(tn_plan *p, const std::vector<Layout> &lay);

// Bytes of a vertex's result buffer: complex64, or the parent's operand planes
// its epilogue writes (8 bytes an entry; the six BF16x3 3M planes 12)
static int64_t out_bytes_of(const Node &n) {
  return std::max<int64_t>(n.out.size(), 1) * (n.fo && n.planes == 6 ? 12 : 8);
}

static u128 mul_check(u128 a, u128 b, bool &ovf) {
  if (a != 0 && b > (~(u128)0) / a) ovf = true;
  return a * b;
}

tn_status build_plan(tn_plan *p, const tn_plan_desc *d) {
  if (!d || d->num_tensors < 1 || !d->rank || !d->data || !d->partition_of) {
    set_error("tn_plan_desc: num_tensors >= 1 and rank/data/partition_of pointers are required");
    return TN_E_INVALID_ARG;
  }
  if (d->data_dtype != TN_C64 && d->data_dtype != TN_C128) {
    set_error("tn_plan_desc: data_dtype must be TN_C64 or TN_C128");
    return TN_E_INVALID_ARG;
  }
  const int nv = d->num_tensors;
  p->nv = nv;
  int64_t total = 0;
  for (int v = 0; v < nv; ++v) {
    if (d->rank[v] < 0 || d->rank[v] > 64) {
      set_error("tensor %d: rank %d out of range [0, 64]", v, d->rank[v]);
      return TN_E_INVALID_PLAN;
    }
    total += d->rank[v];
  }
  if (total > 0 && (!d->legs || !d->leg_dims)) {
    set_error("tn_plan_desc: legs and leg_dims are required");
    return TN_E_INVALID_ARG;
  }
  // edges: a label on two slots of two tensors with equal dims, or on one slot
  struct LabInfo {
    int count = 0;
    int t0 = -1, t1 = -1;
    int64_t dim = 0;
    int64_t first = 0;
  };
  std::unordered_map<int64_t, LabInfo> labs;
  std::vector<int64_t> first_order;
  p->leaf.resize(nv);
  int64_t pos = 0;
  for (int v = 0; v < nv; ++v) {
    Layout &L = p->leaf[v];
    for (int a = 0; a < d->rank[v]; ++a, ++pos) {
      int64_t lab = d->legs[pos], dim = d->leg_dims[pos];
      if (dim < 1) {
        set_error("tensor %d leg %d: dimension %lld < 1", v, a, (long long)dim);
        return TN_E_INVALID_PLAN;
      }
      LabInfo &li = labs[lab];
      if (li.count == 0) {
        li.t0 = v;
        li.dim = dim;
        first_order.push_back(lab);
      } else if (li.count == 1) {
        if (li.t0 == v) {
          set_error("label %lld appears twice on tensor %d (self-loop)", (long long)lab, v);
          return TN_E_INVALID_PLAN;
        }
        if (li.dim != dim) {
          set_error("label %lld: dimensions %lld and %lld differ (n_{u,a} must equal n_{v,b})",
                    (long long)lab, (long long)li.dim, (long long)dim);
          return TN_E_INVALID_PLAN;
        }
        li.t1 = v;
      } else {
        set_error("label %lld appears on more than two slots (hyperedge)", (long long)lab);
        return TN_E_INVALID_PLAN;
      }
      li.count++;
      L.lab.push_back(lab);
      L.dim.push_back(dim);
    }
    if (L.size() > kMaxElems) {
      set_error("tensor %d has more than 2^40 elements", v);
      return TN_E_INVALID_PLAN;
    }
    if (!d->data[v]) {
      set_error("tensor %d: data pointer is NULL", v);
      return TN_E_INVALID_ARG;
    }
  }
  // open legs and their output order
  std::vector<int64_t> open;
  for (int64_t l : first_order)
    if (labs[l].count == 1) open.push_back(l);
  if (d->num_output_legs > 0) {
    if (!d->output_legs || d->num_output_legs != (int)open.size()) {
      set_error("output_legs must list each of the %d open labels exactly once", (int)open.size());
      return TN_E_INVALID_PLAN;
    }
    std::set<int64_t> seen;
    for (int i = 0; i < d->num_output_legs; ++i) {
      int64_t l = d->output_legs[i];
      auto it = labs.find(l);
      if (it == labs.end() || it->second.count != 1 || !seen.insert(l).second) {
        set_error("output_legs[%d] = %lld is not an open label (or repeats)", i, (long long)l);
        return TN_E_INVALID_PLAN;
      }
    }
    p->out_labels.assign(d->output_legs, d->output_legs + d->num_output_legs);
  } else {
    p->out_labels = open;
  }
  p->closed = p->out_labels.empty();

  // partitioning: cover, disjoint (one index per tensor), non-empty
  if (d->num_partitions < 1 || d->num_partitions > nv) {
    set_error("num_partitions %d out of range [1, %d]", d->num_partitions, nv);
    return TN_E_INVALID_PLAN;
  }
  p->K = d->num_partitions;
  p->partition_of.assign(d->partition_of, d->partition_of + nv);
  std::vector<int> count(p->K, 0);
  for (int v = 0; v < nv; ++v) {
    int k = p->partition_of[v];
    if (k < 0 || k >= p->K) {
      set_error("partition_of[%d] = %d out of range", v, k);
      return TN_E_INVALID_PLAN;
    }
    count[k]++;
  }
  for (int k = 0; k < p->K; ++k)
    if (!count[k]) {
      set_error("partition %d is empty (partitions must be non-empty)", k);
      return TN_E_INVALID_PLAN;
    }

  // tree: full binary, leaves in bijection with V, every vertex used once
  const int nn = 2 * nv - 1;
  if (nv > 1 && !d->tree) {
    set_error("tree is required for more than one tensor");
    return TN_E_INVALID_ARG;
  }
  p->tree.assign(d->tree ? d->tree : (const int32_t *)nullptr,
                 d->tree ? d->tree + 2 * (nv - 1) : (const int32_t *)nullptr);
  std::vector<int> parent(nn, -1);
  for (int j = 0; j < nv - 1; ++j) {
    int a = p->tree[2 * j], b = p->tree[2 * j + 1], v = nv + j;
    if (a < 0 || b < 0 || a >= v || b >= v || a == b) {
      set_error("tree pair %d = (%d, %d): children must be distinct earlier vertices", j, a, b);
      return TN_E_INVALID_PLAN;
    }
    if (parent[a] >= 0 || parent[b] >= 0) {
      set_error("tree pair %d: vertex %d already has a parent", j, parent[a] >= 0 ? a : b);
      return TN_E_INVALID_PLAN;
    }
    parent[a] = parent[b] = v;
  }
  p->root = nn - 1;
  // fingerprint (FNV-1a, 64 bits) of what a plan's launch choices depend
  // on: ranks, labels and dimensions, partition, tree, precision and form,
  // output legs; the key of the plan's tuning-table entry
  {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t x) {
      for (int b = 0; b < 8; ++b) {
        h ^= (uint64_t)((x >> (8 * b)) & 0xff);
        h *= 1099511628211ull;
      }
    };
    mix(nv);
    for (int v = 0; v < nv; ++v) {
      mix(p->leaf[v].rank());
      for (int i = 0; i < p->leaf[v].rank(); ++i) {
        mix(p->leaf[v].lab[i]);
        mix(p->leaf[v].dim[i]);
      }
      mix(p->partition_of[v]);
    }
    for (int32_t x : p->tree) mix(x);
    mix(p->flags & (TN_PREC_BF16X3 | TN_FORM_3M));
    for (int i = 0; i < d->num_output_legs; ++i) mix(d->output_legs ? d->output_legs[i] : 0);
    p->fingerprint = h;
  }
  // subtree kernel choices: built-in defaults, the tuning table's entry for
  // this plan, then the TN_TREE_* overrides (tuning runs)
  // (TN_TUNE_OFF, read at every load, sets the table aside: a comparison of
  // tuned and untuned plans in one process)
  p->tuned = !getenv("TN_TUNE_OFF");
  if (const TreeKnobs *k = p->tuned ? tune_tree(p->fingerprint) : nullptr) p->knobs = *k;
  if (const char *e = getenv("TN_TREE_QW")) p->knobs.qw = atoi(e);
  if (const char *e = getenv("TN_TREE_SPILL")) p->knobs.spill = std::max(1, atoi(e));
  if (const char *e = getenv("TN_TREE_PACK_NC")) p->knobs.pack_nc = std::max(1, atoi(e));
  // acceptance: partition of all leaves under each vertex
  std::vector<int> pk(nn), nleaf(nn);
  for (int v = 0; v < nv; ++v) {
    pk[v] = p->partition_of[v];
    nleaf[v] = 1;
  }
  for (int j = 0; j < nv - 1; ++j) {
    int a = p->tree[2 * j], b = p->tree[2 * j + 1], v = nv + j;
    pk[v] = (pk[a] >= 0 && pk[a] == pk[b]) ? pk[a] : -1;
    nleaf[v] = nleaf[a] + nleaf[b];
  }
  std::vector<int> proot(p->K, -1);
  for (int v = 0; v < nn; ++v)
    if (pk[v] >= 0 && nleaf[v] == count[pk[v]]) proot[pk[v]] = v;
  for (int k = 0; k < p->K; ++k)
    if (proot[k] < 0) {
      set_error("the tree does not accept the partitioning: no subtree has exactly the leaves "
                "of partition %d",
                k);
      return TN_E_INVALID_PLAN;
    }

  // legs, 2^vc, schedule
  std::vector<Layout> lay(nn);
  for (int v = 0; v < nv; ++v) lay[v] = p->leaf[v];
  std::vector<u128> w(nn, 0), sz(nn, 0);
  bool ovf = false;
  for (int v = 0; v < nv; ++v) {
    u128 s = 1;
    for (int64_t dd : lay[v].dim) s = mul_check(s, (u128)dd, ovf);
    sz[v] = s;
  }
  p->nodes.resize(nv - 1);
  u128 con_serial = 0, mem = 0;
  int64_t largest = 0;
  // every tensor's leg set (a vertex's: the symmetric difference of its
  // children's), known before the vertices are scheduled, so that a GEMM can
  // order its result's legs by what its parent contracts
  std::vector<std::vector<int64_t>> legset(nn);
  for (int v = 0; v < nv; ++v) {
    legset[v] = lay[v].lab;
    std::sort(legset[v].begin(), legset[v].end());
  }
  for (int j = 0; j < nv - 1; ++j) {
    const std::vector<int64_t> &a = legset[p->tree[2 * j]], &b = legset[p->tree[2 * j + 1]];
    std::set_symmetric_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(legset[nv + j]));
  }
  for (int j = 0; j < nv - 1; ++j) {
    Node &n = p->nodes[j];
    n.id = nv + j;
    n.c1 = p->tree[2 * j];
    n.c2 = p->tree[2 * j + 1];
    n.part = pk[n.id];
    const Layout &A = lay[n.c1], &B = lay[n.c2];
    // E(v) = union of the children's legs; legs(v) = symmetric difference
    u128 wv = 1, sv = 1;
    for (int i = 0; i < A.rank(); ++i) wv = mul_check(wv, (u128)A.dim[i], ovf);
    bool any_free_b = false, any_free_a = false;
    for (int i = 0; i < B.rank(); ++i) {
      if (A.find(B.lab[i]) < 0) {
        wv = mul_check(wv, (u128)B.dim[i], ovf);
        sv = mul_check(sv, (u128)B.dim[i], ovf);
        any_free_b = true;
      }
    }
    for (int i = 0; i < A.rank(); ++i)
      if (B.find(A.lab[i]) < 0) {
        sv = mul_check(sv, (u128)A.dim[i], ovf);
        any_free_a = true;
      }
    if (ovf) {
      set_error("cost integers overflow 128 bits");
      return TN_E_INVALID_PLAN;
    }
    if (sv > (u128)kMaxElems) {
      set_error("intermediate %d would have more than 2^40 elements", n.id);
      return TN_E_INVALID_PLAN;
    }
    n.weight = wv;
    w[n.id] = wv;
    sz[n.id] = sv;
    con_serial += wv;
    u128 m = sv + sz[n.c1] + sz[n.c2];
    if (m > mem) mem = m;
    if ((int64_t)sv > largest) largest = (int64_t)sv;
    n.tiny = sv <= 4096 && sz[n.c1] <= 4096 && sz[n.c2] <= 4096;
    tn_status st;
    if (!any_free_a && !any_free_b) {
      st = schedule_dot(p, n, A, B);
    } else if (std::min(A.size(), B.size()) <= kStreamMax) {
      bool a_big = A.size() >= B.size();
      st = a_big ? schedule_stream(p, n, A, B, n.c1, n.c2) : schedule_stream(p, n, B, A, n.c2, n.c1);
      p->num_stream++;
    } else {
      // the legs of this vertex its parent contracts, and the legs of the
      // parent's result that the grandparent contracts
      auto contracted = [&](int v, std::set<int64_t> &out) {
        const int pv = parent[v];
        if (pv < 0) return false;
        const int sib = p->tree[2 * (pv - nv)] == v ? p->tree[2 * (pv - nv) + 1] : p->tree[2 * (pv - nv)];
        std::set_intersection(legset[v].begin(), legset[v].end(), legset[sib].begin(), legset[sib].end(),
                              std::inserter(out, out.begin()));
        return true;
      };
      std::set<int64_t> pcon, pcon2;
      if (contracted(n.id, pcon)) contracted(parent[n.id], pcon2);
      st = schedule_gemm(p, n, A, B, pcon, pcon2);
      p->num_gemm++;
    }
    if (st) return st;
    if (n.tiny) p->num_tiny++;
    lay[n.id] = n.out;
    if (!node_in_bounds(p, n, lay)) {
      set_error("internal schedule error at vertex %d: an index map leaves its operand", n.id);
      return TN_E_INVALID_PLAN;
    }
  }
  p->con_serial = con_serial;
  p->mem = mem;
  p->largest = largest;
  // critical path
  std::vector<u128> best(nn, 0);
  for (int j = 0; j < nv - 1; ++j) {
    int a = p->tree[2 * j], b = p->tree[2 * j + 1], v = nv + j;
    best[v] = w[v] + std::max(best[a], best[b]);
  }
  p->con_par = nv > 1 ? best[nn - 1] : 0;
  // con_dist with con = con_serial, comm = 0
  u128 cd = 0;
  for (int k = 0; k < p->K; ++k) {
    u128 c = 0;
    for (int v = nv; v < nn; ++v)
      if (pk[v] == k) c += w[v];
    for (int u = parent[proot[k]]; u >= 0; u = parent[u]) c += w[u];
    cd = std::max(cd, c);
  }
  p->con_dist = cd;
  // execution order: partitions in turn, then the reduction path
  for (int k = 0; k < p->K; ++k)
    for (int j = 0; j < nv - 1; ++j)
      if (pk[nv + j] == k) p->order.push_back(j);
  for (int j = 0; j < nv - 1; ++j)
    if (pk[nv + j] < 0) p->order.push_back(j);

  // result layout and the final permutation into output-leg order
  const Layout &R = lay[p->root];
  p->result_layout = make_layout(p->out_labels, R, R);
  if (!p->closed && !same_order(R, p->result_layout)) {
    p->fperm.needed = true;
    p->fperm.dst = p->result_layout;
    if (!make_perm(R, p->fperm.dst, p->fperm.h)) {
      set_error("tensor with too many index segments");
      return TN_E_INVALID_PLAN;
    }
    p->fperm.desc_off = blob_put(p->desc_blob, p->fperm.h);
    int64_t r0, r1, cnt;
    seg_reach(p->fperm.h.map, r0, r1, cnt);
    if (cnt != R.size() || r0 >= R.size() || r1 >= R.size() ||
        (p->fperm.h.bits > 0 && ((int64_t)1 << p->fperm.h.bits) != R.size())) {
      set_error("internal schedule error in the output permutation");
      return TN_E_INVALID_PLAN;
    }
  }

  // leaves as complex64 (rounded once from complex128 input)
  p->leaf_off.resize(nv);
  int64_t off = 0;
  for (int v = 0; v < nv; ++v) {
    p->leaf_off[v] = off;
    off += (p->leaf[v].size() + 31) & ~(int64_t)31;  // 256-byte aligned leaves
  }
  p->leaf_host.assign(off, make_float2(0.f, 0.f));
  for (int v = 0; v < nv; ++v) {
    int64_t n = p->leaf[v].size();
    float2 *dst = p->leaf_host.data() + p->leaf_off[v];
    if (d->data_dtype == TN_C128) {
      const double *s = (const double *)d->data[v];
      for (int64_t i = 0; i < n; ++i) dst[i] = make_float2((float)s[2 * i], (float)s[2 * i + 1]);
    } else {
      memcpy(dst, d->data[v], sizeof(float2) * n);
    }
  }
  select_trees(p, lay);
  p->plain = make_exec_layout(p, {}, false, false);
  if (getenv("TN_DEBUG")) {
    for (const Node &n : p->nodes)
      if (n.kind == NK_GEMM) {
        // (writes: the run of result bits that map to themselves, 2^run
        // consecutive entries of a plane)
        int run = 0;
        while (n.fo && run < n.fo_nbits && n.fo_d[run] == run) ++run;
        fprintf(stderr, "[tn] gemm vertex %d: M %lld N %lld K %lld op %d%d perm %d%d variant %d tile %d ksplit %d planes %d fused %d%d writes %d (run %d)\n",
                n.id, (long long)n.M, (long long)n.N, (long long)n.K, n.opA, n.opB,
                (int)n.pa.needed, (int)n.pb.needed, n.variant, n.tile, n.ksplit, n.planes,
                (int)n.fuse_a, (int)n.fuse_b, (int)n.fo, run);
      }
    fprintf(stderr, "[tn] plan: %d vertices, %d gemm, %d stream, %d in subtrees (%zu roots)\n",
            nv - 1, p->num_gemm, p->num_stream,
            (int)std::count(p->in_tree.begin(), p->in_tree.end(), (char)1), p->tree_roots.size());
  }
  return TN_OK;
}

// ---------------------------------------------------------- memory layout

// Best-fit allocation over a growing range; records the high-water mark.
class Packer {
 public:
  explicit Packer(int64_t granule = 256) : g_(granule) {}
  int64_t alloc(int64_t bytes) {
    bytes = (bytes + g_ - 1) / g_ * g_;
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
    int64_t off;
    if (best != free_.end()) {
      off = best->first;
      int64_t rem = best->second - bytes;
      free_.erase(best);
      if (rem) free_[off + bytes] = rem;
    } else {
      // extend, merging a free block that ends at the top
      off = top_;
      if (!free_.empty()) {
        auto last = std::prev(free_.end());
        if (last->first + last->second == top_) {
          off = last->first;
          free_.erase(last);
        }
      }
      top_ = off + bytes;
    }
    peak_ = std::max(peak_, top_);
    return off;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = (bytes + g_ - 1) / g_ * g_;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t peak() const { return peak_; }

 private:
  int64_t g_;
  std::map<int64_t, int64_t> free_;
  int64_t top_ = 0, peak_ = 0;
};

// ------------------------------------------------------ subtree programs

static size_t tree_lds_bytes(int qw, int nscale, int shared_elems, int perq_elems, bool wave = false) {
  auto r2 = [](int64_t x) { return (x + 1) & ~(int64_t)1; };
  size_t b = 0;
  if (!wave) {
    b += (size_t)2 * kTreeChunk * kTreeStepWords * 4;  // two chunk buffers
    b += 256 * 16;                                      // FP64 reduction buffer
  }
  b += 8 * (size_t)r2((int64_t)qw * nscale);  // scale records
  b += 8 * (size_t)r2(shared_elems);
  b += 8 * (size_t)qw * (size_t)r2(perq_elems);
  return b;
}

static bool tree_fill(const std::vector<LegMap> &legs, int32_t *ext, int32_t *s0, int32_t *s1,
                      int32_t *lg, int32_t &nseg, bool &pow2) {
  SegMap m;
  if (!fill_segmap(legs, m) || m.nseg > kTreeSeg) return false;
  nseg = m.nseg;
  for (int i = 0; i < m.nseg; ++i) {
    ext[i] = (int32_t)m.ext[i];
    s0[i] = (int32_t)m.s0[i];
    s1[i] = (int32_t)m.s1[i];
    lg[i] = m.lg[i];
  }
  if (!m.pow2) pow2 = false;
  return true;
}

// Kind 2 step of vertex n: the small operand Y (<= 16 entries, ns and nfy in
// {1, 2, 4}) applied along the fibers of the large one X.  `swap`: Y is the
// first child (the caller then puts X's location in `a`).
static bool tree_stream_step(const Node &n, const std::vector<Layout> &lay, TreeStep &st,
                             bool &swap) {
  const Layout &L1 = lay[n.c1], &L2 = lay[n.c2];
  swap = L1.size() < L2.size();
  const Layout &X = swap ? L2 : L1, &Y = swap ? L1 : L2;
  if (Y.size() > 16 || n.out.rank() == 0) return false;
  const std::vector<int64_t> xst = X.strides(), yst = Y.strides(), ost = n.out.strides();
  std::vector<int> sh, yf;  // Y's legs: shared with X, free
  for (int i = 0; i < Y.rank(); ++i) (X.find(Y.lab[i]) >= 0 ? sh : yf).push_back(i);
  int64_t ns = 1, nfy = 1;
  for (int i : sh) ns *= Y.dim[i];
  for (int i : yf) nfy *= Y.dim[i];
  auto small = [](int64_t v) { return v == 1 || v == 2 || v == 4; };
  if (!small(ns) || !small(nfy)) return false;
  int64_t ys[4], yj[4];
  for (int64_t v = 0; v < ns; ++v) {  // shared index, last leg fastest
    int64_t r = v, xo = 0, yo = 0;
    for (int k = (int)sh.size() - 1; k >= 0; --k) {
      const int i = sh[k];
      const int64_t d = r % Y.dim[i];
      r /= Y.dim[i];
      yo += d * yst[i];
      xo += d * xst[X.find(Y.lab[i])];
    }
    st.xs[v] = (int32_t)xo;
    ys[v] = yo;
  }
  for (int64_t v = 0; v < nfy; ++v) {  // Y's free index
    int64_t r = v, yo = 0, co = 0;
    for (int k = (int)yf.size() - 1; k >= 0; --k) {
      const int i = yf[k];
      const int64_t d = r % Y.dim[i];
      r /= Y.dim[i];
      yo += d * yst[i];
      const int io = n.out.find(Y.lab[i]);
      if (io < 0) return false;
      co += d * ost[io];
    }
    st.cy[v] = (int32_t)co;
    yj[v] = yo;
  }
  for (int64_t a = 0; a < ns; ++a)
    for (int64_t b = 0; b < nfy; ++b) st.ymap[a * nfy + b] = (int32_t)(ys[a] + yj[b]);
  std::vector<LegMap> fl;  // X's free legs: fiber -> (X offset, C offset)
  int64_t nfib = 1;
  for (int i = 0; i < X.rank(); ++i) {
    if (Y.find(X.lab[i]) >= 0) continue;
    const int io = n.out.find(X.lab[i]);
    if (io < 0) return false;
    fl.push_back({X.dim[i], xst[i], ost[io]});
    nfib *= X.dim[i];
  }
  bool p2 = true;
  if (!tree_fill(fl, st.cext, st.ca, st.cb, st.clg, st.ncs, p2)) return false;
  if (nfib * nfy != n.out.size()) return false;
  st.nc = (int32_t)(nfib * nfy);
  st.ns = (int32_t)ns;
  st.nss = (int32_t)nfy;
  st.kind = 2;
  st.pow2 = p2 ? 1 : 0;
  return true;
}

// Step of vertex n: result index over n.out's legs, shared index over the
// shared legs (A's order); a closed root is a full inner product.
static bool tree_step(const tn_plan *p, const Node &n, const std::vector<Layout> &lay, bool final_dot,
                      TreeStep &st) {
  memset(&st, 0, sizeof(st));
  const Layout &A = lay[n.c1], &B = lay[n.c2];
  std::vector<int64_t> as = A.strides(), bs = B.strides();
  bool p2 = true;
  std::vector<LegMap> cl, sl;
  int64_t nc = 1, ns = 1;
  if (!final_dot) {
    for (int i = 0; i < n.out.rank(); ++i) {
      int ia = A.find(n.out.lab[i]), ib = B.find(n.out.lab[i]);
      cl.push_back({n.out.dim[i], ia >= 0 ? as[ia] : 0, ib >= 0 ? bs[ib] : 0});
      nc *= n.out.dim[i];
    }
  }
  for (int i = 0; i < A.rank(); ++i) {
    int ib = B.find(A.lab[i]);
    if (ib < 0) continue;
    sl.push_back({A.dim[i], as[i], bs[ib]});
    ns *= A.dim[i];
  }
  if (!tree_fill(cl, st.cext, st.ca, st.cb, st.clg, st.ncs, p2)) return false;
  if (!tree_fill(sl, st.sext, st.sa, st.sb, st.slg, st.nss, p2)) return false;
  st.nc = (int32_t)nc;
  st.ns = (int32_t)ns;
  st.kind = final_dot ? 1 : 0;
  st.pow2 = p2 ? 1 : 0;
  (void)p;
  return true;
}

// Level order of a subtree's vertices (level = 1 + the larger level of the
// children, leaves at 0), cut into chunks of at most kTreeChunk vertices of one
// level, and the LDS packing of their results in that order: a chunk's results
// are allocated before the operands it consumes are released.
struct LevelPlan {
  std::vector<std::vector<int>> chunks;
  std::map<int, int64_t> at;  // result offset (float2) of every vertex
  int64_t peak = 0;
};

static LevelPlan level_plan(const tn_plan *p, const std::vector<int> &nodes,
                            const std::vector<char> *spilled = nullptr) {
  const int nv = p->nv;
  auto in_lds = [&](int u) { return !spilled || !(*spilled)[u]; };
  std::map<int, int> lvl;
  for (int u : nodes) {  // nodes are in SSA order, children first
    const Node &n = p->nodes[u - nv];
    int l = 0;
    for (int c : {n.c1, n.c2})
      if (c >= nv && lvl.count(c)) l = std::max(l, lvl[c]);
    lvl[u] = l + 1;
  }
  // within a level, largest contraction first: the kernel deals a chunk's
  // steps to its waves round robin, so this evens out their shares
  std::vector<int> ord(nodes);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (lvl[a] != lvl[b]) return lvl[a] < lvl[b];
    return p->nodes[a - nv].weight > p->nodes[b - nv].weight;
  });
  LevelPlan lp;
  for (size_t i = 0; i < ord.size();) {
    std::vector<int> ch;
    const int l = lvl[ord[i]];
    while (i < ord.size() && lvl[ord[i]] == l && (int)ch.size() < kTreeChunk) ch.push_back(ord[i++]);
    lp.chunks.push_back(ch);
  }
  Packer P(2);
  for (const auto &ch : lp.chunks) {
    for (int u : ch)
      if (in_lds(u)) lp.at[u] = P.alloc(std::max<int64_t>(p->nodes[u - nv].out.size(), 1));
    for (int u : ch)
      for (int c : {p->nodes[u - nv].c1, p->nodes[u - nv].c2})
        if (c >= nv && lp.at.count(c))  // (inputs from outside the subtree live elsewhere)
          P.release(lp.at[c], std::max<int64_t>(p->nodes[c - nv].out.size(), 1));
  }
  lp.peak = P.peak();
  return lp;
}

// Subtrees of small vertices: a vertex qualifies when it, both operands and
// its result stay within kTreeMaxElems and both children are leaves or
// qualifying vertices; a subtree is kept when its worst-case LDS use (one
// query, every leaf copied) fits, otherwise its qualifying children are tried.
static void select_trees(tn_plan *p, const std::vector<Layout> &lay) {
  const int nv = p->nv, nn = 2 * nv - 1;
  p->in_tree.assign(nn, 0);
  p->tree_roots.clear();
  if (!p->use_tree || nv < 2) return;
  std::vector<char> ok(nn, 0);
  std::vector<int> parent(nn, -1);
  std::vector<TreeStep> tmp(1);
  for (int j = 0; j < nv - 1; ++j) {
    const Node &n = p->nodes[j];
    parent[n.c1] = parent[n.c2] = n.id;
    bool small = lay[n.c1].size() <= kTreeMaxElems && lay[n.c2].size() <= kTreeMaxElems &&
                 n.out.size() <= kTreeMaxElems;
    bool kids = (n.c1 < nv || ok[n.c1]) && (n.c2 < nv || ok[n.c2]);
    bool final_dot = n.kind == NK_DOT && n.id == p->root;
    bool dot_inside = n.kind == NK_DOT && !final_dot;
    ok[n.id] = small && kids && !dot_inside && tree_step(p, n, lay, final_dot, tmp[0]);
  }
  // worst-case LDS of the subtree at v
  auto lds_need = [&](int v) {
    std::vector<int> nodes, stack{v};
    int64_t leaf_elems = 0;
    while (!stack.empty()) {
      int u = stack.back();
      stack.pop_back();
      if (u < nv) {
        leaf_elems += (lay[u].size() + 1) & ~(int64_t)1;
        continue;
      }
      nodes.push_back(u);
      stack.push_back(p->nodes[u - nv].c1);
      stack.push_back(p->nodes[u - nv].c2);
    }
    std::sort(nodes.begin(), nodes.end());
    const LevelPlan lp = level_plan(p, nodes);
    return tree_lds_bytes(1, (int)nodes.size(), (int)leaf_elems, (int)lp.peak + 2);
  };
  std::vector<int> cand;
  for (int v = nv; v < nn; ++v)
    if (ok[v] && (parent[v] < 0 || !ok[parent[v]])) cand.push_back(v);
  std::vector<int> roots;
  while (!cand.empty()) {
    int v = cand.back();
    cand.pop_back();
    if (lds_need(v) <= tree_lds_limit() * 3 / 4) {
      roots.push_back(v);
      continue;
    }
    for (int c : {p->nodes[v - nv].c1, p->nodes[v - nv].c2})
      if (c >= nv && ok[c]) cand.push_back(c);
  }
  std::sort(roots.begin(), roots.end());
  for (int r : roots) {
    std::vector<int> stack{r};
    while (!stack.empty()) {
      int u = stack.back();
      stack.pop_back();
      if (u < nv) continue;
      p->in_tree[u] = 1;
      stack.push_back(p->nodes[u - nv].c1);
      stack.push_back(p->nodes[u - nv].c2);
    }
  }
  // a subtree is worth a launch of its own only above one vertex
  for (int r : roots) {
    const Node &n = p->nodes[r - nv];
    if (n.c1 < nv && n.c2 < nv && r != p->root) {
      p->in_tree[r] = 0;
      continue;
    }
    p->tree_roots.push_back(r);
  }
}

static void build_tree_programs(const tn_plan *p, ExecLayout &L, const std::vector<uint8_t> &ovr,
                                const std::vector<Layout> &lay) {
  const int nv = p->nv;
  std::vector<TreeHdr> hdrs;
  std::vector<TreeChunk> chunks;
  std::vector<TreeStep> steps;
  std::vector<TreeLeafLoad> loads;
  std::vector<float2> image;
  std::vector<int> ovr_list;  // overridden leaves in id order: index = TreeLaunch::ovr slot
  for (int t = 0; t < nv; ++t)
    if (ovr[t]) ovr_list.push_back(t);
  if ((int)ovr_list.size() > kTreeMaxOvr) {
    L.tree_error = true;  // more overridden leaves than the launch carries
    return;
  }
  std::vector<TreeSharedLoad> sloads;
  std::vector<int2> sgather;  // (LDS offset, shared-part offset) per island entry
  std::vector<char> is_island(2 * nv - 1, 0), is_spill(2 * nv - 1, 0);
  for (int u : L.islands) is_island[u] = 1;
  for (int u : L.spill) is_spill[u] = 1;
  std::vector<int> order;  // shared subtrees (and islands) first
  for (int r : p->tree_roots)
    if (L.shared[r]) order.push_back(r);
  for (int u : L.islands) order.push_back(u);
  L.n_tree_shared = (int)order.size();
  for (int r : p->tree_roots)
    if (!L.shared[r]) order.push_back(r);
  L.n_tree_perq = (int)order.size() - L.n_tree_shared;
  int max_scale_q = 0, max_sh_q = 0, max_pq_q = 0;
  size_t lds_sh = 0;
  for (int r : order) {
    TreeHdr h;
    memset(&h, 0, sizeof(h));
    std::vector<int> nodes, leaves, inputs, stack{r};  // inputs: islands read in
    while (!stack.empty()) {
      int u = stack.back();
      stack.pop_back();
      if (u < nv) {
        leaves.push_back(u);
        continue;
      }
      if (u != r && is_island[u]) {
        inputs.push_back(u);
        continue;
      }
      nodes.push_back(u);
      stack.push_back(p->nodes[u - nv].c1);
      stack.push_back(p->nodes[u - nv].c2);
    }
    std::sort(nodes.begin(), nodes.end());
    std::sort(leaves.begin(), leaves.end());
    std::sort(inputs.begin(), inputs.end());
    std::map<int, int32_t> loc;
    std::map<int, int> scale;
    // shared leaves: contiguous image; overridden leaves: front of the query region
    h.image_off = (int64_t)image.size();
    h.load0 = (int32_t)loads.size();
    int32_t sh = 0, pq = 0;
    // leaves with the same entries (a circuit's repeated gates) share one copy:
    // leaves are only read, and each step addresses a leaf through its own maps
    std::map<std::pair<int64_t, uint64_t>, std::vector<std::pair<int32_t, int>>> same;
    for (int t : leaves) {
      const int64_t n = p->leaf[t].size();
      if (!ovr[t]) {
        const float2 *src = p->leaf_host.data() + p->leaf_off[t];
        uint64_t hsh = 1469598103934665603ull;  // FNV-1a over the entries' bytes
        for (int64_t i = 0; i < n * 8; ++i) hsh = (hsh ^ ((const uint8_t *)src)[i]) * 1099511628211ull;
        auto &cands = same[{n, hsh}];
        int32_t at = -1;
        for (const auto &c : cands)
          if (memcmp(p->leaf_host.data() + p->leaf_off[c.second], src, (size_t)n * 8) == 0) {
            at = c.first;
            break;
          }
        if (at >= 0) {
          loc[t] = at;
          continue;
        }
        loc[t] = sh;
        cands.push_back({sh, t});
        for (int64_t i = 0; i < n; ++i) image.push_back(src[i]);
        if (n & 1) image.push_back(make_float2(0.f, 0.f));
        sh += (int32_t)((n + 1) & ~(int64_t)1);
      } else {
        loc[t] = kPerQuery | pq;
        TreeLeafLoad ld;
        ld.lds = kPerQuery | pq;
        ld.n = (int32_t)n;
        ld.src = (int32_t)(std::lower_bound(ovr_list.begin(), ovr_list.end(), t) - ovr_list.begin());
        ld.pad = 0;
        loads.push_back(ld);
        pq += (int32_t)((n + 1) & ~(int64_t)1);
      }
    }
    h.nloads = (int32_t)loads.size() - h.load0;
    // islands this subtree reads: after the shared leaves, scale records first
    h.sload0 = (int32_t)sloads.size();
    for (int u : inputs) {
      const int64_t n = std::max<int64_t>(p->nodes[u - nv].out.size(), 1);
      loc[u] = sh;
      scale[u] = (int)scale.size();
      TreeSharedLoad sl;
      sl.lds = sh;
      sl.n = (int32_t)n;
      sl.scale = scale[u];
      sl.slot = u;
      sl.off = L.off[u];
      sloads.push_back(sl);
      sh += (int32_t)((n + 1) & ~(int64_t)1);
    }
    h.nsloads = (int32_t)sloads.size() - h.sload0;
    h.nimg = h.nsloads ? sloads[h.sload0].lds : sh;
    h.sg0 = (int32_t)sgather.size();
    for (int i = h.sload0; i < h.sload0 + h.nsloads; ++i) {
      const TreeSharedLoad &sl = sloads[i];
      if (sl.off % 8 != 0 || sl.off / 8 + sl.n > INT32_MAX) {
        L.tree_error = true;
        return;
      }
      for (int32_t e = 0; e < sl.n; ++e) sgather.push_back(make_int2(sl.lds + e, (int32_t)(sl.off / 8) + e));
    }
    h.nsg = (int32_t)sgather.size() - h.sg0;
    h.shared_elems = sh;
    const int64_t base = pq;
    const LevelPlan lp = level_plan(p, nodes, &is_spill);
    for (int u : nodes) scale[u] = (int)scale.size();
    h.chunk0 = (int32_t)chunks.size();
    for (const auto &ch : lp.chunks) {
      TreeChunk tc;
      tc.step0 = (int32_t)steps.size();
      tc.nsteps = (int32_t)ch.size();
      for (int u : ch)
        if (!is_spill[u]) loc[u] = kPerQuery | (int32_t)(base + lp.at.at(u));
      for (int u : ch) {
        const Node &n = p->nodes[u - nv];
        TreeStep st;
        const bool final_dot = n.kind == NK_DOT && u == p->root;
        // an operand or the result in the query's device workspace: kind 3
        const int glob = (is_spill[n.c1] ? 1 : 0) | (is_spill[n.c2] ? 2 : 0) | (is_spill[u] ? 4 : 0);
        bool swap = false;
        memset(&st, 0, sizeof(st));
        if (final_dot || glob || !tree_stream_step(n, lay, st, swap)) {
          swap = false;
          tree_step(p, n, lay, final_dot, st);
        }
        const int ca_ = swap ? n.c2 : n.c1, cb_ = swap ? n.c1 : n.c2;
        auto dev_loc = [&](int v) { return (int32_t)(L.off[v] / 8); };
        st.a = (glob & 1) ? dev_loc(ca_) : loc[ca_];
        st.b = (glob & 2) ? dev_loc(cb_) : loc[cb_];
        st.c = (glob & 4) ? dev_loc(u) : loc[u];
        if (glob) {
          st.kind = 3;
          st.glob = glob;
        }
        st.asl = ca_ >= nv ? scale[ca_] : -1;
        st.bsl = cb_ >= nv ? scale[cb_] : -1;
        st.csl = scale[u];
        steps.push_back(st);
        if (final_dot) h.final_dot = 1;
      }
      chunks.push_back(tc);
    }
    h.nchunks = (int32_t)chunks.size() - h.chunk0;
    h.step0 = h.nchunks ? chunks[h.chunk0].step0 : (int32_t)steps.size();
    h.nsteps = (int32_t)steps.size() - h.step0;
    h.perq_elems = (int32_t)(base + lp.peak);
    // one record more than the vertices: it stays zero, and a kind 4 lane
    // reads it for an operand that is a leaf (scale 1)
    h.nscale = (int32_t)scale.size() + 1;
    h.root_loc = loc[r];
    h.root_scale = scale[r];
    h.root_elems = (int32_t)std::max<int64_t>(p->nodes[r - nv].out.size(), 1);
    h.root_in_perq = L.shared[r] ? 0 : 1;
    h.root_off = L.off[r];
    h.root_slot = r;
    hdrs.push_back(h);
    if (L.shared[r]) {
      lds_sh = std::max(lds_sh, tree_lds_bytes(1, h.nscale, h.shared_elems, h.perq_elems));
    } else {
      max_scale_q = std::max(max_scale_q, h.nscale);
      max_sh_q = std::max(max_sh_q, h.shared_elems);
      max_pq_q = std::max(max_pq_q, h.perq_elems);
      if (h.nloads) L.tree_reads_ovr = true;
    }
  }
  // every LDS access of every step must stay inside its region, checked here
  // so that a scheduling mistake disables the subtree kernel instead of
  // faulting it
  bool ok = true;
  for (const TreeHdr &h : hdrs) {
    auto reach = [](const int32_t *ext, const int32_t *s, int n) {
      int64_t r = 0;
      for (int i = 0; i < n; ++i) r += (int64_t)(ext[i] - 1) * s[i];
      return r;
    };
    auto inside = [&](int32_t loc, int64_t r) {
      if (loc & kPerQuery) return (loc & ~kPerQuery) + r < h.perq_elems;
      return loc + r < h.shared_elems;
    };
    // the chunks' steps are consecutive: [step0, step0 + nsteps)
    int32_t next = h.step0;
    for (int c = h.chunk0; c < h.chunk0 + h.nchunks; ++c) {
      ok = ok && chunks[c].step0 == next;
      next += chunks[c].nsteps;
    }
    ok = ok && next == h.step0 + h.nsteps && h.step0 >= 0 && h.step0 + h.nsteps <= (int32_t)steps.size();
    // a subtree ending in the closed root has it as its last step (the batch
    // kernel runs that step after its loop)
    ok = ok && h.nsteps >= 1 &&
         (steps[h.step0 + h.nsteps - 1].kind == 1) == (h.final_dot != 0);
    for (int c = h.chunk0; c < h.chunk0 + h.nchunks; ++c) {
      ok = ok && chunks[c].nsteps >= 1 && chunks[c].nsteps <= kTreeChunk;
      for (int k = chunks[c].step0; k < chunks[c].step0 + chunks[c].nsteps; ++k) {
        const TreeStep &st = steps[k];
        if (st.kind == 2) {
          // fibers: X reach + largest shared offset; C reach + largest cy < nc
          const int ns = st.ns, nfy = st.nss;
          ok = ok && (ns == 1 || ns == 2 || ns == 4) && (nfy == 1 || nfy == 2 || nfy == 4) &&
               st.nc % nfy == 0;
          if (!ok) break;
          int64_t mx = 0, mc = 0, my = 0;
          for (int v = 0; v < ns; ++v) mx = std::max<int64_t>(mx, st.xs[v]);
          for (int v = 0; v < nfy; ++v) mc = std::max<int64_t>(mc, st.cy[v]);
          for (int v = 0; v < ns * nfy; ++v) my = std::max<int64_t>(my, st.ymap[v]);
          const bool neg = std::min({st.xs[0], st.cy[0], st.ymap[0]}) < 0;
          // Y's shared and free legs are apart: ymap[s nfy + j] = ymap[s nfy] + ymap[j] - ymap[0]
          for (int a = 0; a < ns; ++a)
            for (int b = 0; b < nfy; ++b)
              ok = ok && st.ymap[a * nfy + b] == st.ymap[a * nfy] + st.ymap[b] - st.ymap[0];
          int64_t fib = 1;
          for (int i = 0; i < st.ncs; ++i) fib *= st.cext[i];
          ok = ok && !neg && fib * nfy == st.nc && inside(st.a, reach(st.cext, st.ca, st.ncs) + mx) &&
               inside(st.b, my) && (st.c & kPerQuery) &&
               reach(st.cext, st.cb, st.ncs) + mc < st.nc &&
               (st.c & ~kPerQuery) + st.nc <= h.perq_elems && st.csl >= 0 && st.csl < h.nscale &&
               st.asl < h.nscale && st.bsl < h.nscale;
          continue;
        }
        const int64_t ra = reach(st.cext, st.ca, st.ncs) + reach(st.sext, st.sa, st.nss);
        const int64_t rb = reach(st.cext, st.cb, st.ncs) + reach(st.sext, st.sb, st.nss);
        // kind 3: an operand in the query's device workspace stays inside it
        const int g = st.kind == 3 ? st.glob : 0;
        auto in_dev = [&](int32_t off, int64_t r) {
          return off >= 0 && 8 * ((int64_t)off + r + 1) <= L.perq_bytes;
        };
        ok = ok && (st.kind != 3 || (g > 0 && g < 8)) && (st.kind == 3 || st.glob == 0);
        ok = ok && ((g & 1) ? in_dev(st.a, ra) : inside(st.a, ra)) &&
             ((g & 2) ? in_dev(st.b, rb) : inside(st.b, rb)) &&
             ((g & 4) ? in_dev(st.c, st.nc - 1)
                      : (st.c & kPerQuery) && (st.c & ~kPerQuery) + st.nc <= h.perq_elems) &&
             st.csl >= 0 && st.csl < h.nscale && st.asl < h.nscale && st.bsl < h.nscale && st.nc >= 1 &&
             st.ns >= 1;
        // a closed-root inner product runs alone in the last chunk
        if (st.kind == 1) ok = ok && chunks[c].nsteps == 1 && c == h.chunk0 + h.nchunks - 1;
      }
    }
    // the islands' scale records are the first nsloads of the table, their
    // entries follow the image
    ok = ok && h.nsloads <= h.nscale && h.nimg >= 0 && h.nimg <= h.shared_elems &&
         h.sg0 >= 0 && h.nsg >= 0 && h.sg0 + h.nsg <= (int32_t)sgather.size();
    for (int i = h.sg0; ok && i < h.sg0 + h.nsg; ++i)
      ok = sgather[i].x >= h.nimg && sgather[i].x < h.shared_elems && sgather[i].y >= 0 &&
           8 * ((int64_t)sgather[i].y + 1) <= L.shared_bytes;
    for (int i = h.sload0; i < h.sload0 + h.nsloads; ++i)
      ok = ok && sloads[i].scale == i - h.sload0 && sloads[i].lds >= h.nimg &&
           sloads[i].lds >= 0 && sloads[i].lds + sloads[i].n <= h.shared_elems &&
           sloads[i].scale >= 0 && sloads[i].scale < h.nscale && sloads[i].slot >= nv &&
           sloads[i].slot < 2 * nv - 1 && sloads[i].off >= 0 &&
           sloads[i].off + 8 * (int64_t)sloads[i].n <= L.shared_bytes &&
           std::max<int64_t>(p->nodes[sloads[i].slot - nv].out.size(), 1) == sloads[i].n;
    for (int i = h.load0; i < h.load0 + h.nloads; ++i)
      ok = ok && (loads[i].lds & kPerQuery) && (loads[i].lds & ~kPerQuery) + loads[i].n <= h.perq_elems &&
           loads[i].src >= 0 && loads[i].src < (int)ovr_list.size() &&
           p->leaf[ovr_list[loads[i].src]].size() == loads[i].n;
    // the image holds the shared leaves; the islands read in follow them in LDS
    ok = ok && h.image_off + h.nimg <= (int64_t)image.size();
    if (!h.final_dot) {
      const int64_t part = h.root_in_perq ? L.perq_bytes : L.shared_bytes;
      ok = ok && (h.root_loc & kPerQuery) && (h.root_loc & ~kPerQuery) + h.root_elems <= h.perq_elems &&
           h.root_off >= 0 && h.root_off + 8 * (int64_t)h.root_elems <= part;
    }
  }
  if (!ok) {
    L.tree_error = true;
    return;
  }
  L.lds_shared = lds_sh;
  // Batches run the wave kernel: four waves a workgroup, one query each (the
  // single-query step forms), as many workgroups per CU as the LDS allows.
  // When four queries do not fit, the level kernel takes the batch.
  const size_t lim = tree_lds_limit();
  L.tree_wave = false;
  L.tree_qw = 1;
  if (tree_lds_bytes(4, max_scale_q, max_sh_q, max_pq_q, true) <= lim) {
    L.tree_qw = 4;
    L.tree_wave = true;
  }
  if (!L.tree_wave)
    for (int qw : {16, 12, 8, 6, 5, 4, 3, 2})
      if (tree_lds_bytes(qw, max_scale_q, max_sh_q, max_pq_q) <= lim / 2) {
        L.tree_qw = qw;
        break;
      }
  if (p->knobs.qw > 0) {  // the plan's tuned (or overridden) choice
    const int qw = p->knobs.qw;
    if (qw >= 1 && qw <= 16 && tree_lds_bytes(qw, max_scale_q, max_sh_q, max_pq_q, L.tree_wave) <= lim)
      L.tree_qw = qw;
  }
  L.lds_perq = tree_lds_bytes(L.tree_qw, max_scale_q, max_sh_q, max_pq_q, L.tree_wave);
  L.lds_perq1 = tree_lds_bytes(1, max_scale_q, max_sh_q, max_pq_q);
  // blob
  auto put = [&](const void *src, size_t bytes) {
    size_t off = (L.tree_blob.size() + 255) & ~(size_t)255;
    L.tree_blob.resize(off + bytes);
    if (bytes) memcpy(L.tree_blob.data() + off, src, bytes);
    return off;
  };
  // Kind 4: the small kind 2 steps of a level (result entries <= 64) packed
  // into steps of up to 64 entries, one lane record per entry, for programs
  // that only single-query groups run: the shared subtrees (one query per
  // launch) and, when their groups hold one query each, the per-query ones.
  // TN_TREE_PACK (tuning): 0 packs nothing, 1 only levels with several such
  // steps of one ns, 2 (the default) every such step.  TN_TREE_PACK_NC
  // (tuning) sets the size limit; a step above 64 entries takes several kind
  // 4 steps.
  std::vector<TreeLaneRec> lanes;
  {
    int mode = 2;
    const int most = p->knobs.pack_nc;
    if (const char *e = getenv("TN_TREE_PACK")) mode = atoi(e);
    const bool one_q = (L.tree_wave && L.tree_qw <= 4) || L.tree_qw == 1;
    std::vector<TreeStep> out;
    out.reserve(steps.size());
    for (size_t hi = 0; hi < hdrs.size(); ++hi) {
      TreeHdr &h = hdrs[hi];
      static const bool pack_shared = !getenv("TN_TREE_PACK_SHARED") || atoi(getenv("TN_TREE_PACK_SHARED")) != 0;
      const bool can = mode > 0 && ((int)hi < L.n_tree_shared ? pack_shared : one_q);
      const int32_t s0 = (int32_t)out.size();
      h.rec0 = (int32_t)lanes.size();
      for (int c = h.chunk0; c < h.chunk0 + h.nchunks; ++c) {
        const int32_t c0 = (int32_t)out.size();
        std::vector<int> cand[3];  // ns = 1, 2, 4
        for (int k = chunks[c].step0; k < chunks[c].step0 + chunks[c].nsteps; ++k) {
          const TreeStep &st = steps[k];
          if (can && st.kind == 2 && st.nc <= most && (st.c & kPerQuery))
            cand[st.ns == 1 ? 0 : st.ns == 2 ? 1 : 2].push_back(k);
          else
            out.push_back(st);
        }
        for (int g = 0; g < 3; ++g) {
          if (cand[g].empty()) continue;
          if (mode == 1 && cand[g].size() == 1) {
            out.push_back(steps[cand[g][0]]);
            continue;
          }
          const int ns = g == 0 ? 1 : g == 1 ? 2 : 4;
          // one record per result entry, in the steps' order
          std::vector<TreeLaneRec> recs;
          std::vector<int32_t> reads;  // query-region X and Y offsets
          std::vector<int32_t> writes;
          bool ok2 = true;
          for (int k : cand[g]) {
            const TreeStep &st = steps[k];
            const int nfy = st.nss;
            // byte offset in the operand's region
            auto addr = [&](int32_t loc, int64_t off) -> uint32_t {
              const bool q = (loc & kPerQuery) != 0;
              const int64_t i = (int64_t)(loc & ~kPerQuery) + off;
              const int64_t lim = q ? h.perq_elems : h.shared_elems;
              if (i < 0 || i >= lim || 8 * i >= 0x10000) ok2 = false;
              if (q) reads.push_back((int32_t)i);
              return (uint32_t)(8 * i) & 0xffffu;
            };
            for (int i = 0; i < st.nc; ++i) {
              const int j = i % nfy;
              int64_t f = i / nfy, xo = 0, co = 0;
              for (int d = 0; d < st.ncs; ++d) {
                const int64_t v = f % st.cext[d];
                f /= st.cext[d];
                xo += v * st.ca[d];
                co += v * st.cb[d];
              }
              uint32_t xa[4] = {0, 0, 0, 0}, ya[4] = {0, 0, 0, 0};
              for (int v = 0; v < ns; ++v) {
                xa[v] = addr(st.a, xo + st.xs[v]);
                ya[v] = addr(st.b, st.ymap[v * nfy + j]);
              }
              const int64_t ci = (int64_t)(st.c & ~kPerQuery) + co + st.cy[j];
              if (ci < 0 || ci >= h.perq_elems || 8 * ci >= 0x10000 || st.csl < 0 ||
                  st.csl >= h.nscale - 1 || h.nscale > 0x7fff || st.asl >= h.nscale - 1 ||
                  st.bsl >= h.nscale - 1)
                ok2 = false;
              writes.push_back((int32_t)ci);
              TreeLaneRec r;
              memset(&r, 0, sizeof(r));
              r.w[0] = xa[0] | xa[1] << 16;
              r.w[1] = ya[0] | ya[1] << 16;
              r.w[2] = (uint32_t)(8 * ci) | (uint32_t)st.csl << 16 | (i == 0 ? 1u << 31 : 0u);
              const int32_t zero = h.nscale - 1;  // the record no step writes
              r.w[3] = (uint32_t)(st.asl < 0 ? zero : st.asl) | ((st.a & kPerQuery) ? 0u : 1u << 15) |
                       (uint32_t)(st.bsl < 0 ? zero : st.bsl) << 16 | ((st.b & kPerQuery) ? 0u : 1u << 31);
              r.w[4] = xa[2] | xa[3] << 16;
              r.w[5] = ya[2] | ya[3] << 16;
              recs.push_back(r);
            }
          }
          // the packed steps are independent: no entry one of them writes is
          // read by another (or by itself), and no two write the same entry
          std::vector<int32_t> w2(writes);
          std::sort(w2.begin(), w2.end());
          ok2 = ok2 && std::adjacent_find(w2.begin(), w2.end()) == w2.end();
          for (const int32_t rd : reads)
            if (std::binary_search(w2.begin(), w2.end(), rd)) ok2 = false;
          if (!ok2) {  // keep the steps as they were
            for (int k : cand[g]) out.push_back(steps[k]);
            continue;
          }
          for (size_t r0 = 0; r0 < recs.size(); r0 += 64) {
            TreeStep ps;
            memset(&ps, 0, sizeof(ps));
            ps.kind = 4;
            ps.nc = (int32_t)std::min<size_t>(64, recs.size() - r0);
            ps.ns = ns;
            // one whole step in one kind 4 step (a larger one, TN_TREE_PACK_NC
            // above 64, spans several, which fold their maxes atomically)
            ps.nss = cand[g].size() == 1 && recs.size() <= 64 ? 1 : 0;
            ps.tab = (int32_t)lanes.size();
            for (int l = 0; l < ps.nc; ++l) lanes.push_back(recs[r0 + l]);
            out.push_back(ps);
          }
        }
        chunks[c].step0 = c0;
        chunks[c].nsteps = (int32_t)out.size() - c0;
        if (chunks[c].nsteps > kTreeChunk) {
          L.tree_error = true;
          return;
        }
      }
      h.step0 = s0;
      h.nsteps = (int32_t)out.size() - s0;
      h.nrec = (int32_t)lanes.size() - h.rec0;
    }
    steps.swap(out);
    // the level kernel keeps a program's lane records in LDS (after the
    // query regions, 16-byte aligned) when they fit: one copy at the start
    // instead of a device-memory round trip in every level
    const size_t lim = tree_lds_limit();
    size_t rec_q = 0;
    bool fit_q = true;
    for (size_t hi = 0; hi < hdrs.size(); ++hi) {
      TreeHdr &h = hdrs[hi];
      const size_t rb = h.nrec ? 16 + 32 * (size_t)h.nrec : 0;
      h.rec_lds = 0;
      if (!h.nrec) continue;
      if ((int)hi < L.n_tree_shared) {
        const size_t need = tree_lds_bytes(1, h.nscale, h.shared_elems, h.perq_elems) + rb;
        if (need <= lim) {
          h.rec_lds = 1;
          L.lds_shared = std::max(L.lds_shared, need);
        }
      } else {
        rec_q = std::max(rec_q, rb);
      }
    }
    // per-query programs: single queries run the level kernel with one query
    // per workgroup (lds_perq1; lds_perq too when there is no batch kernel)
    fit_q = L.lds_perq1 + rec_q <= lim && (L.tree_wave || L.lds_perq + rec_q <= lim);
    if (rec_q && fit_q) {
      for (size_t hi = (size_t)L.n_tree_shared; hi < hdrs.size(); ++hi)
        if (hdrs[hi].nrec) hdrs[hi].rec_lds = 1;
      L.lds_perq1 += rec_q;
      if (!L.tree_wave) L.lds_perq += rec_q;
    }
  }
  // The batch kernel's form of each per-query program: a run of whole-vertex
  // kind 4 steps in which each step's X operand is the step before's result
  // (a gate chain: one consumer per vertex, so no other step reads the
  // results inside the run) becomes one kind 5 step whose running tensor
  // stays in registers.  Its records: 64 per link (lanes past a link's
  // entries are copies of its first record), w[6] = ns | nc << 8; after the
  // first link the X terms name the lanes of the link before that hold them
  // (lane * 4, the ds_bpermute address).  The level kernel, which runs the
  // same programs for single queries and the shared subtrees, keeps the
  // steps as they are.  TN_TREE_CHAIN=0 turns chains off.
  //
  // The same pass fuses a kind 3 pair into one kind 6 step (the pair's two
  // descriptors, the first marked kind 6): P writes an intermediate T to the
  // query's device workspace and Q, the next step, contracts T with an
  // operand B that has no free legs, so each entry of T enters exactly one of
  // Q's products (checked here by enumerating them), and no other step reads
  // T or its scale record.  The batch kernel then keeps T in registers
  // (tree_pair).  TN_TREE_PAIR=0 turns pairs off.
  {
    const bool chain_on = !getenv("TN_TREE_CHAIN") || atoi(getenv("TN_TREE_CHAIN")) != 0;
    const bool pair_on = !getenv("TN_TREE_PAIR") || atoi(getenv("TN_TREE_PAIR")) != 0;
    for (size_t hi = 0; hi < hdrs.size(); ++hi) {
      TreeHdr &h = hdrs[hi];
      h.wstep0 = h.step0;
      h.wnsteps = h.nsteps;
      if ((!chain_on && !pair_on) || (int)hi < L.n_tree_shared || !L.tree_wave) continue;
      auto whole = [&](const TreeStep &st) { return st.kind == 4 && st.nss == 1 && st.nc >= 1 && st.nc <= 64; };
      // entry byte offset -> lane of a whole step's records
      auto lane_of = [&](const TreeStep &st) {
        std::map<uint32_t, int> m;
        for (int l = 0; l < st.nc; ++l) m[lanes[st.tab + l].w[2] & 0xffffu] = l;
        return m;
      };
      auto x_fields = [](const TreeLaneRec &r, int ns, uint32_t *xo) {
        xo[0] = r.w[0] & 0xffffu;
        xo[1] = r.w[0] >> 16;
        xo[2] = r.w[4] & 0xffffu;
        xo[3] = r.w[4] >> 16;
        return ns;
      };
      // B takes A's result as its X operand, every X term an entry A writes
      auto links = [&](const TreeStep &A, const TreeStep &B) {
        if (!whole(A) || !whole(B)) return false;
        const TreeLaneRec &ra = lanes[A.tab], &rb = lanes[B.tab];
        if ((rb.w[3] & 0x8000u) || (rb.w[3] & 0x7fffu) != ((ra.w[2] >> 16) & 0x7fffu)) return false;
        const std::map<uint32_t, int> m = lane_of(A);
        for (int l = 0; l < B.nc; ++l) {
          uint32_t xo[4];
          const int ns = x_fields(lanes[B.tab + l], B.ns, xo);
          for (int v = 0; v < ns; ++v)
            if (!m.count(xo[v])) return false;
        }
        return true;
      };
      std::vector<TreeStep> prog;
      std::vector<TreeLaneRec> crec;
      bool any = false;
      int npairs = 0;
      const int kend = h.step0 + h.nsteps;
      // a map (extents, as the host keeps them): index -> offset
      auto decode = [](const int32_t *ext, const int32_t *st, int nseg, int idx) {
        int o = 0;
        for (int i = 0; i < nseg; ++i) {
          o += (idx % ext[i]) * st[i];
          idx /= ext[i];
        }
        return o;
      };
      // the consumer of P's intermediate, if P and it form a pair that can run
      // at P's place: every step between them is a kind 4 step that neither
      // reads nor writes Q's result entries, writes no entry of Q's B, and
      // touches none of Q's scale records (from its lane records); -1 if not
      auto pair_partner = [&](int k) {
        const TreeStep &P = steps[k];
        if (P.kind != 3 || P.glob != 4 || !P.pow2 || P.csl < 0 || P.ns > 64) return -1;
        auto reads_t = [&](const TreeStep &o) {
          return (o.kind == 3 && (((o.glob & 1) && o.a == P.c) || ((o.glob & 2) && o.b == P.c))) ||
                 (o.kind != 4 && (o.asl == P.csl || o.bsl == P.csl));
        };
        int q = -1;
        for (int j = k + 1; j < kend; ++j)
          if (reads_t(steps[j])) {
            if (q >= 0) return -1;  // a second reader
            q = j;
          }
        if (q < 0) return -1;
        const TreeStep &Q = steps[q];
        if (Q.kind != 3 || Q.glob != 1 || !Q.pow2 || Q.a != P.c || Q.asl != P.csl || Q.ns > 4 ||
            Q.nc > 256 || Q.nc * Q.ns != P.nc || !(Q.c & kPerQuery))
          return -1;
        for (int i = 0; i < Q.ncs; ++i)
          if (Q.cext[i] > 1 && Q.cb[i] != 0) return -1;  // B has a free leg
        std::vector<char> hit((size_t)P.nc, 0);
        for (int co = 0; co < Q.nc; ++co) {
          const int ao = decode(Q.cext, Q.ca, Q.ncs, co);
          for (int sh = 0; sh < Q.ns; ++sh) {
            const int so = decode(Q.sext, Q.sa, Q.nss, sh);
            const int t = ao + so;
            // the kernel splits P's map of t over the bits of ao and of so
            if ((ao & so) != 0 || t < 0 || t >= P.nc || hit[(size_t)t]++) return -1;
          }
        }
        // Q's result entries and B's entries (in the query region or shared)
        const int qc0 = Q.c & ~kPerQuery, qc1 = qc0 + Q.nc;
        const bool b_q = (Q.b & kPerQuery) != 0;
        std::vector<int> bent;
        for (int sh = 0; sh < Q.ns; ++sh) bent.push_back((Q.b & ~kPerQuery) + decode(Q.sext, Q.sb, Q.nss, sh));
        for (int j = k + 1; j < q; ++j) {
          const TreeStep &m = steps[j];
          if (m.kind != 4) return -1;
          for (int l = 0; l < m.nc; ++l) {
            const TreeLaneRec &r = lanes[m.tab + l];
            const int csl = (int)((r.w[2] >> 16) & 0x7fffu), asl = (int)(r.w[3] & 0x7fffu),
                      bsl = (int)((r.w[3] >> 16) & 0x7fffu);
            if (csl == Q.bsl || csl == Q.csl || asl == Q.csl || bsl == Q.csl) return -1;
            const int ce = (int)(r.w[2] & 0xffffu) / 8;  // result entry (query region)
            if (ce >= qc0 && ce < qc1) return -1;
            if (b_q)
              for (int e : bent)
                if (e == ce) return -1;
            const uint32_t xo[4] = {r.w[0] & 0xffffu, r.w[0] >> 16, r.w[4] & 0xffffu, r.w[4] >> 16};
            const uint32_t yo[4] = {r.w[1] & 0xffffu, r.w[1] >> 16, r.w[5] & 0xffffu, r.w[5] >> 16};
            for (int v = 0; v < m.ns; ++v) {
              const int xe = (int)xo[v] / 8, ye = (int)yo[v] / 8;
              if (!(r.w[3] & 0x8000u) && xe >= qc0 && xe < qc1) return -1;
              if (!(r.w[3] & 0x80000000u) && ye >= qc0 && ye < qc1) return -1;
            }
          }
        }
        return q;
      };
      // this kernel's step order: the consumer of each pair moved up to its
      // producer, the steps between them after it
      std::vector<int> ord;
      std::vector<char> head;
      {
        std::vector<char> moved((size_t)(kend - h.step0), 0);
        for (int k = h.step0; k < kend; ++k) {
          if (moved[(size_t)(k - h.step0)]) continue;
          const int q = pair_on ? pair_partner(k) : -1;
          ord.push_back(k);
          head.push_back(q >= 0);
          if (q >= 0) {
            ord.push_back(q);
            head.push_back(0);
            moved[(size_t)(q - h.step0)] = 1;
            ++npairs;
          }
        }
      }
      for (size_t x = 0; x < ord.size();) {
        const int k = ord[x];
        if (head[x]) {
          TreeStep ps = steps[k];
          ps.kind = 6;
          prog.push_back(ps);
          prog.push_back(steps[ord[x + 1]]);
          any = true;
          x += 2;
          continue;
        }
        // a run of chained steps: consecutive in this order, none in a pair
        size_t x2 = x;
        while (chain_on && x2 + 1 < ord.size() && !head[x2 + 1] && ord[x2 + 1] == ord[x2] + 1 &&
               links(steps[ord[x2]], steps[ord[x2 + 1]]))
          ++x2;
        const int k2 = ord[x2];
        if (x2 == x) {
          prog.push_back(steps[k]);
          ++x;
          continue;
        }
        TreeStep ps;
        memset(&ps, 0, sizeof(ps));
        ps.kind = 5;
        ps.nc = k2 - k + 1;  // links
        ps.ns = 4;
        ps.tab = (int32_t)(lanes.size() + crec.size());
        for (int j = k; j <= k2; ++j) {
          const TreeStep &st = steps[j];
          std::map<uint32_t, int> m;
          if (j > k) m = lane_of(steps[j - 1]);
          for (int l = 0; l < 64; ++l) {
            TreeLaneRec r = lanes[st.tab + (l < st.nc ? l : 0)];
            if (j > k) {
              uint32_t xo[4];
              x_fields(r, st.ns, xo);
              uint32_t a[4] = {0, 0, 0, 0};
              for (int v = 0; v < st.ns; ++v) a[v] = 4u * (uint32_t)m.at(xo[v]);
              r.w[0] = a[0] | a[1] << 16;
              r.w[4] = a[2] | a[3] << 16;
            }
            r.w[6] = (uint32_t)st.ns | (uint32_t)st.nc << 8;
            r.w[7] = 0;
            crec.push_back(r);
          }
        }
        prog.push_back(ps);
        any = true;
        x = x2 + 1;
      }
      if (!any) continue;
      h.wstep0 = (int32_t)steps.size();
      h.wnsteps = (int32_t)prog.size();
      steps.insert(steps.end(), prog.begin(), prog.end());
      lanes.insert(lanes.end(), crec.begin(), crec.end());
      if (getenv("TN_DEBUG"))
        fprintf(stderr, "[tn]   subtree root %d: batch program of %d steps (kind 5 chains: %d links; "
                "kind 6 pairs: %d)\n", h.root_slot, h.wnsteps, (int)(crec.size() / 64), npairs);
    }
  }
  if (getenv("TN_DEBUG"))
    for (const TreeHdr &h : hdrs) {
      int gate = 0, packed = 0, nsteps = 0;
      for (int c = h.chunk0; c < h.chunk0 + h.nchunks; ++c)
        for (int k = chunks[c].step0; k < chunks[c].step0 + chunks[c].nsteps; ++k) {
          ++nsteps;
          gate += steps[k].kind == 2;
          packed += steps[k].kind == 4;
        }
      fprintf(stderr, "[tn]   subtree root %d: %d chunks, %d steps (%d gate form, %d packed), %d shared "
              "leaf entries, %d per-query entries, %d scale records, %d loads\n", h.root_slot,
              h.nchunks, nsteps, gate, packed, h.shared_elems, h.perq_elems, h.nscale, h.nloads);
      // TN_DEBUG=steps: one line per step (kind, result and shared-index
      // entries, gate fibers, device-workspace operands)
      if (strcmp(getenv("TN_DEBUG"), "steps") == 0)
        for (int c = h.chunk0; c < h.chunk0 + h.nchunks; ++c)
          for (int k = chunks[c].step0; k < chunks[c].step0 + chunks[c].nsteps; ++k) {
            const TreeStep &s = steps[k];
            fprintf(stderr, "[tn]     chunk %d step %d: kind %d nc %d ns %d nss %d ncs %d pow2 %d glob %d\n",
                    c - h.chunk0, k, s.kind, s.nc, s.ns, s.nss, s.ncs, s.pow2, s.glob);
          }
    }
  // device form of the steps (after the checks above, which read the plain
  // form): power-of-two maps carry their masks (extent - 1) and the kind 2
  // offsets are in bytes, which saves the kernels that arithmetic per step
  for (TreeStep &st : steps) {
    if (st.kind == 4 || st.kind == 5) continue;
    if (st.pow2) {
      // the kernels run every segment of a power-of-two map: the unused ones
      // must be all zero (mask, shift and strides)
      for (int i = st.ncs; i < kTreeSeg; ++i)
        if (st.cext[i] | st.ca[i] | st.cb[i] | st.clg[i]) {
          L.tree_error = true;
          return;
        }
      if (st.kind != 2)
        for (int i = st.nss; i < kTreeSeg; ++i)
          if (st.sext[i] | st.sa[i] | st.sb[i] | st.slg[i]) {
            L.tree_error = true;
            return;
          }
      for (int i = 0; i < st.ncs; ++i) st.cext[i] -= 1;
      if (st.kind != 2)
        for (int i = 0; i < st.nss; ++i) st.sext[i] -= 1;
    }
    if (st.kind == 2) {
      for (int v = 0; v < 4; ++v) {
        st.xs[v] *= 8;
        st.cy[v] *= 8;
      }
      for (int v = 0; v < 16; ++v) st.ymap[v] *= 8;
    }
  }
  put(hdrs.data(), hdrs.size() * sizeof(TreeHdr));
  L.tree_chunk_off = put(chunks.data(), chunks.size() * sizeof(TreeChunk));
  L.tree_step_off = put(steps.data(), steps.size() * sizeof(TreeStep));
  L.tree_load_off = put(loads.data(), loads.size() * sizeof(TreeLeafLoad));
  L.tree_sload_off = put(sloads.data(), sloads.size() * sizeof(TreeSharedLoad));
  L.tree_sg_off = put(sgather.data(), sgather.size() * sizeof(int2));
  L.tree_img_off = put(image.data(), image.size() * sizeof(float2));
  L.tree_lane_off = put(lanes.data(), lanes.size() * sizeof(TreeLaneRec));
}

ExecLayout make_exec_layout(const tn_plan *p, const std::vector<int> &overridden, bool share,
                            bool allow_trees, bool conc) {
  const int nv = p->nv, nn = 2 * nv - 1;
  ExecLayout L;
  // concurrent partitions: the vertices of partition k's subtree (and their
  // scratch) take memory from a packer of their own, laid out after the
  // reduction path's, so partitions running side by side never share memory
  conc = conc && !share && p->K > 1;
  L.conc = conc;
  L.off.assign(nn, -1);
  L.shared.assign(nn, 1);
  L.scr_a.assign(nv > 1 ? nv - 1 : 0, -1);
  L.scr_b = L.scr_a;
  L.partial = L.scr_a;
  L.ovr_off.assign(nv, -1);
  std::vector<uint8_t> ovr(nv, 0);
  for (int t : overridden) ovr[t] = 1;
  // per-query override block: overridden leaves in increasing id order
  int64_t ob = 0;
  for (int t = 0; t < nv; ++t)
    if (ovr[t]) {
      L.ovr_off[t] = ob;
      ob += (p->leaf[t].size() * 8 + 255) & ~(int64_t)255;
    }
  L.ovr_bytes = ob;
  for (int v = 0; v < nv; ++v) L.shared[v] = ovr[v] ? 0 : 1;
  for (const Node &n : p->nodes) L.shared[n.id] = L.shared[n.c1] && L.shared[n.c2];
  if (!share)  // plain execution: every intermediate belongs to the query
    for (int v = nv; v < nn; ++v) L.shared[v] = 0;
  const bool trees = allow_trees && share && !p->tree_roots.empty();
  auto is_root = [&](int v) {
    return std::find(p->tree_roots.begin(), p->tree_roots.end(), v) != p->tree_roots.end();
  };
  Packer pk[2];  // 0: per-query, 1: shared
  std::vector<Packer> pkp(conc ? p->K : 0);  // concurrent partitions
  auto packer_of = [&](const Node &n) -> Packer & {
    if (conc && n.part >= 0) return pkp[n.part];
    return pk[L.shared[n.id] ? 1 : 0];
  };
  std::vector<int8_t> in_part(nn, -1);  // partition packer a vertex's memory came from
  // Islands: the largest vertices that no override reaches inside a per-query
  // subtree.  They run once, as shared subtrees of their own, and the
  // per-query programs read their results instead of recomputing them for
  // every query.
  L.islands.clear();
  if (trees)
    for (int r : p->tree_roots) {
      if (L.shared[r]) continue;
      std::vector<int> stack{r};
      while (!stack.empty()) {
        const int u = stack.back();
        stack.pop_back();
        for (int c : {p->nodes[u - nv].c1, p->nodes[u - nv].c2}) {
          if (c < nv) continue;
          if (L.shared[c])
            L.islands.push_back(c);
          else
            stack.push_back(c);
        }
      }
    }
  std::sort(L.islands.begin(), L.islands.end());
  // subtree results are written before any other vertex runs
  if (trees) {
    for (int r : p->tree_roots)
      L.off[r] = pk[L.shared[r] ? 1 : 0].alloc(out_bytes_of(p->nodes[r - nv]));
    for (int u : L.islands) L.off[u] = pk[1].alloc(out_bytes_of(p->nodes[u - nv]));
    // the large intermediates of per-query subtrees stay in the query's part
    // of the workspace (their whole lifetime), which keeps each query's LDS
    // small enough for more queries per CU
    L.spill.clear();
    const int64_t spill_at = p->knobs.spill;  // the plan's choice (tuning table, TN_TREE_SPILL)
    for (int r : p->tree_roots) {
      if (L.shared[r]) continue;
      std::vector<int> stack{p->nodes[r - nv].c1, p->nodes[r - nv].c2};
      while (!stack.empty()) {
        const int u = stack.back();
        stack.pop_back();
        if (u < nv || L.shared[u]) continue;  // leaves, islands
        const Node &n = p->nodes[u - nv];
        if ((int64_t)n.out.size() >= spill_at) L.spill.push_back(u);
        stack.push_back(n.c1);
        stack.push_back(n.c2);
      }
    }
    std::sort(L.spill.begin(), L.spill.end());
    for (int u : L.spill) L.off[u] = pk[0].alloc(out_bytes_of(p->nodes[u - nv]));
  }
  for (int j : p->order) {
    const Node &n = p->nodes[j];
    if (trees && p->in_tree[n.id]) continue;
    Packer &P = packer_of(n);
    if (conc && n.part >= 0) in_part[n.id] = (int8_t)n.part;
    int64_t out_bytes = out_bytes_of(n);
    L.off[n.id] = P.alloc(out_bytes);
    std::vector<std::pair<int64_t, int64_t>> tmp;
    if (n.kind == NK_GEMM) {
      // complex64 or two float planes (8 bytes an entry), or split bf16 planes
      // (2 bytes a plane)
      const int64_t eb = n.planes > 2 ? 2 * n.planes : 8;
      if (n.pa.needed) {
        L.scr_a[j] = P.alloc(n.pa.h.nelem * eb);
        tmp.push_back({L.scr_a[j], n.pa.h.nelem * eb});
      }
      if (n.pb.needed) {
        L.scr_b[j] = P.alloc(n.pb.h.nelem * eb);
        tmp.push_back({L.scr_b[j], n.pb.h.nelem * eb});
      }
      if (n.ksplit > 1) {
        const int64_t pb = (int64_t)n.ksplit * n.M * n.N * 8;
        L.partial[j] = P.alloc(pb);
        tmp.push_back({L.partial[j], pb});
      }
    } else if (n.kind == NK_DOT) {
      L.partial[j] = P.alloc((int64_t)n.dot_blocks * 16);
      tmp.push_back({L.partial[j], (int64_t)n.dot_blocks * 16});
    }
    for (auto &t : tmp) P.release(t.first, t.second);
    // children die here unless they live in the other part (shared results
    // feeding per-query vertices stay for the whole execution)
    for (int c : {n.c1, n.c2}) {
      if (c < nv || L.off[c] < 0) continue;
      // (a partition's result read by the reduction path stays: it lives in
      // the partition's own region)
      if (in_part[c] != in_part[n.id]) continue;
      if (L.shared[c] == L.shared[n.id]) {
        const Node &cn = p->nodes[c - nv];
        P.release(L.off[c], out_bytes_of(cn));
      }
    }
  }
  (void)is_root;
  L.peak_intermediate = pk[0].peak();
  L.perq_bytes = pk[0].peak();
  L.shared_bytes = pk[1].peak();
  if (conc) {
    // partition regions after the reduction path's, each 256-byte aligned
    std::vector<int64_t> base(p->K);
    int64_t top = (L.perq_bytes + 255) & ~(int64_t)255;
    for (int k = 0; k < p->K; ++k) {
      base[k] = top;
      top += (pkp[k].peak() + 255) & ~(int64_t)255;
    }
    for (const Node &n : p->nodes) {
      if (in_part[n.id] < 0) continue;
      const int64_t b = base[in_part[n.id]];
      const int j = n.id - nv;
      L.off[n.id] += b;
      if (L.scr_a[j] >= 0) L.scr_a[j] += b;
      if (L.scr_b[j] >= 0) L.scr_b[j] += b;
      if (L.partial[j] >= 0) L.partial[j] += b;
    }
    L.perq_bytes = top;
    L.peak_intermediate = top;
  }
  if (trees) {
    L.all_in_tree = true;
    for (const Node &n : p->nodes) L.all_in_tree = L.all_in_tree && p->in_tree[n.id];
    std::vector<Layout> lay(nn);
    for (int v = 0; v < nv; ++v) lay[v] = p->leaf[v];
    for (const Node &n : p->nodes) lay[n.id] = n.out;
    build_tree_programs(p, L, ovr, lay);
  }
  return L;
}

std::shared_ptr<ExecLayout> cached_layout(tn_plan *p, const std::vector<int> &overridden,
                                          bool share, bool conc) {
  std::lock_guard<std::mutex> g(p->cache_mu);
  std::vector<int> key = overridden;
  key.push_back(share ? -1 : conc ? -3 : -2);
  auto it = p->layouts.find(key);
  if (it != p->layouts.end()) return it->second;
  auto L = std::make_shared<ExecLayout>(make_exec_layout(p, overridden, share, true, conc));
  if (L->tree_error)  // fall back to one launch per vertex
    L = std::make_shared<ExecLayout>(make_exec_layout(p, overridden, share, false, conc));
  if (getenv("TN_DEBUG"))
    fprintf(stderr,
            "[tn] layout: %zu overridden leaves, share %d, subtrees %d shared + %d per query, "
            "%d queries/workgroup (wave kernel %d), LDS %zu / %zu bytes, per-query part %lld "
            "bytes, shared part %lld bytes, tree error %d\n",
            overridden.size(), (int)share, L->n_tree_shared, L->n_tree_perq, L->tree_qw,
            (int)L->tree_wave,
            L->lds_shared, L->lds_perq, (long long)L->perq_bytes, (long long)L->shared_bytes,
            (int)L->tree_error);
  p->layouts[key] = L;
  return L;
}

}  // namespace tn
