// Slicing on top of partitioning.  A contraction is a sum over every bound
// index (Section 2.2), so fixing some bound legs value by value and adding
// the results of the fixed networks (the slices) gives the full result; every
// slice has the same network with those legs of dimension 1, hence one plan
// whose tree and partitioning are the original's.  The slices of a call run
// as the queries of one batch (the vertices no sliced leg reaches are shared
// between them) and their results are added on the device in FP64.
#include <algorithm>
#include <cstring>
#include <new>
#include <set>

#include "tn_internal.h"

namespace tn {

// Legs to fix so that no intermediate exceeds `target` entries: greedily the
// bound label whose fixing shrinks the current largest intermediate most
// (ties: the label on more intermediates of that size, then the lower label).
static std::vector<int64_t> choose_slice_labels(const tn_plan *p, int64_t target) {
  const int nv = p->nv;
  std::map<int64_t, int> count;
  std::map<int64_t, int64_t> dim;
  for (int v = 0; v < nv; ++v)
    for (int i = 0; i < p->leaf[v].rank(); ++i) {
      count[p->leaf[v].lab[i]]++;
      dim[p->leaf[v].lab[i]] = p->leaf[v].dim[i];
    }
  std::vector<const Layout *> inter;
  for (const Node &n : p->nodes) inter.push_back(&n.out);
  std::set<int64_t> sliced;
  auto size_with = [&](const Layout &L, const std::set<int64_t> &S) {
    int64_t s = 1;
    for (int i = 0; i < L.rank(); ++i)
      if (!S.count(L.lab[i])) s *= L.dim[i];
    return s;
  };
  auto largest = [&](const std::set<int64_t> &S) {
    int64_t m = 1;
    for (const Layout *L : inter) m = std::max(m, size_with(*L, S));
    return m;
  };
  std::vector<int64_t> out;
  while (out.size() < 30) {
    const int64_t top = largest(sliced);
    if (top <= target) break;
    int64_t best = -1, best_after = 0;
    int best_on = 0;
    for (auto &kv : count) {
      const int64_t e = kv.first;
      if (kv.second != 2 || dim[e] <= 1 || sliced.count(e)) continue;
      int on = 0;
      for (const Layout *L : inter)
        if (size_with(*L, sliced) == top && L->find(e) >= 0) ++on;
      if (!on) continue;
      std::set<int64_t> t = sliced;
      t.insert(e);
      const int64_t after = largest(t);
      if (best < 0 || after < best_after || (after == best_after && on > best_on)) {
        best = e;
        best_after = after;
        best_on = on;
      }
    }
    if (best < 0) break;
    sliced.insert(best);
    out.push_back(best);
  }
  return out;
}

// Row-major sub-tensor of a tensor with layout L whose legs in `fix` are
// fixed to the given values (those legs keep dimension 1 in the result).
static void sub_tensor(const Layout &L, const float2 *src, const std::map<int64_t, int64_t> &fix,
                       float2 *dst) {
  const int r = L.rank();
  std::vector<int64_t> st = L.strides(), sub(r);
  int64_t base = 0, n = 1;
  for (int i = 0; i < r; ++i) {
    auto it = fix.find(L.lab[i]);
    sub[i] = it != fix.end() ? 1 : L.dim[i];
    if (it != fix.end()) base += it->second * st[i];
    n *= sub[i];
  }
  std::vector<int64_t> idx(r, 0);
  for (int64_t o = 0; o < n; ++o) {
    int64_t off = base;
    for (int i = 0; i < r; ++i) off += idx[i] * st[i];
    dst[o] = src[off];
    for (int i = r - 1; i >= 0; --i) {
      if (++idx[i] < sub[i]) break;
      idx[i] = 0;
    }
  }
}

static std::map<int64_t, int64_t> slice_values(const std::vector<int64_t> &labels,
                                                const std::vector<int64_t> &radix, int64_t slice) {
  std::map<int64_t, int64_t> fix;
  for (int k = (int)labels.size() - 1; k >= 0; --k) {
    fix[labels[k]] = slice % radix[k];
    slice /= radix[k];
  }
  return fix;
}

tn_status make_sliced_plan(tn_ctx *ctx, const tn_plan *p, std::vector<int64_t> labels,
                           int64_t max_intermediate, tn_plan **out) {
  if (p->nslices > 0) {
    set_error("tn_plan_slice: the plan is already sliced");
    return TN_E_INVALID_ARG;
  }
  const int nv = p->nv;
  std::map<int64_t, int> count;
  std::map<int64_t, int64_t> dim;
  for (int v = 0; v < nv; ++v)
    for (int i = 0; i < p->leaf[v].rank(); ++i) {
      count[p->leaf[v].lab[i]]++;
      dim[p->leaf[v].lab[i]] = p->leaf[v].dim[i];
    }
  if (labels.empty()) labels = choose_slice_labels(p, std::max<int64_t>(1, max_intermediate));
  if (labels.empty()) {
    set_error("tn_plan_slice: no leg to fix (every intermediate already within %lld entries)",
              (long long)max_intermediate);
    return TN_E_INVALID_ARG;
  }
  std::set<int64_t> S;
  int64_t nslices = 1;
  std::vector<int64_t> radix;
  for (int64_t l : labels) {
    if (!count.count(l) || count[l] != 2 || S.count(l)) {
      set_error("tn_plan_slice: label %lld is not a bound leg (or repeated)", (long long)l);
      return TN_E_INVALID_ARG;
    }
    S.insert(l);
    radix.push_back(dim[l]);
    nslices *= dim[l];
    if (nslices > (1 << 24)) {
      set_error("tn_plan_slice: more than 2^24 slices");
      return TN_E_INVALID_ARG;
    }
  }
  // the sliced network: the same legs, the fixed ones of dimension 1; the
  // tensors that carry one take slice 0's sub-tensors
  std::vector<int32_t> rank(nv);
  std::vector<int64_t> legs, dims;
  std::vector<int> touched;
  for (int v = 0; v < nv; ++v) {
    rank[v] = p->leaf[v].rank();
    bool t = false;
    for (int i = 0; i < rank[v]; ++i) {
      legs.push_back(p->leaf[v].lab[i]);
      const bool f = S.count(p->leaf[v].lab[i]) > 0;
      dims.push_back(f ? 1 : p->leaf[v].dim[i]);
      t = t || f;
    }
    if (t) touched.push_back(v);
  }
  std::vector<int64_t> sub_off(touched.size());
  int64_t block = 0;
  for (size_t k = 0; k < touched.size(); ++k) {
    sub_off[k] = block;
    int64_t n = 1;
    for (int i = 0; i < p->leaf[touched[k]].rank(); ++i)
      n *= S.count(p->leaf[touched[k]].lab[i]) ? 1 : p->leaf[touched[k]].dim[i];
    block += n;
  }
  std::vector<float2> data((size_t)(nslices * block));
  for (int64_t sl = 0; sl < nslices; ++sl) {
    const std::map<int64_t, int64_t> fix = slice_values(labels, radix, sl);
    for (size_t k = 0; k < touched.size(); ++k) {
      const int t = touched[k];
      sub_tensor(p->leaf[t], p->leaf_host.data() + p->leaf_off[t], fix,
                 data.data() + sl * block + sub_off[k]);
    }
  }
  std::vector<const void *> ptr(nv);
  for (int v = 0; v < nv; ++v) ptr[v] = p->leaf_host.data() + p->leaf_off[v];
  for (size_t k = 0; k < touched.size(); ++k) ptr[touched[k]] = data.data() + sub_off[k];
  tn_plan_desc d;
  memset(&d, 0, sizeof(d));
  d.num_tensors = nv;
  d.rank = rank.data();
  d.legs = legs.data();
  d.leg_dims = dims.data();
  d.data = ptr.data();
  d.data_dtype = TN_C64;
  d.partition_of = p->partition_of.data();
  d.num_partitions = p->K;
  d.tree = p->tree.data();
  d.output_legs = p->out_labels.empty() ? nullptr : p->out_labels.data();
  d.num_output_legs = (int32_t)p->out_labels.size();
  tn_plan *s = nullptr;
  tn_status st = tn_plan_load(ctx, &d, p->flags, &s);
  if (st != TN_OK) return st;
  s->nslices = nslices;
  s->slice_labels = labels;
  s->slice_radix = radix;
  s->slice_touched = touched;
  s->slice_sub_off = sub_off;
  s->slice_block = block;
  s->slice_data.swap(data);
  for (int t : touched) s->slice_full.push_back(p->leaf[t]);
  *out = s;
  return TN_OK;
}

static void to_c64(const tn_leaf &l, int64_t n, float2 *dst) {
  if (l.dtype == TN_C128) {
    const double *src = (const double *)l.data;
    for (int64_t i = 0; i < n; ++i) dst[i] = make_float2((float)src[2 * i], (float)src[2 * i + 1]);
  } else {
    memcpy(dst, l.data, sizeof(float2) * n);
  }
}

tn_status run_sliced(tn_ctx *ctx, tn_plan *p, int32_t novr, const tn_leaf *ovr, void *out,
                     tn_dtype out_dtype, double *log2_scale, uint32_t flags, ExecRes &rs) {
  if (out_dtype != TN_C64 && out_dtype != TN_C128) {
    set_error("out_dtype must be TN_C64 or TN_C128");
    return TN_E_INVALID_ARG;
  }
  // slice data of every touched tensor: the plan's own, or a caller's
  // override of that tensor (full size, host memory) cut into slices
  std::vector<int> tk(p->nv, -1);
  for (size_t k = 0; k < p->slice_touched.size(); ++k) tk[p->slice_touched[k]] = (int)k;
  std::vector<float2> own;  // overridden touched tensors, cut per slice
  std::vector<tn_leaf> keep;
  std::vector<std::pair<int, const tn_leaf *>> cut;
  for (int32_t i = 0; i < novr; ++i) {
    const tn_leaf &l = ovr[i];
    if (l.tensor < 0 || l.tensor >= p->nv || !l.data) {
      set_error("override %d: tensor id out of range or NULL data", i);
      return TN_E_INVALID_ARG;
    }
    if (tk[l.tensor] < 0) {
      keep.push_back(l);
      continue;
    }
    if (l.dtype == TN_C64_DEVICE) {
      set_error("override %d: a tensor that carries a sliced leg needs host data", i);
      return TN_E_INVALID_ARG;
    }
    cut.push_back({tk[l.tensor], &l});
  }
  std::vector<float2> slices(p->slice_data);
  if (!cut.empty()) {
    for (auto &c : cut) {
      const Layout &full = p->slice_full[c.first];
      std::vector<float2> src((size_t)full.size());
      to_c64(*c.second, full.size(), src.data());
      for (int64_t sl = 0; sl < p->nslices; ++sl)
        sub_tensor(full, src.data(), slice_values(p->slice_labels, p->slice_radix, sl),
                   slices.data() + sl * p->slice_block + p->slice_sub_off[c.first]);
    }
  }
  // one query per slice: the caller's other overrides and the slice's cuts
  const size_t nt = p->slice_touched.size();
  std::vector<tn_leaf> leaves((size_t)p->nslices * (keep.size() + nt));
  std::vector<QueryIO> qs((size_t)p->nslices);
  std::vector<double> dummy(2);
  for (int64_t sl = 0; sl < p->nslices; ++sl) {
    tn_leaf *q = leaves.data() + sl * (keep.size() + nt);
    for (size_t k = 0; k < keep.size(); ++k) q[k] = keep[k];
    for (size_t k = 0; k < nt; ++k) {
      q[keep.size() + k].tensor = p->slice_touched[k];
      q[keep.size() + k].data = slices.data() + sl * p->slice_block + p->slice_sub_off[k];
      q[keep.size() + k].dtype = TN_C64;
    }
    qs[sl].ovr = q;
    qs[sl].novr = (int32_t)(keep.size() + nt);
    qs[sl].out = dummy.data();
  }
  SliceSum sum;
  tn_status rc = run_group(ctx, p, qs, TN_C128, 0, true, rs, nullptr, &sum);
  if (rc != TN_OK) return rc;
  const size_t n = sum.acc.size() / 2;
  const bool keep_scale = (flags & TN_FLAG_KEEP_SCALE) != 0;
  const int e = (int)sum.log2s;
  for (size_t i = 0; i < n; ++i) {
    double re = sum.acc[2 * i], im = sum.acc[2 * i + 1];
    if (!keep_scale) {
      re = std::ldexp(re, e);
      im = std::ldexp(im, e);
    }
    if (out_dtype == TN_C128) {
      ((double *)out)[2 * i] = re;
      ((double *)out)[2 * i + 1] = im;
    } else {
      ((float *)out)[2 * i] = (float)re;
      ((float *)out)[2 * i + 1] = (float)im;
    }
  }
  if (log2_scale) *log2_scale = keep_scale ? sum.log2s : 0.0;
  return TN_OK;
}

}  // namespace tn
