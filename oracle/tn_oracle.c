/*
 * CPU oracle for partitioned tensor-network contraction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the GPU library against a plain,
 * slow, obviously correct reference.  It shares no code with the library.
 *
 * Contents (all arithmetic in complex128 / exact 128-bit integers):
 *   oracle_contract_tree  - pairwise contraction (eq. basic_contraction,
 *                           generalised to permuted axes, Section 2.2) along
 *                           any contraction tree given in SSA form;
 *   oracle_brute_force    - the full contraction written as its definition:
 *                           a sum over every assignment of every bound edge
 *                           of the product of tensor entries (Section 2.2);
 *   oracle_statevector    - an independent algorithm for circuit amplitudes:
 *                           gate-by-gate application to a 2^n state vector;
 *   oracle_costs          - legs(v) (Section 2.3), 2^vc, con_serial, con_par,
 *                           con_dist (comm = 0), mem (Section 3) recomputed
 *                           with unsigned __int128 arithmetic.
 *
 * Readings of the paper used here: path(v,u) includes both ends, so the
 * critical path of eq. con_par drops only the leaf and the paths of
 * eq. con_dist drop root(B_k) but keep root(B); 2^vc is the exact product of
 * the edge dimensions; comm(c) = 0 (Section 3.3, as in the experiments).
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ tensors */

typedef struct {
  int rank;
  int64_t *labels; /* length rank */
  int64_t *dims;   /* length rank */
  int64_t size;    /* product of dims */
  cplx *data;      /* row-major: last leg fastest */
} otensor;

static int64_t prod_dims(const int64_t *d, int r) {
  int64_t p = 1;
  for (int i = 0; i < r; ++i) p *= d[i];
  return p;
}

static void row_major_strides(const int64_t *dims, int r, int64_t *st) {
  int64_t s = 1;
  for (int i = r - 1; i >= 0; --i) {
    st[i] = s;
    s *= dims[i];
  }
}

static int find_label(const int64_t *labels, int r, int64_t lab) {
  for (int i = 0; i < r; ++i)
    if (labels[i] == lab) return i;
  return -1;
}

static void free_tensor(otensor *t) {
  free(t->labels);
  free(t->dims);
  free(t->data);
  memset(t, 0, sizeof(*t));
}

/*
 * R = contraction of A and B over their common labels.  R's legs are A's
 * remaining legs in A's order followed by B's remaining legs in B's order,
 * which is the index order of eq. basic_contraction.  Every output entry is
 * the plain sum over the shared index of A-entry times B-entry.
 */
static int contract_pair(const otensor *A, const otensor *B, otensor *R, int nthreads) {
  int ra = A->rank, rb = B->rank;
  int64_t sa[64], sb[64];
  row_major_strides(A->dims, ra, sa);
  row_major_strides(B->dims, rb, sb);

  /* free legs of R and the shared legs */
  int rr = 0, ns = 0;
  int64_t rlab[128], rdim[128], rsa[128], rsb[128];
  int64_t sdim[64], ssa[64], ssb[64];
  for (int i = 0; i < ra; ++i) {
    int j = find_label(B->labels, rb, A->labels[i]);
    if (j < 0) {
      rlab[rr] = A->labels[i];
      rdim[rr] = A->dims[i];
      rsa[rr] = sa[i];
      rsb[rr] = 0;
      ++rr;
    } else {
      if (A->dims[i] != B->dims[j]) return -1;
      sdim[ns] = A->dims[i];
      ssa[ns] = sa[i];
      ssb[ns] = sb[j];
      ++ns;
    }
  }
  for (int j = 0; j < rb; ++j) {
    if (find_label(A->labels, ra, B->labels[j]) < 0) {
      rlab[rr] = B->labels[j];
      rdim[rr] = B->dims[j];
      rsa[rr] = 0;
      rsb[rr] = sb[j];
      ++rr;
    }
  }
  int64_t rsize = prod_dims(rdim, rr);
  int64_t ssize = prod_dims(sdim, ns);

  /* offsets of every shared-index value into A and into B */
  int64_t *offa = malloc(sizeof(int64_t) * (size_t)ssize);
  int64_t *offb = malloc(sizeof(int64_t) * (size_t)ssize);
  for (int64_t s = 0; s < ssize; ++s) {
    int64_t rem = s, oa = 0, ob = 0;
    for (int i = ns - 1; i >= 0; --i) {
      int64_t idx = rem % sdim[i];
      rem /= sdim[i];
      oa += idx * ssa[i];
      ob += idx * ssb[i];
    }
    offa[s] = oa;
    offb[s] = ob;
  }

  R->rank = rr;
  R->labels = malloc(sizeof(int64_t) * (size_t)(rr ? rr : 1));
  R->dims = malloc(sizeof(int64_t) * (size_t)(rr ? rr : 1));
  memcpy(R->labels, rlab, sizeof(int64_t) * (size_t)rr);
  memcpy(R->dims, rdim, sizeof(int64_t) * (size_t)rr);
  R->size = rsize;
  R->data = malloc(sizeof(cplx) * (size_t)rsize);
  if (!R->data || !offa || !offb) {
    free(offa);
    free(offb);
    return -2;
  }

  const cplx *ad = A->data, *bd = B->data;
  cplx *rd = R->data;
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t r = 0; r < rsize; ++r) {
    int64_t rem = r, oa = 0, ob = 0;
    for (int i = rr - 1; i >= 0; --i) {
      int64_t idx = rem % rdim[i];
      rem /= rdim[i];
      oa += idx * rsa[i];
      ob += idx * rsb[i];
    }
    cplx acc = 0;
    for (int64_t s = 0; s < ssize; ++s) acc += ad[oa + offa[s]] * bd[ob + offb[s]];
    rd[r] = acc;
  }
  free(offa);
  free(offb);
  return 0;
}

/* Copy `t` into `out` with the legs reordered to `order` (labels). */
static int write_in_order(const otensor *t, int n_out, const int64_t *order, cplx *out) {
  if (n_out != t->rank) return -1;
  int64_t st[128], odim[128], ost[128];
  row_major_strides(t->dims, t->rank, st);
  for (int i = 0; i < n_out; ++i) {
    int j = find_label(t->labels, t->rank, order[i]);
    if (j < 0) return -1;
    odim[i] = t->dims[j];
    ost[i] = st[j];
  }
  for (int64_t o = 0; o < t->size; ++o) {
    int64_t rem = o, off = 0;
    for (int i = n_out - 1; i >= 0; --i) {
      int64_t idx = rem % odim[i];
      rem /= odim[i];
      off += idx * ost[i];
    }
    out[o] = t->data[off];
  }
  return 0;
}

/*
 * Contract the whole network along `tree` (SSA pairs: internal vertex nv+j
 * contracts tree[2j], tree[2j+1]; the last pair is the root).  `data` holds
 * the leaves back to back as interleaved complex128, row-major in each
 * tensor's leg order.  The result is written in the order `out_labels`
 * (length n_out; n_out == 0 for a scalar).  Returns 0, or <0 on a malformed
 * input or allocation failure.
 */
int oracle_contract_tree(int nv, const int32_t *rank, const int64_t *labels, const int64_t *dims,
                         const double *data, const int32_t *tree, int n_out,
                         const int64_t *out_labels, double *out, int nthreads) {
  if (nv <= 0) return -1;
  int nn = 2 * nv - 1;
  otensor *T = calloc((size_t)nn, sizeof(otensor));
  const int64_t *lp = labels, *dp = dims;
  const cplx *src = (const cplx *)data;
  for (int v = 0; v < nv; ++v) {
    int r = rank[v];
    T[v].rank = r;
    T[v].labels = malloc(sizeof(int64_t) * (size_t)(r ? r : 1));
    T[v].dims = malloc(sizeof(int64_t) * (size_t)(r ? r : 1));
    memcpy(T[v].labels, lp, sizeof(int64_t) * (size_t)r);
    memcpy(T[v].dims, dp, sizeof(int64_t) * (size_t)r);
    T[v].size = prod_dims(dp, r);
    T[v].data = malloc(sizeof(cplx) * (size_t)T[v].size);
    memcpy(T[v].data, src, sizeof(cplx) * (size_t)T[v].size);
    src += T[v].size;
    lp += r;
    dp += r;
  }
  int rc = 0;
  for (int j = 0; j < nv - 1; ++j) {
    int a = tree[2 * j], b = tree[2 * j + 1];
    if (a < 0 || b < 0 || a == b || a >= nv + j || b >= nv + j || !T[a].data || !T[b].data) {
      rc = -1;
      break;
    }
    rc = contract_pair(&T[a], &T[b], &T[nv + j], nthreads);
    if (rc) break;
    free_tensor(&T[a]);
    free_tensor(&T[b]);
  }
  if (!rc) rc = write_in_order(&T[nn - 1], n_out, out_labels, (cplx *)out);
  for (int v = 0; v < nn; ++v) free_tensor(&T[v]);
  free(T);
  return rc;
}

/*
 * The contraction as its definition: for every assignment of the open
 * labels (in `out_labels` order, row-major) sum, over every assignment of the
 * bound labels, the product of all tensor entries.  Exponential; for tiny
 * networks only.
 */
int oracle_brute_force(int nv, const int32_t *rank, const int64_t *labels, const int64_t *dims,
                       const double *data, int n_out, const int64_t *out_labels, double *out) {
  /* distinct labels */
  int64_t total_legs = 0;
  for (int v = 0; v < nv; ++v) total_legs += rank[v];
  int64_t *lab = malloc(sizeof(int64_t) * (size_t)(total_legs + 1));
  int64_t *ldim = malloc(sizeof(int64_t) * (size_t)(total_legs + 1));
  int nl = 0;
  for (int64_t i = 0; i < total_legs; ++i) {
    if (find_label(lab, nl, labels[i]) < 0) {
      lab[nl] = labels[i];
      ldim[nl] = dims[i];
      ++nl;
    }
  }
  /* bound labels: those not listed as open */
  int64_t bdim[64];
  int bl[64], nb = 0, ol[64];
  for (int i = 0; i < nl; ++i) {
    if (find_label(out_labels, n_out, lab[i]) < 0) {
      bl[nb] = i;
      bdim[nb] = ldim[i];
      ++nb;
    }
  }
  int64_t odim[64];
  for (int i = 0; i < n_out; ++i) {
    ol[i] = find_label(lab, nl, out_labels[i]);
    if (ol[i] < 0) {
      free(lab);
      free(ldim);
      return -1;
    }
    odim[i] = ldim[ol[i]];
  }
  int64_t osize = prod_dims(odim, n_out), bsize = prod_dims(bdim, nb);
  int64_t *assign = calloc((size_t)(nl + 1), sizeof(int64_t));
  const cplx *td = (const cplx *)data;
  for (int64_t o = 0; o < osize; ++o) {
    int64_t rem = o;
    for (int i = n_out - 1; i >= 0; --i) {
      assign[ol[i]] = rem % odim[i];
      rem /= odim[i];
    }
    cplx total = 0;
    for (int64_t bidx = 0; bidx < bsize; ++bidx) {
      rem = bidx;
      for (int i = nb - 1; i >= 0; --i) {
        assign[bl[i]] = rem % bdim[i];
        rem /= bdim[i];
      }
      cplx term = 1;
      const int64_t *lp = labels, *dp = dims;
      const cplx *p = td;
      for (int v = 0; v < nv; ++v) {
        int64_t off = 0;
        for (int a = 0; a < rank[v]; ++a) off = off * dp[a] + assign[find_label(lab, nl, lp[a])];
        term *= p[off];
        p += prod_dims(dp, rank[v]);
        lp += rank[v];
        dp += rank[v];
      }
      total += term;
    }
    ((cplx *)out)[o] = total;
  }
  free(assign);
  free(lab);
  free(ldim);
  return 0;
}

/*
 * Amplitudes of U|0...0> by applying each gate matrix to the state vector.
 * Gate g acts on nq[g] in {1,2} qubits q[2g], q[2g+1]; its matrix is
 * mats[16g ...] (2x2 or 4x4 complex128, row-major).  A two-qubit matrix on
 * (q1, q2) is indexed [2*o1 + o2][2*i1 + i2].  Qubit q is bit q of the basis
 * index.  `state` receives 2^n complex128 values.
 */
int oracle_statevector(int n, int ngates, const int32_t *nq, const int32_t *q, const double *mats,
                       double *state_out, int nthreads) {
  int64_t dim = (int64_t)1 << n;
  cplx *psi = (cplx *)state_out;
  for (int64_t i = 0; i < dim; ++i) psi[i] = 0;
  psi[0] = 1;
  const cplx *M = (const cplx *)mats;
  for (int g = 0; g < ngates; ++g) {
    const cplx *G = M + 16 * (int64_t)g;
    if (nq[g] == 1) {
      int64_t bit = (int64_t)1 << q[2 * g];
#pragma omp parallel for schedule(static) num_threads(nthreads)
      for (int64_t i = 0; i < dim; ++i) {
        if (i & bit) continue;
        cplx a0 = psi[i], a1 = psi[i | bit];
        psi[i] = G[0] * a0 + G[1] * a1;
        psi[i | bit] = G[2] * a0 + G[3] * a1;
      }
    } else if (nq[g] == 2) {
      int64_t b1 = (int64_t)1 << q[2 * g], b2 = (int64_t)1 << q[2 * g + 1];
      if (b1 == b2) return -1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
      for (int64_t i = 0; i < dim; ++i) {
        if ((i & b1) || (i & b2)) continue;
        int64_t idx[4] = {i, i | b2, i | b1, i | b1 | b2}; /* sub-index 2*bit(q1) + bit(q2) */
        cplx a[4], r[4];
        for (int k = 0; k < 4; ++k) a[k] = psi[idx[k]];
        for (int o = 0; o < 4; ++o) {
          r[o] = 0;
          for (int k = 0; k < 4; ++k) r[o] += G[4 * o + k] * a[k];
        }
        for (int k = 0; k < 4; ++k) psi[idx[k]] = r[k];
      }
    } else {
      return -1;
    }
  }
  return 0;
}

/* ---------------------------------------------------------------- costs */

typedef struct {
  int n;
  int64_t *lab; /* sorted */
} legset;

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

/* symmetric difference (xor) and union of two sorted label sets */
static void set_ops(const legset *a, const legset *b, legset *sym, legset *uni) {
  int i = 0, j = 0;
  sym->n = 0;
  uni->n = 0;
  while (i < a->n || j < b->n) {
    if (j >= b->n || (i < a->n && a->lab[i] < b->lab[j])) {
      sym->lab[sym->n++] = a->lab[i];
      uni->lab[uni->n++] = a->lab[i];
      ++i;
    } else if (i >= a->n || b->lab[j] < a->lab[i]) {
      sym->lab[sym->n++] = b->lab[j];
      uni->lab[uni->n++] = b->lab[j];
      ++j;
    } else {
      uni->lab[uni->n++] = a->lab[i];
      ++i;
      ++j;
    }
  }
}

static int label_dim(const int64_t *all_lab, const int64_t *all_dim, int64_t n, int64_t lab,
                     int64_t *d) {
  for (int64_t i = 0; i < n; ++i)
    if (all_lab[i] == lab) {
      *d = all_dim[i];
      return 0;
    }
  return -1;
}

static int set_size(const legset *s, const int64_t *all_lab, const int64_t *all_dim, int64_t n,
                    u128 *out) {
  u128 p = 1;
  for (int i = 0; i < s->n; ++i) {
    int64_t d;
    if (label_dim(all_lab, all_dim, n, s->lab[i], &d)) return -1;
    u128 np = p * (u128)d;
    if (d != 0 && np / (u128)d != p) return -3; /* overflow */
    p = np;
  }
  *out = p;
  return 0;
}

static void put128(uint64_t *dst, u128 v) {
  dst[0] = (uint64_t)(v >> 64);
  dst[1] = (uint64_t)v;
}

/*
 * Costs of the tree for the given partitioning.  out (uint64 pairs, hi then
 * lo): [0..1] con_serial, [2..3] con_par, [4..5] con_dist, [6..7] mem,
 * [8..9] largest intermediate.  Returns 0, -1 on malformed input, -2 if the
 * tree does not accept the partitioning, -3 on 128-bit overflow.
 */
int oracle_costs(int nv, const int32_t *rank, const int64_t *labels, const int64_t *dims,
                 const int32_t *tree, const int32_t *partition_of, int num_partitions,
                 uint64_t *out) {
  int nn = 2 * nv - 1;
  int64_t total = 0;
  for (int v = 0; v < nv; ++v) total += rank[v];
  legset *L = calloc((size_t)nn, sizeof(legset));
  u128 *w = calloc((size_t)nn, sizeof(u128));        /* 2^vc of internal vertices */
  u128 *sz = calloc((size_t)nn, sizeof(u128));       /* |legs(v)| product */
  int32_t *parent = malloc(sizeof(int32_t) * (size_t)nn);
  int rc = 0;
  int64_t off = 0;
  for (int v = 0; v < nv; ++v) {
    L[v].n = rank[v];
    L[v].lab = malloc(sizeof(int64_t) * (size_t)(rank[v] + 1));
    memcpy(L[v].lab, labels + off, sizeof(int64_t) * (size_t)rank[v]);
    qsort(L[v].lab, (size_t)rank[v], sizeof(int64_t), cmp_i64);
    off += rank[v];
    if (set_size(&L[v], labels, dims, total, &sz[v])) rc = -1;
  }
  for (int v = 0; v < nn; ++v) parent[v] = -1;
  u128 con_serial = 0, mem = 0, largest = 0;
  for (int j = 0; j < nv - 1 && !rc; ++j) {
    int a = tree[2 * j], b = tree[2 * j + 1], v = nv + j;
    if (a < 0 || b < 0 || a >= v || b >= v || a == b || parent[a] >= 0 || parent[b] >= 0) {
      rc = -1;
      break;
    }
    parent[a] = parent[b] = v;
    legset uni;
    uni.lab = malloc(sizeof(int64_t) * (size_t)(L[a].n + L[b].n + 1));
    L[v].lab = malloc(sizeof(int64_t) * (size_t)(L[a].n + L[b].n + 1));
    set_ops(&L[a], &L[b], &L[v], &uni);
    int e1 = set_size(&uni, labels, dims, total, &w[v]);
    int e2 = set_size(&L[v], labels, dims, total, &sz[v]);
    free(uni.lab);
    if (e1 || e2) {
      rc = (e1 == -3 || e2 == -3) ? -3 : -1;
      break;
    }
    con_serial += w[v];
    u128 m = sz[v] + sz[a] + sz[b];
    if (m > mem) mem = m;
    if (sz[v] > largest) largest = sz[v];
  }
  if (!rc) {
    /* critical path: heaviest leaf-to-root chain, leaf excluded */
    u128 *best = calloc((size_t)nn, sizeof(u128));
    for (int j = 0; j < nv - 1; ++j) {
      int a = tree[2 * j], b = tree[2 * j + 1], v = nv + j;
      best[v] = w[v] + (best[a] > best[b] ? best[a] : best[b]);
    }
    u128 con_par = nv > 1 ? best[nn - 1] : 0;
    free(best);

    /* partition roots: the vertex whose leaves are exactly partition k */
    int32_t *cnt_k = calloc((size_t)num_partitions, sizeof(int32_t));
    for (int v = 0; v < nv; ++v) {
      if (partition_of[v] < 0 || partition_of[v] >= num_partitions) rc = -1;
      else cnt_k[partition_of[v]]++;
    }
    /* per vertex: partition of all its leaves (or -1 if mixed) and leaf count */
    int32_t *pk = malloc(sizeof(int32_t) * (size_t)nn);
    int32_t *nleaf = malloc(sizeof(int32_t) * (size_t)nn);
    for (int v = 0; v < nv && !rc; ++v) {
      pk[v] = partition_of[v];
      nleaf[v] = 1;
    }
    for (int j = 0; j < nv - 1 && !rc; ++j) {
      int a = tree[2 * j], b = tree[2 * j + 1], v = nv + j;
      pk[v] = (pk[a] >= 0 && pk[a] == pk[b]) ? pk[a] : -1;
      nleaf[v] = nleaf[a] + nleaf[b];
    }
    u128 con_dist = 0;
    for (int k = 0; k < num_partitions && !rc; ++k) {
      int root = -1;
      for (int v = 0; v < nn; ++v)
        if (pk[v] == k && nleaf[v] == cnt_k[k]) root = v;
      if (cnt_k[k] == 0 || root < 0) {
        rc = -2;
        break;
      }
      /* con_serial of B_k: every internal vertex whose leaves all lie in k */
      u128 c = 0;
      for (int v = nv; v < nn; ++v)
        if (pk[v] == k) c += w[v];
      for (int u = parent[root]; u >= 0; u = parent[u]) c += w[u];
      if (c > con_dist) con_dist = c;
    }
    free(cnt_k);
    free(pk);
    free(nleaf);
    if (!rc) {
      put128(out + 0, con_serial);
      put128(out + 2, con_par);
      put128(out + 4, con_dist);
      put128(out + 6, mem);
      put128(out + 8, largest);
    }
  }
  for (int v = 0; v < nn; ++v) free(L[v].lab);
  free(L);
  free(w);
  free(sz);
  free(parent);
  return rc;
}
