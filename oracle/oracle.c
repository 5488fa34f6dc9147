/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the two-level additive Schwarz
 * preconditioned conjugate gradient method on spatial networks
 * (Goertz, Hellman, Malqvist, "Iterative solution of spatial network models by
 * subspace decomposition", arXiv 2207.07488).
 *
 * TEST INFRASTRUCTURE ONLY. The product library never calls, links or loads
 * anything in this directory; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark do. It shares no code, header, table or
 * helper with the GPU path.
 *
 * Written for a reader who checks it against the paper by eye: single
 * threaded, no blocking, no fusion, built with -ffp-contract=off.
 *
 * Sections of the paper followed:
 *   network, nodes, edges, Dirichlet set      Sec. 2.1
 *   weighted Laplacian / heat operator         Sec. 2.2 eq. (2.2), Example 3.2 eq. (3.3)
 *   tensile (truss) operator                   Example 3.3 eq. (3.4)
 *   mesh T_H of half-open boxes, patches U,
 *   Q1 space restricted to the nodes           Sec. 2.3
 *   subspace decomposition V_0 = V_H,
 *   V_j = V(U(y_j)), projections P_j            Sec. 4.1 eq. (4.1); the
 *     nodes of V_j are those at which phi_j is positive (the support of
 *     phi_j, which Sec. 5 identifies with U(y_j)); the heat experiment of
 *     Sec. 6.2 (Table 6.2, grid row) is reproduced with this set
 *   PCG on P = BK                              Sec. 4.2
 * The fiber generator is the one of Sec. 6.1 with the workload parameters
 * passed in by the caller (segments are an input; see workloads).
 *
 * parity pinned: every function is checked by the CPU tests against closed
 * forms, invariants, brute force or dense linear algebra (see tests/).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ESINGULAR (-4)
#define ORC_ENOTSPD (-5)
#define ORC_ENOCONV (-6)

static char orc_errbuf[512];

const char *orc_last_error(void) { return orc_errbuf; }

static int orc_fail(int code, const char *msg) {
  snprintf(orc_errbuf, sizeof orc_errbuf, "%s", msg);
  return code;
}

static void *zalloc(size_t n, size_t sz) {
  void *p = calloc(n ? n : 1, sz);
  if (!p) {
    fprintf(stderr, "oracle: out of memory\n");
    abort();
  }
  return p;
}

/* ------------------------------------------------------------------ */
/* growable arrays                                                      */
/* ------------------------------------------------------------------ */
typedef struct { int64_t *a; int64_t n, cap; } ivec;

static void ivec_push(ivec *v, int64_t x) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 64;
    v->a = realloc(v->a, (size_t)v->cap * sizeof(int64_t));
    if (!v->a) abort();
  }
  v->a[v->n++] = x;
}
/* squared distance, summed over coordinates in increasing order */
static double dist2(int dim, const double *p, const double *q) {
  double s = 0.0;
  for (int k = 0; k < dim; k++) {
    double t = p[k] - q[k];
    s = s + t * t;
  }
  return s;
}

static double dot3(int dim, const double *u, const double *v) {
  double s = 0.0;
  for (int k = 0; k < dim; k++) s = s + u[k] * v[k];
  return s;
}

static double clamp01(double t) { return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t); }

/* union-find whose root is always the smallest member */
static int64_t uf_find(int64_t *par, int64_t i) {
  while (par[i] != i) {
    par[i] = par[par[i]];
    i = par[i];
  }
  return i;
}
static void uf_union(int64_t *par, int64_t a, int64_t b) {
  a = uf_find(par, a);
  b = uf_find(par, b);
  if (a < b) par[b] = a;
  else if (b < a) par[a] = b;
}

/* ================================================================== */
/* Network (Sec. 2.1; generator of Sec. 6.1)                           */
/* ================================================================== */
typedef struct orc_net {
  int dim;
  int64_t n_nodes, n_edges;
  double *x;     /* n_nodes * dim */
  int32_t *e;    /* 2 * n_edges */
  uint8_t *dir;  /* 1 if the node is in the Dirichlet set N(Gamma) */
  int64_t n_segments_kept, n_raw_nodes;
} orc_net;

/*
 * Clip the segment a->b to the closed unit box (the part outside is removed,
 * Sec. 6.1). Returns 0 if nothing of length >= tol remains. The face that
 * fixes each end is snapped to exactly 0 or 1.
 */
static int clip_segment(int dim, const double *a, const double *b, double tol,
                        double *A, double *B) {
  double d[3];
  double t0 = 0.0, t1 = 1.0;
  int f0 = -1, f1 = -1;
  for (int k = 0; k < dim; k++) d[k] = b[k] - a[k];
  for (int k = 0; k < dim; k++) {
    if (d[k] == 0.0) {
      if (a[k] < 0.0 || a[k] > 1.0) return 0;
      continue;
    }
    double tlo = (0.0 - a[k]) / d[k];
    double thi = (1.0 - a[k]) / d[k];
    double tin, tout;
    int fin, fout;
    if (d[k] > 0.0) {
      tin = tlo; fin = 2 * k;
      tout = thi; fout = 2 * k + 1;
    } else {
      tin = thi; fin = 2 * k + 1;
      tout = tlo; fout = 2 * k;
    }
    if (tin > t0) { t0 = tin; f0 = fin; }
    if (tout < t1) { t1 = tout; f1 = fout; }
  }
  if (!(t0 < t1)) return 0;
  for (int k = 0; k < dim; k++) {
    A[k] = a[k] + t0 * d[k];
    B[k] = a[k] + t1 * d[k];
  }
  if (f0 >= 0) A[f0 / 2] = (double)(f0 & 1);
  if (f1 >= 0) B[f1 / 2] = (double)(f1 & 1);
  for (int k = 0; k < dim; k++) {
    A[k] = clamp01(A[k]);
    B[k] = clamp01(B[k]);
  }
  if (!(dist2(dim, A, B) >= tol * tol)) return 0;
  return 1;
}

typedef struct { int64_t i, j; double ti, tj; double p[3]; } crossing;

/* 2D: proper or touching intersection of two segments (parallel pairs never meet) */
static int cross2d(const double *Ai, const double *Bi, const double *Aj,
                   const double *Bj, crossing *c) {
  double di[2] = {Bi[0] - Ai[0], Bi[1] - Ai[1]};
  double dj[2] = {Bj[0] - Aj[0], Bj[1] - Aj[1]};
  double den = di[0] * dj[1] - di[1] * dj[0];
  if (den == 0.0) return 0;
  double w[2] = {Aj[0] - Ai[0], Aj[1] - Ai[1]};
  double t = (w[0] * dj[1] - w[1] * dj[0]) / den;
  double s = (w[0] * di[1] - w[1] * di[0]) / den;
  if (!(t >= 0.0 && t <= 1.0 && s >= 0.0 && s <= 1.0)) return 0;
  c->ti = t;
  c->tj = s;
  c->p[0] = Ai[0] + t * di[0];
  c->p[1] = Ai[1] + t * di[1];
  return 1;
}

/* 3D: contact when the closest approach of two segments is below eps; the node
 * sits at the midpoint of the two closest points (closest points of two
 * segments as in Ericson, Real-Time Collision Detection, Sec. 5.1.9). */
static int contact3d(const double *Ai, const double *Bi, const double *Aj,
                     const double *Bj, double eps, crossing *c) {
  double d1[3], d2[3], r[3];
  for (int k = 0; k < 3; k++) {
    d1[k] = Bi[k] - Ai[k];
    d2[k] = Bj[k] - Aj[k];
    r[k] = Ai[k] - Aj[k];
  }
  double a = dot3(3, d1, d1);
  double e = dot3(3, d2, d2);
  double f = dot3(3, d2, r);
  double cc = dot3(3, d1, r);
  double b = dot3(3, d1, d2);
  double den = a * e - b * b;
  double s = 0.0, t;
  if (den != 0.0) s = clamp01((b * f - cc * e) / den);
  t = (b * s + f) / e;
  if (t < 0.0) {
    t = 0.0;
    s = clamp01(-cc / a);
  } else if (t > 1.0) {
    t = 1.0;
    s = clamp01((b - cc) / a);
  }
  double P1[3], P2[3];
  for (int k = 0; k < 3; k++) {
    P1[k] = Ai[k] + s * d1[k];
    P2[k] = Aj[k] + t * d2[k];
  }
  if (!(dist2(3, P1, P2) < eps * eps)) return 0;
  c->ti = s;
  c->tj = t;
  for (int k = 0; k < 3; k++) c->p[k] = 0.5 * (P1[k] + P2[k]);
  return 1;
}

static int cmp_crossing(const void *pa, const void *pb) {
  const crossing *a = pa, *b = pb;
  if (a->i != b->i) return a->i < b->i ? -1 : 1;
  if (a->j != b->j) return a->j < b->j ? -1 : 1;
  return 0;
}

typedef struct { double t; int64_t id; } param_node;
static int cmp_param_node(const void *pa, const void *pb) {
  const param_node *a = pa, *b = pb;
  if (a->t != b->t) return a->t < b->t ? -1 : 1;
  if (a->id != b->id) return a->id < b->id ? -1 : 1;
  return 0;
}

typedef struct { double key; int64_t id; } key_id;
static int cmp_key_id(const void *pa, const void *pb) {
  const key_id *a = pa, *b = pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->id != b->id) return a->id < b->id ? -1 : 1;
  return 0;
}

void orc_net_free(orc_net *n) {
  if (!n) return;
  free(n->x);
  free(n->e);
  free(n->dir);
  free(n);
}

/*
 * Build the network from raw segments seg[i] = (a_0..a_{d-1}, b_0..b_{d-1}).
 *   contact_eps  3D contact distance (ignored in 2D, where exact crossings are used)
 *   merge_tol    nodes closer than this are merged (Sec. 6.1 uses r*1e-4)
 *   dir_lo/hi    bit k set: the face x_k = 0 (resp. 1) belongs to Gamma
 *   band         a node is in N(Gamma) if it lies within band of a Gamma face
 *   brute        1: test all segment pairs; 0: only pairs in neighbouring cells
 */
int orc_net_build(int dim, int64_t nseg, const double *seg, double contact_eps,
                  double merge_tol, int dir_lo, int dir_hi, double band, int brute,
                  orc_net **out) {
  if (dim != 2 && dim != 3) return orc_fail(ORC_EINVAL, "dim must be 2 or 3");
  if (nseg < 0 || (nseg > 0 && !seg)) return orc_fail(ORC_EINVAL, "bad segments");
  if (!(merge_tol > 0.0)) return orc_fail(ORC_EINVAL, "merge_tol must be > 0");
  double eps = dim == 3 ? contact_eps : 0.0;
  if (dim == 3 && !(eps > 0.0)) return orc_fail(ORC_EINVAL, "contact_eps must be > 0 in 3D");

  /* 1. clip every segment to the unit box; keep the survivors in input order */
  double *SA = zalloc((size_t)(nseg ? nseg : 1) * dim, sizeof(double));
  double *SB = zalloc((size_t)(nseg ? nseg : 1) * dim, sizeof(double));
  int64_t S = 0;
  for (int64_t i = 0; i < nseg; i++) {
    const double *a = seg + (size_t)i * 2 * dim;
    const double *b = a + dim;
    if (clip_segment(dim, a, b, merge_tol, SA + S * dim, SB + S * dim)) S++;
  }

  /* 2. crossings between pairs (i < j) of kept segments */
  crossing *cr = NULL;
  int64_t ncr = 0, capcr = 0;
#define PUSH_CROSSING(C)                                                  \
  do {                                                                    \
    if (ncr == capcr) {                                                   \
      capcr = capcr ? 2 * capcr : 1024;                                   \
      cr = realloc(cr, (size_t)capcr * sizeof(crossing));                 \
      if (!cr) abort();                                                   \
    }                                                                     \
    cr[ncr++] = (C);                                                      \
  } while (0)

  if (brute) {
    for (int64_t i = 0; i < S; i++)
      for (int64_t j = i + 1; j < S; j++) {
        crossing c;
        int hit = dim == 2 ? cross2d(SA + i * 2, SB + i * 2, SA + j * 2, SB + j * 2, &c)
                           : contact3d(SA + i * 3, SB + i * 3, SA + j * 3, SB + j * 3, eps, &c);
        if (hit) {
          c.i = i;
          c.j = j;
          PUSH_CROSSING(c);
        }
      }
  } else {
    /* cells of side h >= (longest kept segment + eps) over the segment
     * midpoints: two segments closer than eps have midpoints in the same or
     * in neighbouring cells */
    double maxlen = 0.0;
    for (int64_t i = 0; i < S; i++) {
      double l = sqrt(dist2(dim, SA + i * dim, SB + i * dim));
      if (l > maxlen) maxlen = l;
    }
    int64_t nc = (int64_t)floor(1.0 / (maxlen + eps));
    if (nc < 1) nc = 1;
    if (nc > (dim == 2 ? 1024 : 128)) nc = dim == 2 ? 1024 : 128;
    int64_t ncell = 1;
    for (int k = 0; k < dim; k++) ncell *= nc;
    int64_t *cell_of = zalloc((size_t)(S ? S : 1), sizeof(int64_t));
    int64_t *cell_cnt = zalloc((size_t)ncell + 1, sizeof(int64_t));
    for (int64_t i = 0; i < S; i++) {
      int64_t c = 0, mul = 1;
      for (int k = 0; k < dim; k++) {
        double m = 0.5 * (SA[i * dim + k] + SB[i * dim + k]);
        int64_t ck = (int64_t)floor(m * (double)nc);
        if (ck < 0) ck = 0;
        if (ck > nc - 1) ck = nc - 1;
        c += ck * mul;
        mul *= nc;
      }
      cell_of[i] = c;
      cell_cnt[c + 1]++;
    }
    for (int64_t c = 0; c < ncell; c++) cell_cnt[c + 1] += cell_cnt[c];
    int64_t *cell_seg = zalloc((size_t)(S ? S : 1), sizeof(int64_t));
    int64_t *fillp = zalloc((size_t)ncell, sizeof(int64_t));
    for (int64_t i = 0; i < S; i++) cell_seg[cell_cnt[cell_of[i]] + fillp[cell_of[i]]++] = i;
    for (int64_t i = 0; i < S; i++) {
      int64_t ci[3] = {0, 0, 0}, rem = cell_of[i];
      for (int k = 0; k < dim; k++) {
        ci[k] = rem % nc;
        rem /= nc;
      }
      int64_t lo[3], hi[3];
      for (int k = 0; k < 3; k++) {
        lo[k] = (k < dim && ci[k] > 0) ? ci[k] - 1 : ci[k];
        hi[k] = (k < dim && ci[k] < nc - 1) ? ci[k] + 1 : ci[k];
      }
      for (int64_t z = lo[2]; z <= hi[2]; z++)
        for (int64_t y = lo[1]; y <= hi[1]; y++)
          for (int64_t xk = lo[0]; xk <= hi[0]; xk++) {
            int64_t c = xk + nc * (y + nc * z);
            if (dim == 2) c = xk + nc * y;
            for (int64_t q = cell_cnt[c]; q < cell_cnt[c + 1]; q++) {
              int64_t j = cell_seg[q];
              if (j <= i) continue;
              crossing cc;
              int hit = dim == 2 ? cross2d(SA + i * 2, SB + i * 2, SA + j * 2, SB + j * 2, &cc)
                                 : contact3d(SA + i * 3, SB + i * 3, SA + j * 3, SB + j * 3, eps, &cc);
              if (hit) {
                cc.i = i;
                cc.j = j;
                PUSH_CROSSING(cc);
              }
            }
          }
    }
    free(cell_of);
    free(cell_cnt);
    free(cell_seg);
    free(fillp);
    qsort(cr, (size_t)ncr, sizeof(crossing), cmp_crossing);
  }
#undef PUSH_CROSSING

  /* 3. raw nodes: endpoints 2s, 2s+1, then crossings in (i, j) order */
  int64_t NR = 2 * S + ncr;
  double *X = zalloc((size_t)(NR ? NR : 1) * dim, sizeof(double));
  for (int64_t s = 0; s < S; s++)
    for (int k = 0; k < dim; k++) {
      X[(2 * s) * dim + k] = SA[s * dim + k];
      X[(2 * s + 1) * dim + k] = SB[s * dim + k];
    }
  for (int64_t c = 0; c < ncr; c++)
    for (int k = 0; k < dim; k++) X[(2 * S + c) * dim + k] = cr[c].p[k];

  /* 4. edges along each segment between consecutive nodes, ordered by the
   *    parameter along the segment (ties by node id) */
  int64_t *cnt = zalloc((size_t)S + 1, sizeof(int64_t));
  for (int64_t c = 0; c < ncr; c++) {
    cnt[cr[c].i + 1]++;
    cnt[cr[c].j + 1]++;
  }
  for (int64_t s = 0; s < S; s++) cnt[s + 1] += cnt[s];
  param_node *pn = zalloc((size_t)(2 * ncr + 1), sizeof(param_node));
  int64_t *fill = zalloc((size_t)S + 1, sizeof(int64_t));
  for (int64_t c = 0; c < ncr; c++) {
    int64_t i = cr[c].i, j = cr[c].j;
    pn[cnt[i] + fill[i]++] = (param_node){cr[c].ti, 2 * S + c};
    pn[cnt[j] + fill[j]++] = (param_node){cr[c].tj, 2 * S + c};
  }
  ivec eu = {0}, ev = {0};
  param_node *buf = zalloc((size_t)(2 * ncr + 3), sizeof(param_node));
  for (int64_t s = 0; s < S; s++) {
    int64_t m = 0;
    buf[m++] = (param_node){0.0, 2 * s};
    buf[m++] = (param_node){1.0, 2 * s + 1};
    for (int64_t q = cnt[s]; q < cnt[s + 1]; q++) buf[m++] = pn[q];
    qsort(buf, (size_t)m, sizeof(param_node), cmp_param_node);
    for (int64_t q = 0; q + 1 < m; q++) {
      ivec_push(&eu, buf[q].id);
      ivec_push(&ev, buf[q + 1].id);
    }
  }
  free(buf);
  free(pn);
  free(fill);
  free(cnt);

  /* 5. merge nodes closer than merge_tol (sweep over the first coordinate) */
  int64_t *par = zalloc((size_t)(NR ? NR : 1), sizeof(int64_t));
  for (int64_t i = 0; i < NR; i++) par[i] = i;
  key_id *order = zalloc((size_t)(NR ? NR : 1), sizeof(key_id));
  for (int64_t i = 0; i < NR; i++) order[i] = (key_id){X[i * dim], i};
  qsort(order, (size_t)NR, sizeof(key_id), cmp_key_id);
  double tol2 = merge_tol * merge_tol;
  for (int64_t a = 0; a < NR; a++) {
    int64_t p = order[a].id;
    for (int64_t b = a + 1; b < NR; b++) {
      int64_t q = order[b].id;
      if (!(X[q * dim] - X[p * dim] < merge_tol)) break;
      if (dist2(dim, X + p * dim, X + q * dim) < tol2) uf_union(par, p, q);
    }
  }
  free(order);

  /* edges between representatives; self loops dropped */
  ivec fu = {0}, fv = {0};
  for (int64_t k = 0; k < eu.n; k++) {
    int64_t a = uf_find(par, eu.a[k]), b = uf_find(par, ev.a[k]);
    if (a == b) continue;
    ivec_push(&fu, a);
    ivec_push(&fv, b);
  }
  free(eu.a);
  free(ev.a);

  /* 6. largest connected component (ties: the one holding the smallest id) */
  int64_t *comp = zalloc((size_t)(NR ? NR : 1), sizeof(int64_t));
  for (int64_t i = 0; i < NR; i++) comp[i] = i;
  for (int64_t k = 0; k < fu.n; k++) uf_union(comp, fu.a[k], fv.a[k]);
  int64_t *csize = zalloc((size_t)(NR ? NR : 1), sizeof(int64_t));
  for (int64_t i = 0; i < NR; i++)
    if (uf_find(par, i) == i) csize[uf_find(comp, i)]++;
  int64_t best = -1;
  for (int64_t i = 0; i < NR; i++)
    if (csize[i] > 0 && (best < 0 || csize[i] > csize[best])) best = i;
  int64_t *newid = zalloc((size_t)(NR ? NR : 1), sizeof(int64_t));
  int64_t N = 0;
  for (int64_t i = 0; i < NR; i++) {
    newid[i] = -1;
    if (best >= 0 && uf_find(par, i) == i && uf_find(comp, i) == best) newid[i] = N++;
  }

  orc_net *net = zalloc(1, sizeof(orc_net));
  net->dim = dim;
  net->n_nodes = N;
  net->n_segments_kept = S;
  net->n_raw_nodes = NR;
  net->x = zalloc((size_t)(N ? N : 1) * dim, sizeof(double));
  net->dir = zalloc((size_t)(N ? N : 1), sizeof(uint8_t));
  for (int64_t i = 0; i < NR; i++)
    if (newid[i] >= 0)
      for (int k = 0; k < dim; k++) net->x[newid[i] * dim + k] = X[i * dim + k];
  int64_t E = 0;
  for (int64_t k = 0; k < fu.n; k++)
    if (newid[fu.a[k]] >= 0) E++;
  net->n_edges = E;
  net->e = zalloc((size_t)(E ? E : 1) * 2, sizeof(int32_t));
  E = 0;
  for (int64_t k = 0; k < fu.n; k++)
    if (newid[fu.a[k]] >= 0) {
      net->e[2 * E] = (int32_t)newid[fu.a[k]];
      net->e[2 * E + 1] = (int32_t)newid[fv.a[k]];
      E++;
    }

  /* 7. Dirichlet set: nodes within band of a Gamma face */
  for (int64_t i = 0; i < N; i++) {
    int d = 0;
    for (int k = 0; k < dim; k++) {
      double v = net->x[i * dim + k];
      if (((dir_lo >> k) & 1) && v <= band) d = 1;
      if (((dir_hi >> k) & 1) && v >= 1.0 - band) d = 1;
    }
    net->dir[i] = (uint8_t)d;
  }

  free(fu.a);
  free(fv.a);
  free(comp);
  free(csize);
  free(newid);
  free(par);
  free(X);
  free(cr);
  free(SA);
  free(SB);
  *out = net;
  return ORC_OK;
}

/* a network given directly (nodes, edges, Dirichlet flags), e.g. the grid network of Example 3.7 */
int orc_net_from_arrays(int dim, int64_t n_nodes, const double *x, int64_t n_edges,
                        const int32_t *e, const uint8_t *dir, orc_net **out) {
  if (dim != 2 && dim != 3) return orc_fail(ORC_EINVAL, "dim must be 2 or 3");
  for (int64_t k = 0; k < 2 * n_edges; k++)
    if (e[k] < 0 || e[k] >= n_nodes) return orc_fail(ORC_EINVAL, "edge end out of range");
  orc_net *net = zalloc(1, sizeof(orc_net));
  net->dim = dim;
  net->n_nodes = n_nodes;
  net->n_edges = n_edges;
  net->x = zalloc((size_t)(n_nodes ? n_nodes : 1) * dim, sizeof(double));
  net->e = zalloc((size_t)(n_edges ? n_edges : 1) * 2, sizeof(int32_t));
  net->dir = zalloc((size_t)(n_nodes ? n_nodes : 1), 1);
  memcpy(net->x, x, (size_t)n_nodes * dim * sizeof(double));
  memcpy(net->e, e, (size_t)n_edges * 2 * sizeof(int32_t));
  memcpy(net->dir, dir, (size_t)n_nodes);
  *out = net;
  return ORC_OK;
}

void orc_net_sizes(const orc_net *n, int64_t *n_nodes, int64_t *n_edges, int64_t *n_seg_kept,
                   int64_t *n_raw_nodes) {
  *n_nodes = n->n_nodes;
  *n_edges = n->n_edges;
  *n_seg_kept = n->n_segments_kept;
  *n_raw_nodes = n->n_raw_nodes;
}

void orc_net_get(const orc_net *n, double *x, int32_t *e, uint8_t *dir) {
  if (x) memcpy(x, n->x, (size_t)n->n_nodes * n->dim * sizeof(double));
  if (e) memcpy(e, n->e, (size_t)n->n_edges * 2 * sizeof(int32_t));
  if (dir) memcpy(dir, n->dir, (size_t)n->n_nodes);
}

/* ================================================================== */
/* System: K restricted to the free dofs (Sec. 2.2, Examples 3.2/3.3) */
/* ================================================================== */
typedef struct orc_sys {
  int dim, ncomp;
  int64_t n_nodes;
  int64_t n;           /* free dofs = free nodes * ncomp, node-major */
  int64_t nnz;
  int64_t *rowptr;
  int32_t *col;
  double *val;
  /* free rows of K against the dofs of the Dirichlet nodes (columns are
   * node * ncomp + component): the lifting term of non-zero Dirichlet data */
  int64_t nnz_d;
  int64_t *rowptr_d;
  int32_t *col_d;
  double *val_d;
  int32_t *node_free;  /* node -> free node index or -1 */
  int32_t *free_node;  /* free node index -> node */
  int64_t n_free_nodes;
  double *x;           /* node coordinates */
  double *mass;        /* (M 1)(x) at every node, eq. 2.1 */
} orc_sys;

typedef struct { int64_t r, c, seq; double v; } triple;
static int cmp_triple(const void *pa, const void *pb) {
  const triple *a = pa, *b = pb;
  if (a->r != b->r) return a->r < b->r ? -1 : 1;
  if (a->c != b->c) return a->c < b->c ? -1 : 1;
  if (a->seq != b->seq) return a->seq < b->seq ? -1 : 1;
  return 0;
}

void orc_sys_free(orc_sys *s) {
  if (!s) return;
  free(s->rowptr);
  free(s->col);
  free(s->val);
  free(s->rowptr_d);
  free(s->col_d);
  free(s->val_d);
  free(s->node_free);
  free(s->free_node);
  free(s->x);
  free(s->mass);
  free(s);
}

typedef struct {
  triple *T;
  int64_t n, cap;
} triples;

static void tpush(triples *t, int64_t r, int64_t c, int64_t seq, double v) {
  if (t->n == t->cap) {
    t->cap = 2 * t->cap + 1024;
    t->T = realloc(t->T, (size_t)t->cap * sizeof(triple));
    if (!t->T) {
      fprintf(stderr, "oracle: out of memory\n");
      abort();
    }
  }
  t->T[t->n++] = (triple){r, c, seq, v};
}

/* shared start of every model: free numbering, coordinates, lumped mass */
static orc_sys *sys_begin(const orc_net *net, int nc) {
  int dim = net->dim;
  orc_sys *s = zalloc(1, sizeof(orc_sys));
  s->dim = dim;
  s->ncomp = nc;
  s->n_nodes = net->n_nodes;
  s->node_free = zalloc((size_t)(net->n_nodes ? net->n_nodes : 1), sizeof(int32_t));
  s->free_node = zalloc((size_t)(net->n_nodes ? net->n_nodes : 1), sizeof(int32_t));
  int64_t nf = 0;
  for (int64_t i = 0; i < net->n_nodes; i++) {
    if (net->dir[i]) s->node_free[i] = -1;
    else {
      s->node_free[i] = (int32_t)nf;
      s->free_node[nf] = (int32_t)i;
      nf++;
    }
  }
  s->n_free_nodes = nf;
  s->n = nf * nc;
  s->x = zalloc((size_t)(net->n_nodes ? net->n_nodes : 1) * dim, sizeof(double));
  memcpy(s->x, net->x, (size_t)net->n_nodes * dim * sizeof(double));
  /* (M_x 1, 1) = 1/2 sum_{y~x} |x - y| (eq. 2.1) */
  s->mass = zalloc((size_t)(net->n_nodes ? net->n_nodes : 1), sizeof(double));
  for (int64_t k = 0; k < net->n_edges; k++) {
    int32_t u = net->e[2 * k], v = net->e[2 * k + 1];
    double len = sqrt(dist2(dim, net->x + (size_t)u * dim, net->x + (size_t)v * dim));
    s->mass[u] += 0.5 * len;
    s->mass[v] += 0.5 * len;
  }
  return s;
}

/* triples (free row, node dof column) -> K on the free dofs and the block of
 * Dirichlet columns; equal positions summed in the order of their seq */
static void sys_finish(orc_sys *s, triples *t) {
  int nc = s->ncomp;
  qsort(t->T, (size_t)t->n, sizeof(triple), cmp_triple);
  s->rowptr = zalloc((size_t)s->n + 1, sizeof(int64_t));
  s->rowptr_d = zalloc((size_t)s->n + 1, sizeof(int64_t));
  s->col = zalloc((size_t)(t->n ? t->n : 1), sizeof(int32_t));
  s->val = zalloc((size_t)(t->n ? t->n : 1), sizeof(double));
  s->col_d = zalloc((size_t)(t->n ? t->n : 1), sizeof(int32_t));
  s->val_d = zalloc((size_t)(t->n ? t->n : 1), sizeof(double));
  int64_t nnz = 0, nnz_d = 0;
  for (int64_t q = 0; q < t->n; q++) {
    const triple *a = &t->T[q];
    int same = q > 0 && a->r == t->T[q - 1].r && a->c == t->T[q - 1].c;
    int32_t fc = s->node_free[a->c / nc];
    if (fc >= 0) {
      if (same) s->val[nnz - 1] += a->v;
      else {
        s->col[nnz] = (int32_t)((int64_t)fc * nc + a->c % nc);
        s->val[nnz] = a->v;
        s->rowptr[a->r + 1]++;
        nnz++;
      }
    } else {
      if (same) s->val_d[nnz_d - 1] += a->v;
      else {
        s->col_d[nnz_d] = (int32_t)a->c;
        s->val_d[nnz_d] = a->v;
        s->rowptr_d[a->r + 1]++;
        nnz_d++;
      }
    }
  }
  for (int64_t i = 0; i < s->n; i++) {
    s->rowptr[i + 1] += s->rowptr[i];
    s->rowptr_d[i + 1] += s->rowptr_d[i];
  }
  s->nnz = nnz;
  s->nnz_d = nnz_d;
  free(t->T);
  t->T = NULL;
}

/*
 * model 0: heat conduction, (K v, v) = 1/2 sum_x sum_{y~x} gamma_xy (v(x)-v(y))^2/|x-y|
 *          (eq. 3.3). Each edge adds w (e_x - e_y)(e_x - e_y)^T with w = gamma/|e|.
 * model 1: tensile truss, n = d = 3 (eq. 3.4) plus an isotropic 1e-6/|e| term:
 *          each edge adds (1/|e|)(t t^T + 1e-6 I) in the blocks xx, yy (+) and xy, yx (-).
 * gamma may be NULL (all ones). Dirichlet rows and columns are removed (v in V).
 */
int orc_sys_build(const orc_net *net, int model, const double *gamma, orc_sys **out) {
  int dim = net->dim;
  int nc = model == 0 ? 1 : 3;
  if (model != 0 && model != 1) return orc_fail(ORC_EINVAL, "model must be 0 or 1");
  if (model == 1 && dim != 3) return orc_fail(ORC_EINVAL, "truss model needs dim 3");
  orc_sys *s = sys_begin(net, nc);
  if (s->n_free_nodes == net->n_nodes) {
    orc_sys_free(s);
    return orc_fail(ORC_ESINGULAR, "no Dirichlet node: K is singular on V");
  }
  triples t = {NULL, 0, 0};
  for (int64_t k = 0; k < net->n_edges; k++) {
    int32_t u = net->e[2 * k], v = net->e[2 * k + 1];
    const double *xu = net->x + (size_t)u * dim, *xv = net->x + (size_t)v * dim;
    double len = sqrt(dist2(dim, xv, xu));
    double g = gamma ? gamma[k] : 1.0;
    double blk[9];
    if (model == 0) {
      blk[0] = g / len;
    } else {
      double tv[3];
      for (int a = 0; a < 3; a++) tv[a] = (xv[a] - xu[a]) / len;
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
          blk[a * 3 + b] = g * (tv[a] * tv[b]) / len + (a == b ? 1e-6 / len : 0.0);
    }
    int32_t fu = s->node_free[u], fv = s->node_free[v];
    for (int a = 0; a < nc; a++)
      for (int b = 0; b < nc; b++) {
        double w = blk[a * nc + b];
        if (fu >= 0) {
          tpush(&t, (int64_t)fu * nc + a, (int64_t)u * nc + b, 4 * k, w);
          tpush(&t, (int64_t)fu * nc + a, (int64_t)v * nc + b, 4 * k + 2, -w);
        }
        if (fv >= 0) {
          tpush(&t, (int64_t)fv * nc + a, (int64_t)v * nc + b, 4 * k + 1, w);
          tpush(&t, (int64_t)fv * nc + a, (int64_t)u * nc + b, 4 * k + 3, -w);
        }
      }
  }
  sys_finish(s, &t);
  *out = s;
  return ORC_OK;
}

static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/*
 * Beam model (Example 3.3 with the constants of Sec. 6.3), n = ncomp
 * components (n = 2: in-plane problem of a 2D network, Sec. 6.3.1; n = 3: 2D
 * or 3D network). With d_xy = (x - y)/|x - y| and L_xy = |x - y|:
 *
 *   (K v, v) = sum_x 1/2 sum_{y~x} g1 ((v(x) - v(y)) . d_xy)^2 / L_xy          (eq. 3.4)
 *            + sum_x sum_{y~x, z~x, y != z} sum_k g_xyz (L_xy + L_xz)/2 a_k^2     (eq. 3.5)
 *   a_k = (v(y) - v(x)) . eta_y^k / L_xy + (v(z) - v(x)) . eta_z^k / L_xz,
 *   g_xyz = g1 r_w^2 / (4 (L_xy + L_xz)^2).
 *
 * eta^1 (k = 1, only for n = 3) is one unit vector normal to both edges: e_3
 * for a 2D network, the normalised d_xy x d_xz in 3D (any unit normal of
 * d_xy when the edges are parallel). For k = 2 this build takes
 * eta_y^2 = d_xy x eta^1 and eta_z^2 = eta^1 x d_xz: the printed
 * eta_w^2 = d_xw x eta^1 for both edges would make a_2 twice the rotation of
 * a rigid motion about eta^1, while with the second sign flipped a_2 is the
 * change of the angle between the two edges (zero for rigid motions) and, on
 * a straight fiber, its curvature. The pair sum runs over ordered pairs, as
 * printed. Every term is a rank-one element w c c^T on the dofs of x, y, z.
 */
int orc_sys_build_beam(const orc_net *net, int ncomp, double gamma1, double r_w, orc_sys **out) {
  int dim = net->dim;
  if (ncomp != 2 && ncomp != 3) return orc_fail(ORC_EINVAL, "beam model needs 2 or 3 components");
  if (ncomp == 2 && dim != 2) return orc_fail(ORC_EINVAL, "2 components need a 2D network");
  if (!(gamma1 > 0.0) || !(r_w >= 0.0)) return orc_fail(ORC_EINVAL, "beam constants must be positive");
  int nc = ncomp;
  orc_sys *s = sys_begin(net, nc);
  if (s->n_free_nodes == net->n_nodes) {
    orc_sys_free(s);
    return orc_fail(ORC_ESINGULAR, "no Dirichlet node: K is singular on V");
  }
  int64_t N = net->n_nodes, E = net->n_edges;
  /* neighbours of every node, in edge order */
  int64_t *nb0 = zalloc((size_t)N + 1, sizeof(int64_t));
  for (int64_t k = 0; k < E; k++) {
    nb0[net->e[2 * k] + 1]++;
    nb0[net->e[2 * k + 1] + 1]++;
  }
  for (int64_t i = 0; i < N; i++) nb0[i + 1] += nb0[i];
  int32_t *nb = zalloc((size_t)(nb0[N] ? nb0[N] : 1), sizeof(int32_t));
  int64_t *fillp = zalloc((size_t)(N ? N : 1), sizeof(int64_t));
  for (int64_t k = 0; k < E; k++) {
    int32_t u = net->e[2 * k], v = net->e[2 * k + 1];
    nb[nb0[u] + fillp[u]++] = v;
    nb[nb0[v] + fillp[v]++] = u;
  }
  free(fillp);
  triples t = {NULL, 0, 0};
  int64_t seq = 0;
  /* tensile part, eq. 3.4: each edge adds g1/L (d d^T) in the blocks uu, vv and minus it in uv, vu */
  for (int64_t k = 0; k < E; k++) {
    int32_t u = net->e[2 * k], v = net->e[2 * k + 1];
    double d[3] = {0.0, 0.0, 0.0};
    double len = sqrt(dist2(dim, net->x + (size_t)u * dim, net->x + (size_t)v * dim));
    for (int a = 0; a < dim; a++) d[a] = (net->x[(size_t)u * dim + a] - net->x[(size_t)v * dim + a]) / len;
    int32_t ends[2] = {u, v};
    for (int p = 0; p < 2; p++) {
      int32_t row_node = ends[p];
      int32_t f = s->node_free[row_node];
      if (f < 0) continue;
      for (int q = 0; q < 2; q++) {
        double sg = p == q ? 1.0 : -1.0;
        for (int a = 0; a < nc; a++)
          for (int b = 0; b < nc; b++)
            tpush(&t, (int64_t)f * nc + a, (int64_t)ends[q] * nc + b, seq, sg * gamma1 * d[a] * d[b] / len);
      }
    }
    seq++;
  }
  /* bending part, eq. 3.5 */
  for (int64_t x = 0; x < N; x++) {
    const double *px = net->x + (size_t)x * dim;
    for (int64_t iy = nb0[x]; iy < nb0[x + 1]; iy++)
      for (int64_t iz = nb0[x]; iz < nb0[x + 1]; iz++) {
        int32_t y = nb[iy], z = nb[iz];
        if (y == z) continue;
        const double *py = net->x + (size_t)y * dim, *pz = net->x + (size_t)z * dim;
        double dy[3] = {0.0, 0.0, 0.0}, dz[3] = {0.0, 0.0, 0.0};
        double ly = sqrt(dist2(dim, px, py)), lz = sqrt(dist2(dim, px, pz));
        for (int a = 0; a < dim; a++) {
          dy[a] = (px[a] - py[a]) / ly;
          dz[a] = (px[a] - pz[a]) / lz;
        }
        double e1[3] = {0.0, 0.0, 1.0};
        if (dim == 3) {
          cross3(dy, dz, e1);
          double nn = sqrt(dot3(3, e1, e1));
          if (nn > 1e-12) {
            for (int a = 0; a < 3; a++) e1[a] /= nn;
          } else {
            /* parallel edges: the axis least aligned with d_xy, made normal to it */
            int am = 0;
            for (int a = 1; a < 3; a++)
              if (fabs(dy[a]) < fabs(dy[am])) am = a;
            double ax[3] = {0.0, 0.0, 0.0};
            ax[am] = 1.0;
            cross3(dy, ax, e1);
            nn = sqrt(dot3(3, e1, e1));
            for (int a = 0; a < 3; a++) e1[a] /= nn;
          }
        }
        double ey[2][3], ez[2][3];
        for (int a = 0; a < 3; a++) ey[0][a] = ez[0][a] = e1[a];
        cross3(dy, e1, ey[1]);
        cross3(e1, dz, ez[1]);
        double w = gamma1 * r_w * r_w / (4.0 * (ly + lz) * (ly + lz)) * (ly + lz) / 2.0;
        int32_t nodes[3] = {(int32_t)x, y, z};
        for (int kk = (nc == 3 ? 0 : 1); kk < 2; kk++) {
          /* c over (x, y, z) x components */
          double c[3][3];
          for (int a = 0; a < nc; a++) {
            c[1][a] = ey[kk][a] / ly;
            c[2][a] = ez[kk][a] / lz;
            c[0][a] = -(c[1][a] + c[2][a]);
          }
          for (int p = 0; p < 3; p++) {
            int32_t f = s->node_free[nodes[p]];
            if (f < 0) continue;
            for (int q = 0; q < 3; q++)
              for (int a = 0; a < nc; a++)
                for (int b = 0; b < nc; b++)
                  tpush(&t, (int64_t)f * nc + a, (int64_t)nodes[q] * nc + b, seq, w * c[p][a] * c[q][b]);
          }
          seq++;
        }
      }
  }
  free(nb0);
  free(nb);
  sys_finish(s, &t);
  *out = s;
  return ORC_OK;
}

/* y = (K g) on the free rows, g given on every node (n_nodes x ncomp): the
 * term a non-zero Dirichlet lifting moves to the right-hand side (Sec. 6.3) */
void orc_sys_apply_full(const orc_sys *s, const double *g, double *y) {
  int nc = s->ncomp;
  for (int64_t i = 0; i < s->n; i++) {
    double acc = 0.0;
    for (int64_t q = s->rowptr[i]; q < s->rowptr[i + 1]; q++) {
      int64_t fc = s->col[q] / nc, comp = s->col[q] % nc;
      acc += s->val[q] * g[(int64_t)s->free_node[fc] * nc + comp];
    }
    for (int64_t q = s->rowptr_d[i]; q < s->rowptr_d[i + 1]; q++) acc += s->val_d[q] * g[s->col_d[q]];
    y[i] = acc;
  }
}

/* (M 1)(x) at every free node (eq. 2.1) */
void orc_sys_mass(const orc_sys *s, double *m) {
  for (int64_t f = 0; f < s->n_free_nodes; f++) m[f] = s->mass[s->free_node[f]];
}

void orc_sys_sizes(const orc_sys *s, int64_t *n, int64_t *nnz, int64_t *n_free_nodes) {
  *n = s->n;
  *nnz = s->nnz;
  *n_free_nodes = s->n_free_nodes;
}

void orc_sys_get_csr(const orc_sys *s, int64_t *rowptr, int32_t *col, double *val) {
  if (rowptr) memcpy(rowptr, s->rowptr, (size_t)(s->n + 1) * sizeof(int64_t));
  if (col) memcpy(col, s->col, (size_t)s->nnz * sizeof(int32_t));
  if (val) memcpy(val, s->val, (size_t)s->nnz * sizeof(double));
}

void orc_sys_get_free_nodes(const orc_sys *s, int32_t *free_node) {
  memcpy(free_node, s->free_node, (size_t)s->n_free_nodes * sizeof(int32_t));
}

/* y = K x */
void orc_apply_K(const orc_sys *s, const double *x, double *y) {
  for (int64_t i = 0; i < s->n; i++) {
    double acc = 0.0;
    for (int64_t q = s->rowptr[i]; q < s->rowptr[i + 1]; q++) acc += s->val[q] * x[s->col[q]];
    y[i] = acc;
  }
}

/* ================================================================== */
/* Envelope Cholesky (George & Liu), used for every local and the      */
/* coarse direct solve ("direct solution of decoupled local linear     */
/* systems and one coarse scale linear system", Sec. 4.1).             */
/* ================================================================== */
typedef struct {
  int64_t n;
  int32_t *perm;     /* position -> original local index */
  int64_t *rowoff;   /* row i holds columns first[i]..i at L[rowoff[i] + c - first[i]] */
  int32_t *first;
  double *L;
} env_factor;

static void env_free(env_factor *F) {
  free(F->perm);
  free(F->rowoff);
  free(F->first);
  free(F->L);
  memset(F, 0, sizeof *F);
}

static double *env_at(env_factor *F, int64_t i, int64_t c) { return F->L + F->rowoff[i] + (c - F->first[i]); }

/* allocate the envelope given first[], zero it */
static void env_alloc(env_factor *F) {
  F->rowoff = zalloc((size_t)F->n + 1, sizeof(int64_t));
  for (int64_t i = 0; i < F->n; i++) F->rowoff[i + 1] = F->rowoff[i] + (i - F->first[i] + 1);
  F->L = zalloc((size_t)(F->rowoff[F->n] ? F->rowoff[F->n] : 1), sizeof(double));
}

/* in-place Cholesky by the bordering method, row by row */
static int env_factorize(env_factor *F) {
  for (int64_t i = 0; i < F->n; i++) {
    int64_t fi = F->first[i];
    for (int64_t j = fi; j < i; j++) {
      int64_t fj = F->first[j];
      int64_t k0 = fi > fj ? fi : fj;
      double s = *env_at(F, i, j);
      for (int64_t k = k0; k < j; k++) s -= *env_at(F, i, k) * *env_at(F, j, k);
      *env_at(F, i, j) = s / *env_at(F, j, j);
    }
    double d = *env_at(F, i, i);
    for (int64_t k = fi; k < i; k++) d -= *env_at(F, i, k) * *env_at(F, i, k);
    if (!(d > 0.0)) return -1 - (int)(i & 0x3fffffff);
    *env_at(F, i, i) = sqrt(d);
  }
  return 0;
}

/* solve (L L^T) y = y in place, in the factor's own ordering */
static void env_solve_inplace(const env_factor *F, double *y) {
  for (int64_t i = 0; i < F->n; i++) {
    const double *Li = F->L + F->rowoff[i];
    double s = y[i];
    for (int64_t k = F->first[i]; k < i; k++) s -= Li[k - F->first[i]] * y[k];
    y[i] = s / Li[i - F->first[i]];
  }
  for (int64_t i = F->n - 1; i >= 0; i--) {
    const double *Li = F->L + F->rowoff[i];
    y[i] = y[i] / Li[i - F->first[i]];
    for (int64_t k = F->first[i]; k < i; k++) y[k] -= Li[k - F->first[i]] * y[i];
  }
}

/*
 * Reverse Cuthill-McKee ordering of a symmetric local graph given in CSR
 * (diagonal entries ignored). Each connected piece starts from an unvisited
 * vertex of least degree (ties: smallest index); neighbours are queued by
 * increasing degree (ties: smallest index). perm[position] = vertex.
 */
typedef struct { int64_t deg, id; } deg_id;
static int cmp_deg_id(const void *pa, const void *pb) {
  const deg_id *a = pa, *b = pb;
  if (a->deg != b->deg) return a->deg < b->deg ? -1 : 1;
  if (a->id != b->id) return a->id < b->id ? -1 : 1;
  return 0;
}
static void rcm_order(int64_t n, const int64_t *ap, const int32_t *ai, int32_t *perm) {
  int64_t *deg = zalloc((size_t)(n ? n : 1), sizeof(int64_t));
  for (int64_t v = 0; v < n; v++)
    for (int64_t q = ap[v]; q < ap[v + 1]; q++)
      if (ai[q] != v) deg[v]++;
  char *seen = zalloc((size_t)(n ? n : 1), 1);
  int32_t *cm = zalloc((size_t)(n ? n : 1), sizeof(int32_t));
  deg_id *nb = zalloc((size_t)(n ? n : 1), sizeof(deg_id));
  int64_t head = 0, tail = 0;
  while (tail < n) {
    int64_t start = -1;
    for (int64_t v = 0; v < n; v++)
      if (!seen[v] && (start < 0 || deg[v] < deg[start])) start = v;
    seen[start] = 1;
    cm[tail++] = (int32_t)start;
    while (head < tail) {
      int64_t v = cm[head++];
      int64_t m = 0;
      for (int64_t q = ap[v]; q < ap[v + 1]; q++) {
        int64_t w = ai[q];
        if (w != v && !seen[w]) {
          seen[w] = 1;
          nb[m++] = (deg_id){deg[w], w};
        }
      }
      qsort(nb, (size_t)m, sizeof(deg_id), cmp_deg_id);
      for (int64_t k = 0; k < m; k++) cm[tail++] = (int32_t)nb[k].id;
    }
  }
  for (int64_t k = 0; k < n; k++) perm[k] = cm[n - 1 - k];
  free(deg);
  free(seen);
  free(cm);
  free(nb);
}

/* ================================================================== */
/* Coarse space V_H and local spaces V_j = V(U(y_j)) (Sec. 2.3, 4.1)   */
/* ================================================================== */
typedef struct orc_pre {
  const orc_sys *sys;
  int dim, ncomp, nH, policy;
  int64_t nvert;          /* (nH+1)^d mesh nodes y_k, x index fastest */
  int64_t m0;             /* coarse dofs = kept vertices * ncomp */
  int32_t *cvert;         /* kept vertex -> vertex id */
  int32_t *vert_c;        /* vertex id -> kept vertex index or -1 */
  /* P restricted to free nodes: for free node f, 2^d (vertex, phi) pairs */
  int32_t *Pvert;
  double *Pphi;
  int64_t nstars;
  int64_t *star_ptr;      /* dof lists, ascending */
  int32_t *star_dofs;
  int32_t *star_vertex;
  env_factor *sf;         /* star factors */
  env_factor cf;          /* coarse factor */
  double *K0dense;        /* optional, only when m0 is small (for tests) */
  int factored;
} orc_pre;

void orc_pre_free(orc_pre *p) {
  if (!p) return;
  free(p->cvert);
  free(p->vert_c);
  free(p->Pvert);
  free(p->Pphi);
  free(p->star_ptr);
  free(p->star_dofs);
  free(p->star_vertex);
  if (p->sf) {
    for (int64_t s = 0; s < p->nstars; s++) env_free(&p->sf[s]);
    free(p->sf);
  }
  env_free(&p->cf);
  free(p->K0dense);
  free(p);
}

/* element index e_k(x) = min(floor(x_k nH), nH-1): the half-open boxes of
 * T_H, closed at the upper face of Omega (Sec. 2.3) */
static int64_t elem_index(double xk, int nH) {
  int64_t e = (int64_t)floor(xk * (double)nH);
  if (e > nH - 1) e = nH - 1;
  if (e < 0) e = 0;
  return e;
}

static int vertex_on_gamma(const int64_t *v, int dim, int nH, int dir_lo, int dir_hi) {
  for (int k = 0; k < dim; k++) {
    if (((dir_lo >> k) & 1) && v[k] == 0) return 1;
    if (((dir_hi >> k) & 1) && v[k] == nH) return 1;
  }
  return 0;
}

/*
 * nH = 1/H elements per axis; policy 0 (ALL): one local space per mesh node
 * y_j, j = 1..m, as in Sec. 4.1; policy 1 (FREE): only mesh nodes off Gamma.
 * Local spaces with no free dof are dropped.
 */
int orc_pre_build(const orc_sys *s, int nH, int policy, int dir_lo, int dir_hi, orc_pre **out) {
  if (nH < 1) return orc_fail(ORC_EINVAL, "nH must be >= 1");
  int dim = s->dim, nc = s->ncomp, nv = 1 << dim;
  orc_pre *p = zalloc(1, sizeof(orc_pre));
  p->sys = s;
  p->dim = dim;
  p->ncomp = nc;
  p->nH = nH;
  p->policy = policy;
  p->nvert = 1;
  for (int k = 0; k < dim; k++) p->nvert *= (nH + 1);
  int64_t nf = s->n_free_nodes;

  /* Q1 basis values at every free node: phi_v(x) = prod_k (b_k ? xi_k : 1 - xi_k);
   * supp[f, b] = 1 when every factor is positive, i.e. x lies in the open
   * patch |x_k nH - v_k| < 1 of the mesh node v = e + b */
  p->Pvert = zalloc((size_t)(nf ? nf : 1) * nv, sizeof(int32_t));
  p->Pphi = zalloc((size_t)(nf ? nf : 1) * nv, sizeof(double));
  char *supp = zalloc((size_t)(nf ? nf : 1) * nv, 1);
  int64_t *eidx = zalloc((size_t)(nf ? nf : 1) * dim, sizeof(int64_t));
  for (int64_t f = 0; f < nf; f++) {
    const double *x = s->x + (size_t)s->free_node[f] * dim;
    int64_t e[3];
    double xi[3];
    for (int k = 0; k < dim; k++) {
      e[k] = elem_index(x[k], nH);
      xi[k] = x[k] * (double)nH - (double)e[k];
      eidx[f * dim + k] = e[k];
    }
    for (int b = 0; b < nv; b++) {
      int64_t vid = 0, mul = 1;
      double phi = 1.0;
      int pos = 1;
      for (int k = 0; k < dim; k++) {
        int bk = (b >> k) & 1;
        vid += (e[k] + bk) * mul;
        mul *= (nH + 1);
        phi = phi * (bk ? xi[k] : 1.0 - xi[k]);
        if (bk ? !(xi[k] > 0.0) : !(xi[k] < 1.0)) pos = 0;
      }
      p->Pvert[f * nv + b] = (int32_t)vid;
      p->Pphi[f * nv + b] = phi;
      supp[f * nv + b] = (char)pos;
    }
  }

  /* coarse dofs: vertices off Gamma whose restricted basis function is non-zero somewhere */
  char *nonzero = zalloc((size_t)p->nvert, 1);
  for (int64_t q = 0; q < nf * nv; q++)
    if (supp[q]) nonzero[p->Pvert[q]] = 1;
  p->vert_c = zalloc((size_t)p->nvert, sizeof(int32_t));
  p->cvert = zalloc((size_t)p->nvert, sizeof(int32_t));
  int64_t nk = 0;
  for (int64_t vid = 0; vid < p->nvert; vid++) {
    int64_t v[3] = {0, 0, 0}, rem = vid;
    for (int k = 0; k < dim; k++) {
      v[k] = rem % (nH + 1);
      rem /= (nH + 1);
    }
    p->vert_c[vid] = -1;
    if (!vertex_on_gamma(v, dim, nH, dir_lo, dir_hi) && nonzero[vid]) {
      p->vert_c[vid] = (int32_t)nk;
      p->cvert[nk++] = (int32_t)vid;
    }
  }
  p->m0 = nk * nc;
  free(nonzero);

  /* local spaces: S_v = free nodes at which phi_v is positive, i.e. the
   * network nodes inside the support of the basis function of y_v (the mesh
   * star; Sec. 4.1 with the support of phi_k taken as U(y_k), as in Sec. 5),
   * expanded to their dofs. A node strictly inside an element lies in the 2^d
   * stars of that element's vertices; a node on a face of T_H only in those
   * of the vertices of that face. */
  int64_t *cnt = zalloc((size_t)p->nvert + 1, sizeof(int64_t));
  for (int64_t f = 0; f < nf; f++)
    for (int b = 0; b < nv; b++)
      if (supp[f * nv + b]) cnt[p->Pvert[f * nv + b] + 1]++;
  for (int64_t vid = 0; vid < p->nvert; vid++) cnt[vid + 1] += cnt[vid];
  int32_t *members = zalloc((size_t)(nf > 0 ? nf * nv : 1), sizeof(int32_t));
  int64_t *fillv = zalloc((size_t)p->nvert, sizeof(int64_t));
  for (int64_t f = 0; f < nf; f++)
    for (int b = 0; b < nv; b++) {
      if (!supp[f * nv + b]) continue;
      int32_t vid = p->Pvert[f * nv + b];
      members[cnt[vid] + fillv[vid]++] = (int32_t)f;  /* ascending f */
    }
  p->star_ptr = zalloc((size_t)p->nvert + 1, sizeof(int64_t));
  p->star_vertex = zalloc((size_t)p->nvert, sizeof(int32_t));
  p->star_dofs = zalloc((size_t)(nf > 0 ? nf * nv * nc : 1), sizeof(int32_t));
  int64_t ns = 0, tot = 0;
  for (int64_t vid = 0; vid < p->nvert; vid++) {
    int64_t v[3] = {0, 0, 0}, rem = vid;
    for (int k = 0; k < dim; k++) {
      v[k] = rem % (nH + 1);
      rem /= (nH + 1);
    }
    if (policy == 1 && vertex_on_gamma(v, dim, nH, dir_lo, dir_hi)) continue;
    if (cnt[vid + 1] == cnt[vid]) continue;
    p->star_vertex[ns] = (int32_t)vid;
    for (int64_t q = cnt[vid]; q < cnt[vid + 1]; q++)
      for (int c = 0; c < nc; c++) p->star_dofs[tot++] = members[q] * nc + c;
    ns++;
    p->star_ptr[ns] = tot;
  }
  p->nstars = ns;
  free(cnt);
  free(members);
  free(fillv);
  free(eidx);
  free(supp);
  *out = p;
  return ORC_OK;
}

void orc_pre_sizes(const orc_pre *p, int64_t *m0, int64_t *nstars, int64_t *star_total) {
  *m0 = p->m0;
  *nstars = p->nstars;
  *star_total = p->star_ptr[p->nstars];
}

void orc_pre_get_stars(const orc_pre *p, int64_t *star_ptr, int32_t *star_dofs, int32_t *star_vertex) {
  if (star_ptr) memcpy(star_ptr, p->star_ptr, (size_t)(p->nstars + 1) * sizeof(int64_t));
  if (star_dofs) memcpy(star_dofs, p->star_dofs, (size_t)p->star_ptr[p->nstars] * sizeof(int32_t));
  if (star_vertex) memcpy(star_vertex, p->star_vertex, (size_t)p->nstars * sizeof(int32_t));
}

void orc_pre_get_coarse_vertices(const orc_pre *p, int32_t *cvert) {
  memcpy(cvert, p->cvert, (size_t)(p->m0 / p->ncomp) * sizeof(int32_t));
}

/* dense P (n x m0), for tests on small systems */
void orc_pre_get_P_dense(const orc_pre *p, double *Pd) {
  int nv = 1 << p->dim, nc = p->ncomp;
  memset(Pd, 0, (size_t)p->sys->n * p->m0 * sizeof(double));
  for (int64_t f = 0; f < p->sys->n_free_nodes; f++)
    for (int b = 0; b < nv; b++) {
      int32_t kv = p->vert_c[p->Pvert[f * nv + b]];
      if (kv < 0) continue;
      for (int c = 0; c < nc; c++)
        Pd[(f * nc + c) * p->m0 + (int64_t)kv * nc + c] += p->Pphi[f * nv + b];
    }
}

/* r_H = P^T r */
static void restrict_P(const orc_pre *p, const double *r, double *rH) {
  int nv = 1 << p->dim, nc = p->ncomp;
  memset(rH, 0, (size_t)(p->m0 ? p->m0 : 1) * sizeof(double));
  for (int64_t f = 0; f < p->sys->n_free_nodes; f++)
    for (int b = 0; b < nv; b++) {
      int32_t kv = p->vert_c[p->Pvert[f * nv + b]];
      if (kv < 0) continue;
      for (int c = 0; c < nc; c++) rH[(int64_t)kv * nc + c] += p->Pphi[f * nv + b] * r[f * nc + c];
    }
}

/* z += P c */
static void prolong_P_add(const orc_pre *p, const double *c, double *z) {
  int nv = 1 << p->dim, nc = p->ncomp;
  for (int64_t f = 0; f < p->sys->n_free_nodes; f++)
    for (int b = 0; b < nv; b++) {
      int32_t kv = p->vert_c[p->Pvert[f * nv + b]];
      if (kv < 0) continue;
      for (int cc = 0; cc < nc; cc++) z[f * nc + cc] += p->Pphi[f * nv + b] * c[(int64_t)kv * nc + cc];
    }
}

/*
 * Factor every local matrix K_j = K[S_j, S_j] (RCM order) and the coarse
 * matrix K_0 = P^T K P (lexicographic order), all in FP64.
 * Returns ORC_ENOTSPD if a pivot is not positive.
 */
int orc_pre_factor(orc_pre *p) {
  const orc_sys *s = p->sys;
  int nv = 1 << p->dim, nc = p->ncomp;
  /* local factors */
  p->sf = zalloc((size_t)(p->nstars ? p->nstars : 1), sizeof(env_factor));
  int32_t *loc = zalloc((size_t)(s->n ? s->n : 1), sizeof(int32_t));
  for (int64_t i = 0; i < s->n; i++) loc[i] = -1;
  for (int64_t st = 0; st < p->nstars; st++) {
    int64_t b0 = p->star_ptr[st], m = p->star_ptr[st + 1] - b0;
    const int32_t *dofs = p->star_dofs + b0;
    for (int64_t a = 0; a < m; a++) loc[dofs[a]] = (int32_t)a;
    /* local CSR of K_j */
    int64_t *ap = zalloc((size_t)m + 1, sizeof(int64_t));
    for (int64_t a = 0; a < m; a++)
      for (int64_t q = s->rowptr[dofs[a]]; q < s->rowptr[dofs[a] + 1]; q++)
        if (loc[s->col[q]] >= 0) ap[a + 1]++;
    for (int64_t a = 0; a < m; a++) ap[a + 1] += ap[a];
    int32_t *ai = zalloc((size_t)(ap[m] ? ap[m] : 1), sizeof(int32_t));
    double *ax = zalloc((size_t)(ap[m] ? ap[m] : 1), sizeof(double));
    for (int64_t a = 0, q2 = 0; a < m; a++)
      for (int64_t q = s->rowptr[dofs[a]]; q < s->rowptr[dofs[a] + 1]; q++)
        if (loc[s->col[q]] >= 0) {
          ai[q2] = loc[s->col[q]];
          ax[q2] = s->val[q];
          q2++;
        }
    env_factor *F = &p->sf[st];
    F->n = m;
    F->perm = zalloc((size_t)(m ? m : 1), sizeof(int32_t));
    rcm_order(m, ap, ai, F->perm);
    int32_t *pos = zalloc((size_t)(m ? m : 1), sizeof(int32_t));
    for (int64_t k = 0; k < m; k++) pos[F->perm[k]] = (int32_t)k;
    F->first = zalloc((size_t)(m ? m : 1), sizeof(int32_t));
    for (int64_t k = 0; k < m; k++) F->first[k] = (int32_t)k;
    for (int64_t a = 0; a < m; a++)
      for (int64_t q = ap[a]; q < ap[a + 1]; q++) {
        int32_t i = pos[a], j = pos[ai[q]];
        if (j < i && j < F->first[i]) F->first[i] = j;
      }
    env_alloc(F);
    for (int64_t a = 0; a < m; a++)
      for (int64_t q = ap[a]; q < ap[a + 1]; q++) {
        int32_t i = pos[a], j = pos[ai[q]];
        if (j <= i) *env_at(F, i, j) += ax[q];
      }
    int rc = env_factorize(F);
    for (int64_t a = 0; a < m; a++) loc[dofs[a]] = -1;
    free(ap);
    free(ai);
    free(ax);
    free(pos);
    if (rc != 0) {
      free(loc);
      snprintf(orc_errbuf, sizeof orc_errbuf, "local matrix of star %lld is not SPD", (long long)st);
      return ORC_ENOTSPD;
    }
  }
  free(loc);

  /* coarse matrix K_0 = P^T K P in its envelope (lexicographic coarse order) */
  int64_t m0 = p->m0;
  env_factor *C = &p->cf;
  C->n = m0;
  C->perm = zalloc((size_t)(m0 ? m0 : 1), sizeof(int32_t));
  for (int64_t k = 0; k < m0; k++) C->perm[k] = (int32_t)k;
  C->first = zalloc((size_t)(m0 ? m0 : 1), sizeof(int32_t));
  for (int64_t k = 0; k < m0; k++) C->first[k] = (int32_t)k;
  /* dof-level P rows: coarse index of each (free node f, vertex b, comp c) */
  for (int pass = 0; pass < 2; pass++) {
    if (pass == 1) env_alloc(C);
    for (int64_t i = 0; i < s->n; i++) {
      int64_t fi = i / nc;
      int ci = (int)(i % nc);
      for (int64_t q = s->rowptr[i]; q < s->rowptr[i + 1]; q++) {
        int64_t j = s->col[q], fj = j / nc;
        int cj = (int)(j % nc);
        for (int a = 0; a < nv; a++) {
          int32_t ka = p->vert_c[p->Pvert[fi * nv + a]];
          if (ka < 0) continue;
          int64_t A = (int64_t)ka * nc + ci;
          for (int b = 0; b < nv; b++) {
            int32_t kb = p->vert_c[p->Pvert[fj * nv + b]];
            if (kb < 0) continue;
            int64_t B = (int64_t)kb * nc + cj;
            if (B > A) continue;
            if (pass == 0) {
              if (B < C->first[A]) C->first[A] = (int32_t)B;
            } else {
              *env_at(C, A, B) += p->Pphi[fi * nv + a] * s->val[q] * p->Pphi[fj * nv + b];
            }
          }
        }
      }
    }
  }
  if (m0 > 0 && m0 <= 3000) {
    p->K0dense = zalloc((size_t)m0 * m0, sizeof(double));
    for (int64_t i = 0; i < m0; i++)
      for (int64_t j = C->first[i]; j <= i; j++) {
        p->K0dense[i * m0 + j] = *env_at(C, i, j);
        p->K0dense[j * m0 + i] = *env_at(C, i, j);
      }
  }
  if (m0 > 0 && env_factorize(C) != 0) return orc_fail(ORC_ENOTSPD, "coarse matrix is not SPD");
  p->factored = 1;
  return ORC_OK;
}

/* dense K_0 (only kept for m0 <= 3000) */
int orc_pre_get_K0_dense(const orc_pre *p, double *K0) {
  if (!p->K0dense) return orc_fail(ORC_EINVAL, "K0 not kept densely");
  memcpy(K0, p->K0dense, (size_t)p->m0 * p->m0 * sizeof(double));
  return ORC_OK;
}

int64_t orc_pre_factor_nnz(const orc_pre *p, int64_t *coarse_nnz) {
  int64_t t = 0;
  for (int64_t st = 0; st < p->nstars; st++) t += p->sf[st].rowoff[p->sf[st].n];
  if (coarse_nnz) *coarse_nnz = p->cf.n ? p->cf.rowoff[p->cf.n] : 0;
  return t;
}

/*
 * Structural non-zeros of the Cholesky factors of all local matrices K_j
 * (incl. the diagonal) under a minimum degree order (Tinney-Walker / Rose):
 * repeatedly eliminate a vertex of least degree in the elimination graph,
 * ties by the smallest local index; eliminating v joins its neighbours
 * pairwise, and column v of L holds v and those neighbours, so the count is the
 * sum of 1 + degree at elimination. A measuring stick for the factor sizes the
 * library stores (it does not enter any solve). Quadratic per star: fine for
 * stars of a few thousand dofs.
 */
int64_t orc_pre_star_md_nnz(const orc_pre *p) {
  const orc_sys *s = p->sys;
  int32_t *loc = zalloc((size_t)(s->n ? s->n : 1), sizeof(int32_t));
  for (int64_t i = 0; i < s->n; i++) loc[i] = -1;
  int64_t total = 0;
  for (int64_t st = 0; st < p->nstars; st++) {
    int64_t b0 = p->star_ptr[st], m = p->star_ptr[st + 1] - b0;
    const int32_t *dofs = p->star_dofs + b0;
    for (int64_t a = 0; a < m; a++) loc[dofs[a]] = (int32_t)a;
    /* neighbour lists of the elimination graph (growable) */
    const size_t mm = (size_t)(m > 0 ? m : 1);
    ivec *nb = zalloc(mm, sizeof(ivec));
    for (int64_t a = 0; a < m; a++)
      for (int64_t q = s->rowptr[dofs[a]]; q < s->rowptr[dofs[a] + 1]; q++) {
        int32_t b = loc[s->col[q]];
        if (b >= 0 && b != a) ivec_push(&nb[a], b);
      }
    char *gone = zalloc(mm, 1);
    int64_t *mark = zalloc(mm, sizeof(int64_t));
    for (int64_t a = 0; a < m; a++) mark[a] = -1;
    for (int64_t step = 0; step < m; step++) {
      int64_t v = -1;
      for (int64_t a = 0; a < m; a++)
        if (!gone[a] && (v < 0 || nb[a].n < nb[v].n)) v = a;
      total += 1 + nb[v].n;
      gone[v] = 1;
      /* every neighbour a of v: drop v, add the other neighbours of v */
      for (int64_t i = 0; i < nb[v].n; i++) {
        int64_t a = nb[v].a[i];
        ivec keep = {0, 0, 0};
        for (int64_t t = 0; t < nb[a].n; t++)
          if (nb[a].a[t] != v) {
            ivec_push(&keep, nb[a].a[t]);
            mark[nb[a].a[t]] = step * m + a;
          }
        for (int64_t t = 0; t < nb[v].n; t++) {
          int64_t b = nb[v].a[t];
          if (b != a && mark[b] != step * m + a) {
            ivec_push(&keep, b);
            mark[b] = step * m + a;
          }
        }
        free(nb[a].a);
        nb[a] = keep;
      }
    }
    for (int64_t a = 0; a < m; a++) free(nb[a].a);
    free(nb);
    free(gone);
    free(mark);
    for (int64_t a = 0; a < m; a++) loc[dofs[a]] = -1;
  }
  free(loc);
  return total;
}

/* z = K_j^{-1} g for one local space (g, z indexed like star_dofs of star st) */
int orc_star_solve(const orc_pre *p, int64_t st, const double *g, double *z) {
  if (st < 0 || st >= p->nstars || !p->factored) return orc_fail(ORC_EINVAL, "bad star");
  const env_factor *F = &p->sf[st];
  double *y = zalloc((size_t)(F->n ? F->n : 1), sizeof(double));
  for (int64_t k = 0; k < F->n; k++) y[k] = g[F->perm[k]];
  env_solve_inplace(F, y);
  for (int64_t k = 0; k < F->n; k++) z[F->perm[k]] = y[k];
  free(y);
  return ORC_OK;
}

/*
 * z = B r with B = P K_0^{-1} P^T + sum_j R_j^T K_j^{-1} R_j, the operator for
 * which BK = P_0 + P_1 + ... + P_m (Sec. 4.1-4.2). Coarse part first, then the
 * local parts in ascending mesh-node order.
 */
int orc_apply_B(const orc_pre *p, const double *r, double *z) {
  const orc_sys *s = p->sys;
  if (!p->factored) return orc_fail(ORC_EINVAL, "not factored");
  memset(z, 0, (size_t)s->n * sizeof(double));
  if (p->m0 > 0) {
    double *rH = zalloc((size_t)p->m0, sizeof(double));
    restrict_P(p, r, rH);
    env_solve_inplace(&p->cf, rH);
    prolong_P_add(p, rH, z);
    free(rH);
  }
  int64_t maxm = 0;
  for (int64_t st = 0; st < p->nstars; st++) {
    int64_t m = p->star_ptr[st + 1] - p->star_ptr[st];
    if (m > maxm) maxm = m;
  }
  double *g = zalloc((size_t)(maxm ? maxm : 1), sizeof(double));
  double *w = zalloc((size_t)(maxm ? maxm : 1), sizeof(double));
  for (int64_t st = 0; st < p->nstars; st++) {
    int64_t b0 = p->star_ptr[st], m = p->star_ptr[st + 1] - b0;
    for (int64_t a = 0; a < m; a++) g[a] = r[p->star_dofs[b0 + a]];
    orc_star_solve(p, st, g, w);
    for (int64_t a = 0; a < m; a++) z[p->star_dofs[b0 + a]] += w[a];
  }
  free(g);
  free(w);
  return ORC_OK;
}

static double vdot(int64_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

/*
 * Preconditioned conjugate gradients on P = BK (Sec. 4.2), one right-hand side.
 *   u        in: initial guess u^(0) (zero for the default), out: u^(l)
 *   rtol     stop after the first iteration with ||r||_2 <= rtol ||f||_2 (recurrence r)
 *   fixed    if > 0, run exactly that many iterations and ignore rtol
 *   uref     optional exact solution; hist_e[l] = |u - u^(l)|_K for l = 0..iters
 *   hist_r   optional; hist_r[l] = ||r^(l)||_2 for l = 0..iters
 * Returns the iteration count l (>= 0) or a negative status.
 */
int64_t orc_pcg(const orc_pre *p, const double *f, double *u, double rtol, int64_t max_iter,
                int64_t fixed, const double *uref, double *hist_r, double *hist_e,
                double *true_res) {
  const orc_sys *s = p->sys;
  int64_t n = s->n;
  double *r = zalloc((size_t)n, sizeof(double));
  double *z = zalloc((size_t)n, sizeof(double));
  double *pp = zalloc((size_t)n, sizeof(double));
  double *q = zalloc((size_t)n, sizeof(double));
  double *e = uref ? zalloc((size_t)n, sizeof(double)) : NULL;
  double *Ke = uref ? zalloc((size_t)n, sizeof(double)) : NULL;

  orc_apply_K(s, u, q);
  for (int64_t i = 0; i < n; i++) r[i] = f[i] - q[i];
  double fn = sqrt(vdot(n, f, f));
  orc_apply_B(p, r, z);
  memcpy(pp, z, (size_t)n * sizeof(double));
  double rho = vdot(n, r, z);
  int64_t it = 0;
#define RECORD(L)                                                 \
  do {                                                            \
    if (hist_r) hist_r[L] = sqrt(vdot(n, r, r));                  \
    if (uref) {                                                   \
      for (int64_t i_ = 0; i_ < n; i_++) e[i_] = uref[i_] - u[i_];\
      orc_apply_K(s, e, Ke);                                      \
      hist_e[L] = sqrt(fmax(vdot(n, e, Ke), 0.0));                \
    }                                                             \
  } while (0)
  RECORD(0);
  int64_t limit = fixed > 0 ? fixed : max_iter;
  int converged = (fixed <= 0 && sqrt(vdot(n, r, r)) <= rtol * fn);
  while (!converged && it < limit) {
    orc_apply_K(s, pp, q);
    double alpha = rho / vdot(n, pp, q);
    for (int64_t i = 0; i < n; i++) {
      u[i] += alpha * pp[i];
      r[i] -= alpha * q[i];
    }
    it++;
    RECORD(it);
    if (fixed <= 0 && sqrt(vdot(n, r, r)) <= rtol * fn) {
      converged = 1;
      break;
    }
    orc_apply_B(p, r, z);
    double rho_new = vdot(n, r, z);
    double beta = rho_new / rho;
    for (int64_t i = 0; i < n; i++) pp[i] = z[i] + beta * pp[i];
    rho = rho_new;
  }
#undef RECORD
  if (true_res) {
    orc_apply_K(s, u, q);
    for (int64_t i = 0; i < n; i++) q[i] = f[i] - q[i];
    *true_res = fn > 0.0 ? sqrt(vdot(n, q, q)) / fn : sqrt(vdot(n, q, q));
  }
  free(r);
  free(z);
  free(pp);
  free(q);
  free(e);
  free(Ke);
  if (fixed <= 0 && !converged) return ORC_ENOCONV;
  return it;
}
