/*
 * FP64 CPU oracle for the GMCP hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP implementation; the two meet only through the seeded inputs.
 *
 * Everything is double precision, straight-line and unoptimised: one sample
 * at a time, every quantity taken from its definition in the paper
 * (Sec. 4 "Geometric Mortar Contact Potential"):
 *   - sample positions by barycentric interpolation (Sec. 4.1),
 *   - signed gap along the slave normal, Eq. (gap),
 *   - master barycentrics from the 2x2 Gram system, Eq. (gram),
 *   - the barrier sum, Eq. (gmcp_potential), with the IPC log barrier,
 *   - gradient / Hessian approximation and PSD projection (Sec. 4.2),
 *   - Hermite step and face weight f_T, Eqs. (smoothstep), (gamma),
 *   - adaptive support radius, Eq. (adaptive_eps),
 *   - linearised-gap step bound, Eqs. (ccd), (global_ccd),
 *   - additive CCD (Li, Kaufman, Jiang 2021, "Codimensional Incremental
 *     Potential Contact", Sec. on additive CCD) for swept sample/triangle pairs.
 *
 * Candidate search is either brute force (every master triangle) or a plain
 * uniform grid that only prunes triangles whose bounding box cannot contain
 * the hit point; both give the same selection (a test checks this).
 *
 * Compiled with gcc (optionally -fopenmp); see oracle/build.py.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
  ORA_OK = 0,
  ORA_E_ARG = 1,
  ORA_E_CAPACITY = 2,
  ORA_E_PENETRATION = 3,
  ORA_E_DEGENERATE = 4,
  ORA_E_NONFINITE = 5
};

/* per-sample ambiguity flags: decisions a float32 evaluation may take
 * differently from this FP64 one */
#define ORA_FLAG_SUPPORT 1  /* gap within 1e-4 eps of the support edge */
#define ORA_FLAG_INSIDE 2   /* a relevant hit with min barycentric within 1e-5 of 0 */
#define ORA_FLAG_TIE 4      /* runner-up gap within 1e-6 eps of the best */
#define ORA_FLAG_PARALLEL 8 /* master plane almost parallel to the slave normal */
#define ORA_FLAG_ZERO 16    /* gap within 1e-6 eps of zero */

#define TOL_BETA 1e-5
#define TOL_SUPPORT 1e-4
#define TOL_TIE 1e-6
#define TOL_ZERO 1e-6
#define TOL_PARALLEL 1e-6

/* ------------------------------------------------------------------ vec3 */
static void v_sub(const double *a, const double *b, double *o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double v_dot(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void v_cross(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double v_norm(const double *a) { return sqrt(v_dot(a, a)); }

/* ------------------------------------------------------------ barrier B
 * IPC log barrier on the linear gap g with support radius eps:
 *   B(g) = -(g - eps)^2 ln(g / eps)  for 0 < g < eps, 0 for g >= eps.     */
double ora_barrier(double g, double eps) {
  if (g >= eps) return 0.0;
  double d = g - eps;
  return -d * d * log(g / eps);
}
double ora_barrier_d1(double g, double eps) {
  if (g >= eps) return 0.0;
  double d = g - eps;
  return -2.0 * d * log(g / eps) - d * d / g;
}
double ora_barrier_d2(double g, double eps) {
  if (g >= eps) return 0.0;
  double d = g - eps;
  return -2.0 * log(g / eps) - 4.0 * d / g + d * d / (g * g);
}

/* C^1 Hermite step, Eq. (smoothstep) */
double ora_hermite(double x, double delta) {
  if (x <= 0.0) return 0.0;
  if (x >= delta) return 1.0;
  double t = x / delta;
  return 3.0 * t * t - 2.0 * t * t * t;
}

/* face weight gamma = f_T = H(min_a beta^m_a, delta_T), Eq. (gamma).
 * delta_T = 0 is read as a sharp step: 1 for every inside hit. */
static double face_gamma(const double bm[3], double delta_T) {
  if (delta_T <= 0.0) return 1.0;
  double mn = bm[0];
  if (bm[1] < mn) mn = bm[1];
  if (bm[2] < mn) mn = bm[2];
  return ora_hermite(mn, delta_T);
}

/* ---------------------------------------------------------- rest areas */
void ora_rest_area(int T, const double *x, const int *tri, double *area) {
  for (int t = 0; t < T; ++t) {
    const double *a = x + 3 * tri[3 * t], *b = x + 3 * tri[3 * t + 1], *c = x + 3 * tri[3 * t + 2];
    double e1[3], e2[3], n[3];
    v_sub(b, a, e1);
    v_sub(c, a, e2);
    v_cross(e1, e2, n);
    area[t] = 0.5 * v_norm(n);
  }
}

/* ------------------------------------------------------- slave frame
 * unit normal n_T = (e1 x e2)/|e1 x e2| (the formula of the dual-mesh
 * section, applied to the slave triangle).  Returns 0 if degenerate. */
static int slave_frame(const double *xs, const int *tri, int T, double s0[3], double e1[3],
                       double e2[3], double n[3]) {
  const double *a = xs + 3 * tri[3 * T], *b = xs + 3 * tri[3 * T + 1], *c = xs + 3 * tri[3 * T + 2];
  s0[0] = a[0]; s0[1] = a[1]; s0[2] = a[2];
  v_sub(b, a, e1);
  v_sub(c, a, e2);
  double cr[3];
  v_cross(e1, e2, cr);
  double len = v_norm(cr);
  if (!(len > 1e-14 * (v_dot(e1, e1) + v_dot(e2, e2)))) return 0;
  n[0] = cr[0] / len; n[1] = cr[1] / len; n[2] = cr[2] / len;
  return 1;
}

/* ------------------------------------------------------------ ray hit
 * Sample point p, slave normal n, master triangle (m0,m1,m2).
 * The master point x_m is where the line p + t n meets the master plane;
 * the signed gap is g = n.(x_m - p) = t (Eq. gap).  Master barycentrics of
 * x_m from the Gram system of Eq. (gram) built on the master edges.
 * Returns 0 when the master triangle is degenerate or the line is parallel
 * to its plane (den == 0); den_out receives n.N_M / |N_M|.                */
static int ray_hit(const double p[3], const double n[3], const double *m0, const double *m1,
                   const double *m2, double *t_out, double bm[3], double *den_out) {
  double f1[3], f2[3], N[3];
  v_sub(m1, m0, f1);
  v_sub(m2, m0, f2);
  v_cross(f1, f2, N);
  double nN = v_norm(N);
  if (nN == 0.0) return 0;
  double den = v_dot(n, N);
  *den_out = den / nN;
  if (den == 0.0) return 0;
  double d[3];
  v_sub(m0, p, d);
  double t = v_dot(N, d) / den;
  double xm[3] = {p[0] + t * n[0], p[1] + t * n[1], p[2] + t * n[2]};
  double r[3];
  v_sub(xm, m0, r);
  double a11 = v_dot(f1, f1), a12 = v_dot(f1, f2), a22 = v_dot(f2, f2);
  double r1 = v_dot(r, f1), r2 = v_dot(r, f2);
  double det = a11 * a22 - a12 * a12;
  if (det == 0.0) return 0;
  double b1 = (a22 * r1 - a12 * r2) / det;
  double b2 = (a11 * r2 - a12 * r1) / det;
  bm[0] = 1.0 - b1 - b2;
  bm[1] = b1;
  bm[2] = b2;
  *t_out = t;
  return 1;
}

static double min3(const double b[3]) {
  double m = b[0];
  if (b[1] < m) m = b[1];
  if (b[2] < m) m = b[2];
  return m;
}

/* ------------------------------------------------------- uniform grid
 * Plain candidate pruning: items are boxes; a query box returns every item
 * whose box overlaps it (each once).                                     */
typedef struct {
  double lo[3];
  double h;
  int64_t nc[3];
  int64_t *start; /* [ncell + 1] */
  int *items;
} ogrid;

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void ogrid_cell_range(const ogrid *g, const double *lo, const double *hi, int64_t c0[3], int64_t c1[3]) {
  for (int d = 0; d < 3; ++d) {
    c0[d] = clampi((int64_t)floor((lo[d] - g->lo[d]) / g->h), 0, g->nc[d] - 1);
    c1[d] = clampi((int64_t)floor((hi[d] - g->lo[d]) / g->h), 0, g->nc[d] - 1);
  }
}

typedef struct {
  int64_t cell;
  int item;
} cell_item;

static int cmp_cell_item(const void *a, const void *b) {
  const cell_item *x = (const cell_item *)a, *y = (const cell_item *)b;
  if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
  return (x->item > y->item) - (x->item < y->item);
}

/* box arrays are [n][3]; h <= 0 selects the mean item extent */
static int ogrid_build(ogrid *g, int n, const double *blo, const double *bhi, double h) {
  memset(g, 0, sizeof(*g));
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  double ext = 0.0;
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      if (blo[3 * i + d] < lo[d]) lo[d] = blo[3 * i + d];
      if (bhi[3 * i + d] > hi[d]) hi[d] = bhi[3 * i + d];
      ext += bhi[3 * i + d] - blo[3 * i + d];
    }
  if (n == 0) {
    lo[0] = lo[1] = lo[2] = 0.0;
    hi[0] = hi[1] = hi[2] = 1.0;
  }
  if (h <= 0.0) h = n ? ext / (3.0 * n) : 1.0;
  double span = 0.0;
  for (int d = 0; d < 3; ++d)
    if (hi[d] - lo[d] > span) span = hi[d] - lo[d];
  if (h < span * 1e-4) h = span * 1e-4;
  if (!(h > 0.0)) h = 1.0;
  for (;;) {
    int64_t tot = 1;
    for (int d = 0; d < 3; ++d) {
      g->nc[d] = (int64_t)floor((hi[d] - lo[d]) / h) + 1;
      tot *= g->nc[d];
    }
    if (tot <= (1 << 24)) break;
    h *= 1.5;
  }
  g->h = h;
  for (int d = 0; d < 3; ++d) g->lo[d] = lo[d];
  int64_t ncell = g->nc[0] * g->nc[1] * g->nc[2];
  int64_t cnt = 0;
  for (int i = 0; i < n; ++i) {
    int64_t c0[3], c1[3];
    ogrid_cell_range(g, blo + 3 * i, bhi + 3 * i, c0, c1);
    cnt += (c1[0] - c0[0] + 1) * (c1[1] - c0[1] + 1) * (c1[2] - c0[2] + 1);
  }
  cell_item *ci = (cell_item *)malloc(sizeof(cell_item) * (size_t)(cnt ? cnt : 1));
  if (!ci) return 0;
  int64_t k = 0;
  for (int i = 0; i < n; ++i) {
    int64_t c0[3], c1[3];
    ogrid_cell_range(g, blo + 3 * i, bhi + 3 * i, c0, c1);
    for (int64_t z = c0[2]; z <= c1[2]; ++z)
      for (int64_t y = c0[1]; y <= c1[1]; ++y)
        for (int64_t x = c0[0]; x <= c1[0]; ++x) {
          ci[k].cell = (z * g->nc[1] + y) * g->nc[0] + x;
          ci[k].item = i;
          ++k;
        }
  }
  qsort(ci, (size_t)cnt, sizeof(cell_item), cmp_cell_item);
  g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  g->items = (int *)malloc(sizeof(int) * (size_t)(cnt ? cnt : 1));
  if (!g->start || !g->items) {
    free(ci);
    return 0;
  }
  for (int64_t j = 0; j < cnt; ++j) {
    g->items[j] = ci[j].item;
    g->start[ci[j].cell + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
  free(ci);
  return 1;
}

static void ogrid_free(ogrid *g) {
  free(g->start);
  free(g->items);
  memset(g, 0, sizeof(*g));
}

/* stamp[] has one slot per item and must start at values != stamp_id */
static int ogrid_query(const ogrid *g, const double *lo, const double *hi, const double *blo,
                       const double *bhi, int *stamp, int stamp_id, int *out, int cap) {
  int64_t c0[3], c1[3];
  ogrid_cell_range(g, lo, hi, c0, c1);
  int cnt = 0;
  for (int64_t z = c0[2]; z <= c1[2]; ++z)
    for (int64_t y = c0[1]; y <= c1[1]; ++y)
      for (int64_t x = c0[0]; x <= c1[0]; ++x) {
        int64_t c = (z * g->nc[1] + y) * g->nc[0] + x;
        for (int64_t j = g->start[c]; j < g->start[c + 1]; ++j) {
          int it = g->items[j];
          if (stamp[it] == stamp_id) continue;
          stamp[it] = stamp_id;
          const double *a = blo + 3 * it, *b = bhi + 3 * it;
          if (a[0] > hi[0] || b[0] < lo[0] || a[1] > hi[1] || b[1] < lo[1] || a[2] > hi[2] || b[2] < lo[2])
            continue;
          if (cnt < cap) out[cnt] = it;
          ++cnt;
        }
      }
  return cnt;
}

static void tri_boxes(int T, const double *x, const int *tri, double *blo, double *bhi) {
  for (int t = 0; t < T; ++t)
    for (int d = 0; d < 3; ++d) {
      double a = x[3 * tri[3 * t] + d], b = x[3 * tri[3 * t + 1] + d], c = x[3 * tri[3 * t + 2] + d];
      double lo = a < b ? a : b, hi = a > b ? a : b;
      if (c < lo) lo = c;
      if (c > hi) hi = c;
      blo[3 * t + d] = lo;
      bhi[3 * t + d] = hi;
    }
}

/* ------------------------------------------------------ narrow phase
 * For every sample k = T*nq + q of every slave triangle T:
 *   x_s,k = s0 + xi e1 + eta e2  (beta^s = (1-xi-eta, xi, eta)),
 *   eps_k = min(0.9 g_ref,k, dhat)          Eq. (adaptive_eps)
 * and, over the opposing master triangles (n_T . N_M < 0) whose line hit
 * is inside (min beta^m >= 0, inclusive):
 *   accept 0 < g < eps_k, select the smallest g, ties -> smaller index;
 *   an inside hit with -eps_k < g <= 0 is a penetration.
 * Outputs per sample: M (-1 if inactive), g, beta^m[3], flags.
 * Returns ORA_OK, ORA_E_DEGENERATE (*bad = triangle) or
 * ORA_E_PENETRATION (*bad = smallest penetrating sample id).             */
int ora_narrow(int Vs, int Ts, const double *xs, const int *ts, int Vm, int Tm, const double *xm,
               const int *tm, int nq, const double *rule, double dhat, const double *g_ref,
               int use_grid, int *M_out, double *g_out, double *bm_out, int *flag_out, int64_t *bad) {
  (void)Vs;
  (void)Vm;
  *bad = -1;
  for (int T = 0; T < Ts; ++T) {
    double s0[3], e1[3], e2[3], n[3];
    if (!slave_frame(xs, ts, T, s0, e1, e2, n)) {
      *bad = T;
      return ORA_E_DEGENERATE;
    }
  }
  double *blo = (double *)malloc(sizeof(double) * 3 * (size_t)(Tm ? Tm : 1));
  double *bhi = (double *)malloc(sizeof(double) * 3 * (size_t)(Tm ? Tm : 1));
  tri_boxes(Tm, xm, tm, blo, bhi);
  ogrid grid;
  int have_grid = 0;
  if (use_grid) have_grid = ogrid_build(&grid, Tm, blo, bhi, 0.0);
  int64_t pen_min = INT64_MAX;

#pragma omp parallel
  {
    int *stamp = NULL, *cand = NULL;
    int cap = Tm > 0 ? Tm : 1;
    if (have_grid) {
      stamp = (int *)malloc(sizeof(int) * (size_t)cap);
      for (int i = 0; i < Tm; ++i) stamp[i] = -1;
    }
    cand = (int *)malloc(sizeof(int) * (size_t)cap);
    int64_t my_pen = INT64_MAX;
#pragma omp for schedule(dynamic, 16)
    for (int T = 0; T < Ts; ++T) {
      double s0[3], e1[3], e2[3], n[3];
      slave_frame(xs, ts, T, s0, e1, e2, n);
      for (int q = 0; q < nq; ++q) {
        int64_t k = (int64_t)T * nq + q;
        double xi = rule[3 * q], eta = rule[3 * q + 1];
        double p[3];
        for (int d = 0; d < 3; ++d) p[d] = s0[d] + xi * e1[d] + eta * e2[d];
        double eps = dhat;
        if (g_ref && 0.9 * g_ref[k] < eps) eps = 0.9 * g_ref[k];
        int nc;
        if (have_grid) {
          double lo[3], hi[3];
          for (int d = 0; d < 3; ++d) {
            double a = p[d] - eps * n[d], b = p[d] + eps * n[d];
            lo[d] = a < b ? a : b;
            hi[d] = a > b ? a : b;
          }
          nc = ogrid_query(&grid, lo, hi, blo, bhi, stamp, (int)(k & 0x7fffffff), cand, cap);
        } else {
          nc = Tm;
          for (int i = 0; i < Tm; ++i) cand[i] = i;
        }
        int best = -1, flags = 0;
        double bt = 0.0, bb[3] = {0, 0, 0}, t2 = INFINITY;
        int pen = 0;
        for (int c = 0; c < nc; ++c) {
          int M = cand[c];
          double t, bm[3], den;
          if (!ray_hit(p, n, xm + 3 * tm[3 * M], xm + 3 * tm[3 * M + 1], xm + 3 * tm[3 * M + 2], &t, bm, &den))
            continue;
          double mb = min3(bm);
          int near_in = mb >= -TOL_BETA;
          int in_range = t > -eps * (1.0 + TOL_SUPPORT) && t < eps * (1.0 + TOL_SUPPORT);
          if (fabs(den) <= TOL_PARALLEL && near_in && in_range) flags |= ORA_FLAG_PARALLEL;
          if (den >= 0.0) continue; /* not opposing */
          if (fabs(mb) <= TOL_BETA && in_range) flags |= ORA_FLAG_INSIDE;
          if (near_in && fabs(t - eps) <= TOL_SUPPORT * eps) flags |= ORA_FLAG_SUPPORT;
          if (near_in && fabs(t) <= TOL_ZERO * eps) flags |= ORA_FLAG_ZERO;
          if (mb < 0.0) continue; /* outside */
          if (t > 0.0 && t < eps) {
            if (best < 0 || t < bt || (t == bt && M < best)) {
              if (best >= 0 && bt < t2) t2 = bt;
              best = M;
              bt = t;
              bb[0] = bm[0]; bb[1] = bm[1]; bb[2] = bm[2];
            } else if (t < t2) {
              t2 = t;
            }
          } else if (t > -eps && t <= 0.0) {
            pen = 1;
          }
        }
        if (best >= 0 && t2 - bt <= TOL_TIE * eps) flags |= ORA_FLAG_TIE;
        if (pen && k < my_pen) my_pen = k;
        M_out[k] = best;
        g_out[k] = best >= 0 ? bt : 0.0;
        bm_out[3 * k] = bb[0];
        bm_out[3 * k + 1] = bb[1];
        bm_out[3 * k + 2] = bb[2];
        flag_out[k] = flags;
      }
    }
#pragma omp critical
    {
      if (my_pen < pen_min) pen_min = my_pen;
    }
    free(stamp);
    free(cand);
  }
  if (have_grid) ogrid_free(&grid);
  free(blo);
  free(bhi);
  if (pen_min != INT64_MAX) {
    *bad = pen_min;
    return ORA_E_PENETRATION;
  }
  return ORA_OK;
}

/* ---------------------------------------------------- sample evaluation
 * Re-evaluates the geometry of sample k against a given master triangle M
 * (used when a caller imposes the assignment, e.g. for ambiguous samples). */
int ora_sample_geom(const double *xs, const int *ts, const double *xm, const int *tm, int nq,
                    const double *rule, int64_t k, int M, double *g, double bm[3], double n[3]) {
  int T = (int)(k / nq), q = (int)(k % nq);
  double s0[3], e1[3], e2[3];
  if (!slave_frame(xs, ts, T, s0, e1, e2, n)) return ORA_E_DEGENERATE;
  double p[3];
  for (int d = 0; d < 3; ++d) p[d] = s0[d] + rule[3 * q] * e1[d] + rule[3 * q + 1] * e2[d];
  double den;
  if (!ray_hit(p, n, xm + 3 * tm[3 * M], xm + 3 * tm[3 * M + 1], xm + 3 * tm[3 * M + 2], g, bm, &den))
    return ORA_E_DEGENERATE;
  return ORA_OK;
}

/* ---------------------------------------------- symmetric Jacobi eigen
 * Cyclic Jacobi rotations on a dense symmetric n x n matrix (row-major),
 * eigenvalues to w, eigenvectors as columns of V.                         */
static void jacobi_eigen(int n, double *A, double *w, double *V) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double app = A[p * n + p], aqq = A[q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

/* Projects a symmetric n x n matrix onto the PSD cone (clamp negative
 * eigenvalues to 0).  Returns the largest clamped |lambda|.               */
double ora_psd_project(int n, double *H) {
  double *A = (double *)malloc(sizeof(double) * (size_t)(n * n));
  double *V = (double *)malloc(sizeof(double) * (size_t)(n * n));
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  memcpy(A, H, sizeof(double) * (size_t)(n * n));
  jacobi_eigen(n, A, w, V);
  double clamped = 0.0;
  for (int i = 0; i < n; ++i)
    if (w[i] < 0.0) {
      if (-w[i] > clamped) clamped = -w[i];
      w[i] = 0.0;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += V[i * n + k] * w[k] * V[j * n + k];
      H[i * n + j] = s;
    }
  free(A);
  free(V);
  free(w);
  return clamped;
}

/* Virtual-point 12x12 block of one sample over (x_s,k, m0, m1, m2):
 *   g = n.(sum_j bm_j m_j - x_s,k), grad g = shat (x) n with
 *   shat = (-1, bm0, bm1, bm2);  H12 = c2 (shat shat^T) (x) (n n^T),
 * projected to the PSD cone (Sec. 4.2).  Returns the clamped |lambda|.   */
double ora_local_block12(double c2, const double bm[3], const double n[3], double *H12) {
  double sh[4] = {-1.0, bm[0], bm[1], bm[2]};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) H12[(3 * a + i) * 12 + 3 * b + j] = c2 * sh[a] * sh[b] * n[i] * n[j];
  return ora_psd_project(12, H12);
}

/* ------------------------------------------------------------ assembly */
typedef struct {
  int64_t key; /* row * Vtot + col */
  int64_t k;   /* sample */
  int a, b;    /* local dof blocks in 0..5 */
} hcontrib;

static int cmp_hc(const void *x, const void *y) {
  const hcontrib *p = (const hcontrib *)x, *q = (const hcontrib *)y;
  if (p->key != q->key) return p->key < q->key ? -1 : 1;
  if (p->k != q->k) return p->k < q->k ? -1 : 1;
  if (p->a != q->a) return p->a - q->a;
  return p->b - q->b;
}

static double pairwise_sum(const double *v, int64_t n) {
  if (n <= 8) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[i];
    return s;
  }
  int64_t h = n / 2;
  return pairwise_sum(v, h) + pairwise_sum(v + h, n - h);
}

/*
 * Energy, gradient, Hessian of Eq. (gmcp_potential) for face samples
 * (q = 2), with every sample's master triangle given in M[k] (-1: none).
 *   w_k   = 2 A_rest(T) what_q           (sample weight = area share)
 *   g_k   = geometric gap + delta_gap[k]  (delta_gap nullable)
 *   E_k   = kappa w_k gamma_k B(g_k, eps_k)
 *   c1_k  = kappa w_k gamma_k B'(g_k),  c2_k = kappa w_k gamma_k B''(g_k)
 *   p_k   = -kappa gamma_k B'(g_k)        (pressure: force per sample area)
 *   grad g_k = -beta^s_a n_T at slave vertex a, +beta^m_j n_T at master j.
 * The Hessian of each sample, c2 (s s^T) (x) (n n^T) over the six vertices,
 * is formed from the PSD-projected 12x12 virtual-point block when
 * project != 0 (eigen-decomposition), else with c2 clamped at 0.
 * Global vertex numbering: slave 0..Vs-1, master Vs..Vs+Vm-1.
 * kinematic != 0 drops master rows/columns and the master gradient.
 * BSR: rows ascending, columns ascending, both triangles, 3x3 row-major.
 * E_k, c1, c2, press are per-sample outputs (may be NULL).
 * Returns ORA_E_CAPACITY with *nnzb = needed count if cap_nnzb is short.  */
int ora_assemble(int Vs, int Ts, const double *xs, const int *ts, int Vm, int Tm, const double *xm,
                 const int *tm, int nq, const double *rule, const double *area, double kappa,
                 double dhat, double delta_T, const double *g_ref, const double *delta_gap,
                 const int *M, int kinematic, int project, double *energy, double *Ek, double *c1o,
                 double *c2o, double *press, double *grad, int64_t cap_nnzb, int64_t *row_ptr,
                 int64_t *col, double *val, int64_t *nnzb, double *max_clamped, int64_t *bad) {
  (void)Tm;
  int64_t Ns = (int64_t)Ts * nq;
  int64_t Vt = (int64_t)Vs + Vm;
  *bad = -1;
  double *e = (double *)calloc((size_t)(Ns ? Ns : 1), sizeof(double));
  double *c1 = (double *)calloc((size_t)(Ns ? Ns : 1), sizeof(double));
  double *c2 = (double *)calloc((size_t)(Ns ? Ns : 1), sizeof(double));
  double *nrm = (double *)calloc((size_t)(3 * (Ns ? Ns : 1)), sizeof(double));
  double *bmv = (double *)calloc((size_t)(3 * (Ns ? Ns : 1)), sizeof(double));
  int64_t err_k = INT64_MAX;
  int err_code = ORA_OK;
  double clamp_max = 0.0;
  int64_t nact = 0;

#pragma omp parallel for schedule(dynamic, 256) reduction(max : clamp_max) reduction(+ : nact)
  for (int64_t k = 0; k < Ns; ++k) {
    if (press) press[k] = 0.0;
    if (M[k] < 0) continue;
    double g, bm[3], n[3];
    if (ora_sample_geom(xs, ts, xm, tm, nq, rule, k, M[k], &g, bm, n) != ORA_OK) {
#pragma omp critical
      {
        if (k < err_k) { err_k = k; err_code = ORA_E_DEGENERATE; }
      }
      continue;
    }
    if (delta_gap) g += delta_gap[k];
    double eps = dhat;
    if (g_ref && 0.9 * g_ref[k] < eps) eps = 0.9 * g_ref[k];
    if (!(g > 0.0)) {
#pragma omp critical
      {
        if (k < err_k) { err_k = k; err_code = ORA_E_PENETRATION; }
      }
      continue;
    }
    if (g >= eps) continue; /* zero energy, gradient and Hessian beyond eps */
    int T = (int)(k / nq), q = (int)(k % nq);
    double w = 2.0 * area[T] * rule[3 * q + 2];
    double gam = face_gamma(bm, delta_T);
    double B = ora_barrier(g, eps), B1 = ora_barrier_d1(g, eps), B2 = ora_barrier_d2(g, eps);
    e[k] = kappa * w * gam * B;
    c1[k] = kappa * w * gam * B1;
    c2[k] = kappa * w * gam * B2;
    if (press) press[k] = -kappa * gam * B1;
    for (int d = 0; d < 3; ++d) {
      nrm[3 * k + d] = n[d];
      bmv[3 * k + d] = bm[d];
    }
    if (project) {
      double H12[144];
      double cl = ora_local_block12(c2[k], bm, n, H12);
      if (cl > clamp_max) clamp_max = cl;
      /* recover the projected rank-1 coefficient: the projected block is
       * c2p (shat shat^T)(x)(n n^T); read it off the (0,0) dof entry along n */
      double v00 = 0.0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) v00 += n[i] * H12[i * 12 + j] * n[j];
      c2[k] = v00; /* shat_0^2 = 1 */
    } else if (c2[k] < 0.0) {
      if (-c2[k] > clamp_max) clamp_max = -c2[k];
      c2[k] = 0.0;
    }
    nact += 1;
  }
  if (max_clamped) *max_clamped = clamp_max;
  if (err_code != ORA_OK) {
    *bad = err_k;
    free(e); free(c1); free(c2); free(nrm); free(bmv);
    return err_code;
  }
  *energy = pairwise_sum(e, Ns);
  if (Ek) memcpy(Ek, e, sizeof(double) * (size_t)Ns);
  if (c1o) memcpy(c1o, c1, sizeof(double) * (size_t)Ns);
  if (c2o) memcpy(c2o, c2, sizeof(double) * (size_t)Ns);

  /* gradient: plain serial scatter over samples in order */
  if (grad) {
    memset(grad, 0, sizeof(double) * 3 * (size_t)Vt);
    for (int64_t k = 0; k < Ns; ++k) {
      if (M[k] < 0 || c1[k] == 0.0) continue;
      int T = (int)(k / nq), q = (int)(k % nq);
      double xi = rule[3 * q], eta = rule[3 * q + 1];
      double bs[3] = {1.0 - xi - eta, xi, eta};
      const double *n = nrm + 3 * k;
      for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) grad[3 * (int64_t)ts[3 * T + a] + d] += -c1[k] * bs[a] * n[d];
      if (!kinematic)
        for (int j = 0; j < 3; ++j)
          for (int d = 0; d < 3; ++d)
            grad[3 * ((int64_t)Vs + tm[3 * M[k] + j]) + d] += c1[k] * bmv[3 * k + j] * n[d];
    }
  }

  /* Hessian: collect (row, col, sample, a, b), sort, reduce in order */
  if (row_ptr) {
    int64_t ncon = 0;
    int nd = kinematic ? 3 : 6;
    for (int64_t k = 0; k < Ns; ++k)
      if (M[k] >= 0 && c1[k] != 0.0) ncon += nd * nd;
    hcontrib *hc = (hcontrib *)malloc(sizeof(hcontrib) * (size_t)(ncon ? ncon : 1));
    int64_t m = 0;
    for (int64_t k = 0; k < Ns; ++k) {
      if (M[k] < 0 || c1[k] == 0.0) continue;
      int T = (int)(k / nq);
      int64_t vid[6];
      for (int a = 0; a < 3; ++a) vid[a] = ts[3 * T + a];
      for (int j = 0; j < 3; ++j) vid[3 + j] = (int64_t)Vs + tm[3 * M[k] + j];
      for (int a = 0; a < nd; ++a)
        for (int b = 0; b < nd; ++b) {
          hc[m].key = vid[a] * Vt + vid[b];
          hc[m].k = k;
          hc[m].a = a;
          hc[m].b = b;
          ++m;
        }
    }
    qsort(hc, (size_t)ncon, sizeof(hcontrib), cmp_hc);
    int64_t nb = 0;
    for (int64_t i = 0; i < ncon; ++i)
      if (i == 0 || hc[i].key != hc[i - 1].key) ++nb;
    *nnzb = nb;
    if (nb > cap_nnzb) {
      free(hc); free(e); free(c1); free(c2); free(nrm); free(bmv);
      return ORA_E_CAPACITY;
    }
    for (int64_t r = 0; r <= Vt; ++r) row_ptr[r] = 0;
    int64_t b = -1;
    for (int64_t i = 0; i < ncon; ++i) {
      if (i == 0 || hc[i].key != hc[i - 1].key) {
        ++b;
        int64_t row = hc[i].key / Vt;
        col[b] = hc[i].key % Vt;
        row_ptr[row + 1] += 1;
        for (int z = 0; z < 9; ++z) val[9 * b + z] = 0.0;
      }
      int64_t k = hc[i].k;
      int T = (int)(k / nq), q = (int)(k % nq);
      double xi = rule[3 * q], eta = rule[3 * q + 1];
      double s[6] = {-(1.0 - xi - eta), -xi, -eta, bmv[3 * k], bmv[3 * k + 1], bmv[3 * k + 2]};
      (void)T;
      const double *n = nrm + 3 * k;
      double coef = c2[k] * s[hc[i].a] * s[hc[i].b];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) val[9 * b + 3 * r + c] += coef * n[r] * n[c];
    }
    for (int64_t r = 0; r < Vt; ++r) row_ptr[r + 1] += row_ptr[r];
    free(hc);
  }
  free(e); free(c1); free(c2); free(nrm); free(bmv);
  return ORA_OK;
}

/*
 * Pressure-map loss L = 1/2 sum_k (p_k - p*_k)^2 with p_k = -kappa gamma B'(g_k)
 * and its gradient with samples frozen:
 *   dL/dx     = sum_k (p_k - p*_k) (-kappa gamma B''(g_k)) grad g_k
 *   dL/ddelta = (p_k - p*_k) (-kappa gamma B''(g_k)).
 * M, delta_gap as in ora_assemble.  Returns L.                            */
double ora_pressure_loss(int Vs, int Ts, const double *xs, const int *ts, int Vm, const double *xm,
                         const int *tm, int nq, const double *rule, double kappa, double dhat,
                         double delta_T, const double *g_ref, const double *delta_gap, const int *M,
                         const double *ptarget, double *dLdx, double *dLddelta) {
  int64_t Ns = (int64_t)Ts * nq, Vt = (int64_t)Vs + Vm;
  if (dLdx) memset(dLdx, 0, sizeof(double) * 3 * (size_t)Vt);
  double *res = (double *)calloc((size_t)(Ns ? Ns : 1), sizeof(double));
  for (int64_t k = 0; k < Ns; ++k) {
    double p = 0.0, dp = 0.0, g = 0.0, bm[3] = {0, 0, 0}, n[3] = {0, 0, 0};
    int act = 0;
    if (M[k] >= 0 && ora_sample_geom(xs, ts, xm, tm, nq, rule, k, M[k], &g, bm, n) == ORA_OK) {
      if (delta_gap) g += delta_gap[k];
      double eps = dhat;
      if (g_ref && 0.9 * g_ref[k] < eps) eps = 0.9 * g_ref[k];
      if (g > 0.0 && g < eps) {
        double gam = face_gamma(bm, delta_T);
        p = -kappa * gam * ora_barrier_d1(g, eps);
        dp = -kappa * gam * ora_barrier_d2(g, eps);
        act = 1;
      }
    }
    double r = p - ptarget[k];
    res[k] = 0.5 * r * r;
    if (dLddelta) dLddelta[k] = act ? r * dp : 0.0;
    if (act && dLdx) {
      int T = (int)(k / nq), q = (int)(k % nq);
      double xi = rule[3 * q], eta = rule[3 * q + 1];
      double bs[3] = {1.0 - xi - eta, xi, eta};
      for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) dLdx[3 * (int64_t)ts[3 * T + a] + d] += r * dp * (-bs[a]) * n[d];
      for (int j = 0; j < 3; ++j)
        for (int d = 0; d < 3; ++d) dLdx[3 * ((int64_t)Vs + tm[3 * M[k] + j]) + d] += r * dp * bm[j] * n[d];
    }
  }
  double L = pairwise_sum(res, Ns);
  free(res);
  return L;
}

/*
 * Joint Hessian-vector product of E(x, delta) with the samples frozen:
 *   H [v_x; v_d] = sum_k c2_k (grad g_k . v_x + v_d,k) [grad g_k ; e_k]
 * c2 from ora_assemble (per sample, 0 for inactive).  v_d / out_d nullable. */
void ora_hvp(int Vs, int Ts, const double *xs, const int *ts, int Vm, const double *xm, const int *tm,
             int nq, const double *rule, const int *M, const double *c2, const double *vx,
             const double *vd, double *out_x, double *out_d) {
  int64_t Ns = (int64_t)Ts * nq, Vt = (int64_t)Vs + Vm;
  memset(out_x, 0, sizeof(double) * 3 * (size_t)Vt);
  for (int64_t k = 0; k < Ns; ++k) {
    if (out_d) out_d[k] = 0.0;
    if (M[k] < 0 || c2[k] == 0.0) continue;
    double g, bm[3], n[3];
    if (ora_sample_geom(xs, ts, xm, tm, nq, rule, k, M[k], &g, bm, n) != ORA_OK) continue;
    int T = (int)(k / nq), q = (int)(k % nq);
    double xi = rule[3 * q], eta = rule[3 * q + 1];
    double bs[3] = {1.0 - xi - eta, xi, eta};
    double dot = 0.0;
    for (int a = 0; a < 3; ++a) dot += -bs[a] * v_dot(n, vx + 3 * (int64_t)ts[3 * T + a]);
    for (int j = 0; j < 3; ++j) dot += bm[j] * v_dot(n, vx + 3 * ((int64_t)Vs + tm[3 * M[k] + j]));
    if (vd) dot += vd[k];
    double s = c2[k] * dot;
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) out_x[3 * (int64_t)ts[3 * T + a] + d] += s * (-bs[a]) * n[d];
    for (int j = 0; j < 3; ++j)
      for (int d = 0; d < 3; ++d) out_x[3 * ((int64_t)Vs + tm[3 * M[k] + j]) + d] += s * bm[j] * n[d];
    if (out_d) out_d[k] = s;
  }
}

/* ---------------------------------------------- linearised step bound
 * Eq. (ccd):  alpha_k = 0.9 g_k / (-grad g_k . dx) for grad g_k . dx < 0,
 * Eq. (global_ccd): alpha = min_k alpha_k over the active samples.
 * Returns +inf if no active sample approaches.  dxm nullable (static). */
double ora_step_linear(int Ts, const double *xs, const int *ts, const double *xm, const int *tm,
                       int nq, const double *rule, const int *M, const double *dxs, const double *dxm) {
  int64_t Ns = (int64_t)Ts * nq;
  double alpha = INFINITY;
  for (int64_t k = 0; k < Ns; ++k) {
    if (M[k] < 0) continue;
    double g, bm[3], n[3];
    if (ora_sample_geom(xs, ts, xm, tm, nq, rule, k, M[k], &g, bm, n) != ORA_OK) continue;
    int T = (int)(k / nq), q = (int)(k % nq);
    double xi = rule[3 * q], eta = rule[3 * q + 1];
    double bs[3] = {1.0 - xi - eta, xi, eta};
    double gd = 0.0;
    for (int a = 0; a < 3; ++a) gd -= bs[a] * v_dot(n, dxs + 3 * (int64_t)ts[3 * T + a]);
    if (dxm)
      for (int j = 0; j < 3; ++j) gd += bm[j] * v_dot(n, dxm + 3 * (int64_t)tm[3 * M[k] + j]);
    if (gd < 0.0) {
      double a = 0.9 * g / (-gd);
      if (a < alpha) alpha = a;
    }
  }
  return alpha;
}

/* ------------------------------------------- point-triangle distance */
static double seg_dist2(const double *p, const double *a, const double *b) {
  double ab[3], ap[3];
  v_sub(b, a, ab);
  v_sub(p, a, ap);
  double l2 = v_dot(ab, ab);
  double t = l2 > 0.0 ? v_dot(ap, ab) / l2 : 0.0;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  double d[3] = {ap[0] - t * ab[0], ap[1] - t * ab[1], ap[2] - t * ab[2]};
  return v_dot(d, d);
}

/* squared distance from p to the closed triangle (a, b, c): the plane
 * distance if the foot point is inside, else the nearest edge distance. */
double ora_point_tri_dist2(const double *p, const double *a, const double *b, const double *c) {
  double e1[3], e2[3], N[3], r[3];
  v_sub(b, a, e1);
  v_sub(c, a, e2);
  v_cross(e1, e2, N);
  double nn = v_dot(N, N);
  if (nn > 0.0) {
    v_sub(p, a, r);
    double s = v_dot(r, N) / nn;
    double f[3] = {r[0] - s * N[0], r[1] - s * N[1], r[2] - s * N[2]};
    double a11 = v_dot(e1, e1), a12 = v_dot(e1, e2), a22 = v_dot(e2, e2);
    double r1 = v_dot(f, e1), r2 = v_dot(f, e2);
    double det = a11 * a22 - a12 * a12;
    if (det > 0.0) {
      double b1 = (a22 * r1 - a12 * r2) / det, b2 = (a11 * r2 - a12 * r1) / det;
      if (b1 >= 0.0 && b2 >= 0.0 && b1 + b2 <= 1.0) return s * s * nn;
    }
  }
  double d = seg_dist2(p, a, b), d2 = seg_dist2(p, b, c), d3 = seg_dist2(p, c, a);
  if (d2 < d) d = d2;
  if (d3 < d) d = d3;
  return d;
}

/*
 * Additive CCD for a point p moving by dp against a triangle (a,b,c) moving
 * by (da,db,dc), thickness 0, separation ratio s, horizon tmax.
 * Following the published description: remove the common mean
 * displacement; bound the relative speed by |dp| + max|d_tri|; starting at
 * t = 0, repeatedly advance by a step that cannot close the current
 * distance (first (1-s) d0 / l, later 0.9 d / l), and stop at the first
 * configuration whose distance falls below s d0, returning the time reached
 * before that step.  Returns tmax when the pair does not come closer than
 * s d0 before tmax.  Returns 0 if the pair already touches.               */
double ora_accd(const double *p, const double *dp, const double *a, const double *da, const double *b,
                const double *db, const double *c, const double *dc, double s, double tmax) {
  double mean[3], u[4][3];
  for (int d = 0; d < 3; ++d) {
    mean[d] = 0.25 * (dp[d] + da[d] + db[d] + dc[d]);
    u[0][d] = dp[d] - mean[d];
    u[1][d] = da[d] - mean[d];
    u[2][d] = db[d] - mean[d];
    u[3][d] = dc[d] - mean[d];
  }
  double lt = v_norm(u[1]);
  if (v_norm(u[2]) > lt) lt = v_norm(u[2]);
  if (v_norm(u[3]) > lt) lt = v_norm(u[3]);
  double l = v_norm(u[0]) + lt;
  if (l == 0.0) return tmax;
  double x[4][3];
  for (int d = 0; d < 3; ++d) {
    x[0][d] = p[d];
    x[1][d] = a[d];
    x[2][d] = b[d];
    x[3][d] = c[d];
  }
  double dist = sqrt(ora_point_tri_dist2(x[0], x[1], x[2], x[3]));
  if (dist <= 0.0) return 0.0;
  double gmin = s * dist;
  double t = 0.0;
  double step = (1.0 - s) * dist / l;
  for (long it = 0; it < 100000000L; ++it) {
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) x[v][d] += step * u[v][d];
    dist = sqrt(ora_point_tri_dist2(x[0], x[1], x[2], x[3]));
    if (t > 0.0 && dist < gmin) break;
    t += step;
    if (t > tmax) return tmax;
    step = 0.9 * dist / l;
  }
  return t;
}

/*
 * Step bound over one assembly's current state:
 *   alpha = min(1, min over active samples of Eq. (ccd),
 *               min over swept (sample point, master triangle) pairs of ACCD)
 * A swept pair is one whose axis-aligned boxes over the motion overlap:
 * the segment x_s,k -> x_s,k + dx_s,k against the box of the triangle's
 * six positions at t = 0 and t = 1.  dxm nullable.  *n_swept receives the
 * pair count, *alpha_lin the linear bound (+inf if none).                 */
double ora_ccd_step(int Vs, int Ts, const double *xs, const int *ts, int Vm, int Tm, const double *xm,
                    const int *tm, int nq, const double *rule, const int *M, const double *dxs,
                    const double *dxm, double s_accd, int use_grid, int64_t *n_swept,
                    double *alpha_lin, double *alpha_accd) {
  (void)Vs;
  (void)Vm;
  double al = ora_step_linear(Ts, xs, ts, xm, tm, nq, rule, M, dxs, dxm);
  double *blo = (double *)malloc(sizeof(double) * 3 * (size_t)(Tm ? Tm : 1));
  double *bhi = (double *)malloc(sizeof(double) * 3 * (size_t)(Tm ? Tm : 1));
  for (int t = 0; t < Tm; ++t)
    for (int d = 0; d < 3; ++d) {
      double lo = 1e300, hi = -1e300;
      for (int j = 0; j < 3; ++j) {
        const double *v = xm + 3 * (int64_t)tm[3 * t + j];
        double v0 = v[d], v1 = v[d] + (dxm ? dxm[3 * (int64_t)tm[3 * t + j] + d] : 0.0);
        if (v0 < lo) lo = v0;
        if (v0 > hi) hi = v0;
        if (v1 < lo) lo = v1;
        if (v1 > hi) hi = v1;
      }
      blo[3 * t + d] = lo;
      bhi[3 * t + d] = hi;
    }
  ogrid grid;
  int have_grid = use_grid ? ogrid_build(&grid, Tm, blo, bhi, 0.0) : 0;
  double amin = INFINITY;
  int64_t npairs = 0;
  static const double zero3[3] = {0, 0, 0};
#pragma omp parallel reduction(min : amin) reduction(+ : npairs)
  {
    int cap = Tm > 0 ? Tm : 1;
    int *stamp = NULL;
    int *cand = (int *)malloc(sizeof(int) * (size_t)cap);
    if (have_grid) {
      stamp = (int *)malloc(sizeof(int) * (size_t)cap);
      for (int i = 0; i < Tm; ++i) stamp[i] = -1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int T = 0; T < Ts; ++T) {
      const double *A = xs + 3 * (int64_t)ts[3 * T], *Bv = xs + 3 * (int64_t)ts[3 * T + 1],
                   *C = xs + 3 * (int64_t)ts[3 * T + 2];
      const double *dA = dxs + 3 * (int64_t)ts[3 * T], *dB = dxs + 3 * (int64_t)ts[3 * T + 1],
                   *dC = dxs + 3 * (int64_t)ts[3 * T + 2];
      for (int q = 0; q < nq; ++q) {
        int64_t k = (int64_t)T * nq + q;
        double xi = rule[3 * q], eta = rule[3 * q + 1], b0 = 1.0 - xi - eta;
        double p[3], dp[3], lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
          p[d] = b0 * A[d] + xi * Bv[d] + eta * C[d];
          dp[d] = b0 * dA[d] + xi * dB[d] + eta * dC[d];
          double e = p[d] + dp[d];
          lo[d] = p[d] < e ? p[d] : e;
          hi[d] = p[d] > e ? p[d] : e;
        }
        int nc;
        if (have_grid) {
          nc = ogrid_query(&grid, lo, hi, blo, bhi, stamp, (int)(k & 0x7fffffff), cand, cap);
        } else {
          nc = 0;
          for (int t = 0; t < Tm; ++t) {
            const double *a = blo + 3 * t, *b = bhi + 3 * t;
            if (a[0] > hi[0] || b[0] < lo[0] || a[1] > hi[1] || b[1] < lo[1] || a[2] > hi[2] || b[2] < lo[2])
              continue;
            cand[nc++] = t;
          }
        }
        for (int c = 0; c < nc; ++c) {
          int t = cand[c];
          const int *v = tm + 3 * (int64_t)t;
          const double *d0 = dxm ? dxm + 3 * (int64_t)v[0] : zero3;
          const double *d1 = dxm ? dxm + 3 * (int64_t)v[1] : zero3;
          const double *d2 = dxm ? dxm + 3 * (int64_t)v[2] : zero3;
          double a = ora_accd(p, dp, xm + 3 * (int64_t)v[0], d0, xm + 3 * (int64_t)v[1], d1,
                              xm + 3 * (int64_t)v[2], d2, s_accd, 1.0);
          if (a < amin) amin = a;
          npairs += 1;
        }
      }
    }
    free(stamp);
    free(cand);
  }
  if (have_grid) ogrid_free(&grid);
  free(blo);
  free(bhi);
  *n_swept = npairs;
  *alpha_lin = al;
  *alpha_accd = amin;
  double alpha = 1.0;
  if (al < alpha) alpha = al;
  if (amin < alpha) alpha = amin;
  return alpha;
}

/* ------------------------------------------------ swept-pair count
 * Number of (sample point, master triangle) pairs whose axis-aligned boxes
 * over the linear motion t in [0, 1] overlap: the pair set that additive CCD
 * runs over in the step bound (the count ora_ccd_step reports as n_swept).
 * With pad_rel = pad_abs = 0 this is that definition.  A positive margin
 * grows every box (both the point's and the triangle's) outward by
 * pad_rel * |coordinate| + pad_abs per bound, which gives the count for
 * boxes widened by a rounding margin: an upper bound for an implementation
 * that rounds its boxes outward by no more than that.                   */
int64_t ora_swept_count(int Ts, const double *xs, const int *ts, int Tm, const double *xm, const int *tm,
                        int nq, const double *rule, const double *dxs, const double *dxm, double pad_rel,
                        double pad_abs, int use_grid) {
  double *blo = (double *)malloc(sizeof(double) * 3 * (size_t)(Tm ? Tm : 1));
  double *bhi = (double *)malloc(sizeof(double) * 3 * (size_t)(Tm ? Tm : 1));
  for (int t = 0; t < Tm; ++t)
    for (int d = 0; d < 3; ++d) {
      double lo = 1e300, hi = -1e300;
      for (int j = 0; j < 3; ++j) {
        const int64_t v = tm[3 * t + j];
        double v0 = xm[3 * v + d], v1 = v0 + (dxm ? dxm[3 * v + d] : 0.0);
        double l0 = v0 - (pad_rel * fabs(v0) + pad_abs), h0 = v0 + (pad_rel * fabs(v0) + pad_abs);
        double l1 = v1 - (pad_rel * fabs(v1) + pad_abs), h1 = v1 + (pad_rel * fabs(v1) + pad_abs);
        if (l0 < lo) lo = l0;
        if (l1 < lo) lo = l1;
        if (h0 > hi) hi = h0;
        if (h1 > hi) hi = h1;
      }
      blo[3 * t + d] = lo;
      bhi[3 * t + d] = hi;
    }
  ogrid grid;
  int have_grid = use_grid ? ogrid_build(&grid, Tm, blo, bhi, 0.0) : 0;
  int64_t npairs = 0;
#pragma omp parallel reduction(+ : npairs)
  {
    int cap = Tm > 0 ? Tm : 1;
    int *cand = (int *)malloc(sizeof(int) * (size_t)cap);
    int *stamp = NULL;
    if (have_grid) {
      stamp = (int *)malloc(sizeof(int) * (size_t)cap);
      for (int i = 0; i < Tm; ++i) stamp[i] = -1;
    }
#pragma omp for schedule(dynamic, 64)
    for (int T = 0; T < Ts; ++T) {
      const double *A = xs + 3 * (int64_t)ts[3 * T], *B = xs + 3 * (int64_t)ts[3 * T + 1],
                   *C = xs + 3 * (int64_t)ts[3 * T + 2];
      const double *dA = dxs + 3 * (int64_t)ts[3 * T], *dB = dxs + 3 * (int64_t)ts[3 * T + 1],
                   *dC = dxs + 3 * (int64_t)ts[3 * T + 2];
      for (int q = 0; q < nq; ++q) {
        int64_t k = (int64_t)T * nq + q;
        double xi = rule[3 * q], eta = rule[3 * q + 1], b0 = 1.0 - xi - eta;
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
          double p = b0 * A[d] + xi * B[d] + eta * C[d];
          double e = p + (b0 * dA[d] + xi * dB[d] + eta * dC[d]);
          double l = p < e ? p : e, h = p > e ? p : e;
          lo[d] = l - (pad_rel * fabs(l) + pad_abs);
          hi[d] = h + (pad_rel * fabs(h) + pad_abs);
        }
        if (have_grid) {
          npairs += ogrid_query(&grid, lo, hi, blo, bhi, stamp, (int)(k & 0x7fffffff), cand, 0);
        } else {
          for (int t = 0; t < Tm; ++t) {
            const double *a = blo + 3 * t, *b = bhi + 3 * t;
            if (a[0] > hi[0] || b[0] < lo[0] || a[1] > hi[1] || b[1] < lo[1] || a[2] > hi[2] || b[2] < lo[2])
              continue;
            ++npairs;
          }
        }
      }
    }
    free(stamp);
    free(cand);
  }
  if (have_grid) ogrid_free(&grid);
  free(blo);
  free(bhi);
  return npairs;
}

/* Thread count of the OpenMP loops above (for timing at 1 and at n threads). */
void ora_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

int ora_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
