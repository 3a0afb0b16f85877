/* Drives every entry point of the FP64 oracle (oracle/gmcp_oracle.c) on a
 * small synthetic contact scene, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer on the CPU (test infrastructure only; built
 * and run by tests/test_oracle_sanitize.py).  Exits non-zero if an entry
 * point reports an unexpected status; the sanitizers abort on a memory or
 * undefined-behaviour error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int ora_narrow(int, int, const double *, const int *, int, int, const double *, const int *, int, const double *,
               double, const double *, int, int *, double *, double *, int *, int64_t *);
int ora_assemble(int, int, const double *, const int *, int, int, const double *, const int *, int, const double *,
                 const double *, double, double, double, const double *, const double *, const int *, int, int,
                 double *, double *, double *, double *, double *, double *, int64_t, int64_t *, int64_t *, double *,
                 int64_t *, double *, int64_t *);
double ora_pressure_loss(int, int, const double *, const int *, int, const double *, const int *, int, const double *,
                         double, double, double, const double *, const double *, const int *, const double *,
                         double *, double *);
void ora_hvp(int, int, const double *, const int *, int, const double *, const int *, int, const double *,
             const int *, const double *, const double *, const double *, double *, double *);
double ora_step_linear(int, const double *, const int *, const double *, const int *, int, const double *,
                       const int *, const double *, const double *);
double ora_ccd_step(int, int, const double *, const int *, int, int, const double *, const int *, int,
                    const double *, const int *, const double *, const double *, double, int, int64_t *, double *,
                    double *);
int64_t ora_swept_count(int, const double *, const int *, int, const double *, const int *, int, const double *,
                        const double *, const double *, double, double, int);
void ora_rest_area(int, const double *, const int *, double *);
double ora_psd_project(int, double *);
double ora_local_block12(double, const double *, const double *, double *);
double ora_point_tri_dist2(const double *, const double *, const double *, const double *);
double ora_accd(const double *, const double *, const double *, const double *, const double *, const double *,
                const double *, const double *, double, double);
int ora_sample_geom(const double *, const int *, const double *, const int *, int, const double *, int64_t, int,
                    double *, double *, double *);

/* n x n quad grid over [-L/2, L/2]^2 at height z(x, y); two triangles per
 * quad, counter-clockwise seen from +z (flip != 0: seen from -z) */
static void grid(int n, double L, double z0, double tilt, int flip, double *x, int *t) {
  for (int i = 0; i <= n; ++i)
    for (int j = 0; j <= n; ++j) {
      double *p = x + 3 * (i * (n + 1) + j);
      p[0] = -0.5 * L + L * i / n;
      p[1] = -0.5 * L + L * j / n;
      p[2] = z0 + tilt * p[0] + 1e-6 * sin(7.0 * i + 3.0 * j);
    }
  int k = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      int a = i * (n + 1) + j, b = (i + 1) * (n + 1) + j, c = (i + 1) * (n + 1) + j + 1, d = i * (n + 1) + j + 1;
      int tr[2][3] = {{a, b, c}, {a, c, d}};
      for (int s = 0; s < 2; ++s) {
        t[3 * k] = tr[s][0];
        t[3 * k + 1] = flip ? tr[s][2] : tr[s][1];
        t[3 * k + 2] = flip ? tr[s][1] : tr[s][2];
        ++k;
      }
    }
}

int main(void) {
  const int ns = 6, nm = 5, Vs = (ns + 1) * (ns + 1), Ts = 2 * ns * ns, Vm = (nm + 1) * (nm + 1), Tm = 2 * nm * nm;
  const double dhat = 1e-3, kappa = 1e5;
  /* 3-point rule with positive weights (sum 1/2): (xi, eta, w) */
  const double rule[9] = {1.0 / 6, 1.0 / 6, 1.0 / 6, 2.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 2.0 / 3, 1.0 / 6};
  const int nq = 3;
  const int64_t Ns = (int64_t)Ts * nq;
  double *xs = malloc(sizeof(double) * 3 * Vs), *xm = malloc(sizeof(double) * 3 * Vm);
  int *ts = malloc(sizeof(int) * 3 * Ts), *tm = malloc(sizeof(int) * 3 * Tm);
  grid(ns, 1e-2, 0.0, 0.0, 0, xs, ts);
  grid(nm, 1.3e-2, 5e-4, 0.04, 1, xm, tm); /* tilted punch: gaps from about 2.4e-4 to 7.6e-4 */
  double *area = malloc(sizeof(double) * Ts);
  ora_rest_area(Ts, xs, ts, area);
  int *M = malloc(sizeof(int) * Ns), *M2 = malloc(sizeof(int) * Ns), *fl = malloc(sizeof(int) * Ns);
  double *g = malloc(sizeof(double) * Ns), *bm = malloc(sizeof(double) * 3 * Ns);
  int64_t bad = -1;
  int bad_runs = 0;
  for (int use_grid = 0; use_grid < 2; ++use_grid) {
    int rc = ora_narrow(Vs, Ts, xs, ts, Vm, Tm, xm, tm, nq, rule, dhat, NULL, use_grid, use_grid ? M2 : M, g, bm, fl,
                        &bad);
    if (rc != 0) bad_runs++;
  }
  int act = 0;
  for (int64_t k = 0; k < Ns; ++k) {
    if (M[k] != M2[k]) bad_runs++;
    act += M[k] >= 0;
  }
  if (act < Ns / 2) bad_runs++;
  double *gref = malloc(sizeof(double) * Ns), *dgap = malloc(sizeof(double) * Ns);
  for (int64_t k = 0; k < Ns; ++k) {
    gref[k] = 2e-3;
    dgap[k] = 1e-7;
  }
  const int Vt = Vs + Vm;
  double *Ek = malloc(sizeof(double) * Ns), *c1 = malloc(sizeof(double) * Ns), *c2 = malloc(sizeof(double) * Ns),
         *pr = malloc(sizeof(double) * Ns), *grad = malloc(sizeof(double) * 3 * Vt);
  const int64_t cap = 36 * (int64_t)Ns;
  int64_t *rp = malloc(sizeof(int64_t) * (Vt + 1)), *col = malloc(sizeof(int64_t) * cap), nnzb = 0;
  double *val = malloc(sizeof(double) * 9 * cap), E = 0, clamped = 0;
  for (int kin = 0; kin < 2; ++kin)
    for (int hess = 0; hess < 2; ++hess) {
      int rc = ora_assemble(Vs, Ts, xs, ts, Vm, Tm, xm, tm, nq, rule, area, kappa, dhat, 0.05, kin ? gref : NULL,
                            kin ? dgap : NULL, M, kin, 1, &E, Ek, c1, c2, pr, grad, hess ? cap : 0,
                            hess ? rp : NULL, hess ? col : NULL, hess ? val : NULL, &nnzb, &clamped, &bad);
      if (rc != 0 || !(E > 0)) bad_runs++;
    }
  double *pt = malloc(sizeof(double) * Ns), *dLdx = malloc(sizeof(double) * 3 * Vt), *dLdd = malloc(sizeof(double) * Ns);
  for (int64_t k = 0; k < Ns; ++k) pt[k] = 1e3;
  double Lp = ora_pressure_loss(Vs, Ts, xs, ts, Vm, xm, tm, nq, rule, kappa, dhat, 0.0, NULL, dgap, M, pt, dLdx, dLdd);
  if (!(Lp > 0)) bad_runs++;
  double *vx = malloc(sizeof(double) * 3 * Vt), *ox = malloc(sizeof(double) * 3 * Vt), *od = malloc(sizeof(double) * Ns);
  for (int i = 0; i < 3 * Vt; ++i) vx[i] = sin(0.3 * i);
  ora_hvp(Vs, Ts, xs, ts, Vm, xm, tm, nq, rule, M, c2, vx, dgap, ox, od);
  double *dxs = malloc(sizeof(double) * 3 * Vs), *dxm = malloc(sizeof(double) * 3 * Vm);
  for (int i = 0; i < 3 * Vs; ++i) dxs[i] = (i % 3 == 2) ? 1e-4 : 2e-5 * cos(i);
  for (int i = 0; i < 3 * Vm; ++i) dxm[i] = (i % 3 == 2) ? -2e-4 : 1e-5 * sin(i);
  double al = ora_step_linear(Ts, xs, ts, xm, tm, nq, rule, M, dxs, dxm);
  if (!(al > 0)) bad_runs++;
  int64_t nsw[2] = {0, 0};
  double alin = 0, aacc = 0;
  for (int use_grid = 0; use_grid < 2; ++use_grid) {
    double a = ora_ccd_step(Vs, Ts, xs, ts, Vm, Tm, xm, tm, nq, rule, M, dxs, dxm, 0.1, use_grid, &nsw[use_grid],
                            &alin, &aacc);
    if (!(a > 0 && a <= 1)) bad_runs++;
    if (ora_swept_count(Ts, xs, ts, Tm, xm, tm, nq, rule, dxs, dxm, 0.0, 0.0, use_grid) != nsw[use_grid]) bad_runs++;
  }
  if (nsw[0] != nsw[1] || ora_swept_count(Ts, xs, ts, Tm, xm, tm, nq, rule, dxs, NULL, 1e-6, 1e-11, 1) < 0) bad_runs++;
  double H[144], H2[144], bmv[3] = {0.2, 0.3, 0.5}, nv[3] = {0, 0, 1};
  ora_local_block12(3.0, bmv, nv, H);
  for (int i = 0; i < 144; ++i) H2[i] = H[i] - (i % 13 == 0 ? 0.1 : 0.0);
  ora_psd_project(12, H2);
  const double p[3] = {0.1, 0.2, 0.3}, a[3] = {0, 0, 0}, b[3] = {1, 0, 0}, c[3] = {0, 1, 0};
  const double dp[3] = {0, 0, -0.5}, z[3] = {0, 0, 0};
  if (!(ora_point_tri_dist2(p, a, b, c) > 0)) bad_runs++;
  if (!(ora_accd(p, dp, a, z, b, z, c, z, 0.1, 1.0) > 0)) bad_runs++;
  double gk, bmk[3], nk[3];
  for (int64_t k = 0; k < Ns; ++k)
    if (M[k] >= 0 && ora_sample_geom(xs, ts, xm, tm, nq, rule, k, M[k], &gk, bmk, nk) != 0) bad_runs++;
  printf("active %d of %lld, nnzb %lld, swept %lld, alpha_lin %.6g, bad %d\n", act, (long long)Ns, (long long)nnzb,
         (long long)nsw[1], al, bad_runs);
  free(xs); free(xm); free(ts); free(tm); free(area); free(M); free(M2); free(fl); free(g); free(bm);
  free(gref); free(dgap); free(Ek); free(c1); free(c2); free(pr); free(grad); free(rp); free(col); free(val);
  free(pt); free(dLdx); free(dLdd); free(vx); free(ox); free(od); free(dxs); free(dxm);
  return bad_runs == 0 ? 0 : 1;
}
