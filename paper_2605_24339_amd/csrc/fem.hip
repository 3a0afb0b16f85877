// Implicit-step system around the contact potential: linear-elastic
// tetrahedra, lumped mass, block-Jacobi preconditioned CG on
//   A = M / dt^2 + K + H_contact,
// with Dirichlet vertices held fixed.  Double precision throughout.
//
// K is static: its 3x3 BSR pattern is the vertex adjacency of the tets and
// every block is the sum, in a fixed order, of the element blocks
//   K_e(a,b)_ik = vol (mu (gN_a . gN_b) d_ik + mu gN_b,i gN_a,k + lambda gN_a,i gN_b,k)
// of the tets containing both vertices (gN = gradients of the linear shape
// functions), so the assembled matrix is deterministic.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <vector>

#include "../../include/gmcp_fem.h"
#include "common.h"

namespace {

constexpr int kT = 256;

struct FemDev {
  int32_t *k_row_ptr, *k_col;  // static BSR pattern of K (V rows)
  double *k_val;               // [nnzb][9]
  int32_t *c_off, *c_list;     // per K block: contributions tet*16 + a*4 + b
  double *mass;                // [V] lumped mass
  uint8_t *fixed;              // [V] Dirichlet components: bit d = component d held
  double *X;                   // [V][3] rest positions
  int32_t *tets;               // [n_tet][4]
  double *Pinv;                // [V][9] block-Jacobi inverse
  double *r, *z, *p, *q;       // CG vectors [3V]
  double *partial;             // [nblk] partial dot products
  double *scal;                // [16] device scalars
};

}  // namespace

struct gmcp_fem {
  hipStream_t stream;
  int64_t V, n_tet, nnzb, nblk;
  double mu, lambda, rho, dt;
  FemDev d;
  std::vector<uint8_t> hfixed;  // host copy of the Dirichlet component masks
};

namespace {

__device__ inline void shape_grads(const double *X, const int32_t *tet, double g[4][3], double *vol) {
  double a[3], b[3], c[3];
  const double *x0 = X + 3 * (int64_t)tet[0];
  for (int d = 0; d < 3; ++d) {
    a[d] = X[3 * (int64_t)tet[1] + d] - x0[d];
    b[d] = X[3 * (int64_t)tet[2] + d] - x0[d];
    c[d] = X[3 * (int64_t)tet[3] + d] - x0[d];
  }
  // Dm = [a b c] (columns); rows of Dm^{-1} are the gradients of N_1..N_3
  double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - b[0] * (a[1] * c[2] - a[2] * c[1]) +
               c[0] * (a[1] * b[2] - a[2] * b[1]);
  double id = 1.0 / det;
  // inverse rows = (b x c, c x a, a x b) / det
  double r1[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
  double r2[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
  double r3[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  for (int d = 0; d < 3; ++d) {
    g[1][d] = r1[d] * id;
    g[2][d] = r2[d] * id;
    g[3][d] = r3[d] * id;
    g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
  }
  *vol = fabs(det) / 6.0;
}

__global__ void k_kvals(const double *X, const int32_t *tets, const int32_t *c_off, const int32_t *c_list,
                        int64_t nnzb, double mu, double lambda, double *k_val) {
  int64_t bk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (bk >= nnzb) return;
  double K[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int c = c_off[bk]; c < c_off[bk + 1]; ++c) {
    int code = c_list[c];
    int t = code >> 4, a = (code >> 2) & 3, b = code & 3;
    double g[4][3], vol;
    shape_grads(X, tets + 4 * (int64_t)t, g, &vol);
    double dab = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k)
        K[3 * i + k] += vol * (mu * (i == k ? dab : 0.0) + mu * g[b][i] * g[a][k] + lambda * g[a][i] * g[b][k]);
  }
  for (int z = 0; z < 9; ++z) k_val[9 * bk + z] = K[z];
}

// component d of vertex c, 0 when that component is held (Dirichlet
// columns removed)
__device__ inline void free_part(const double *x, const uint8_t *fixed, int64_t c, double v[3]) {
  const int m = fixed[c];
  for (int d = 0; d < 3; ++d) v[d] = (m >> d) & 1 ? 0.0 : x[3 * c + d];
}

// y = (M/dt^2) x + K x + H x (H optional) over the free components; 0 in
// the held ones
__global__ void k_apply(const int32_t *__restrict__ krp, const int32_t *__restrict__ kcol,
                        const double *__restrict__ kval, const int32_t *__restrict__ hrp,
                        const int32_t *__restrict__ hcol, const double *__restrict__ hval,
                        const double *__restrict__ mass, const uint8_t *__restrict__ fixed, double inv_dt2,
                        const double *__restrict__ x, double *__restrict__ y, int64_t V) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  const int mi = fixed[i];
  if (mi == 7) {
    y[3 * i] = y[3 * i + 1] = y[3 * i + 2] = 0.0;
    return;
  }
  double s[3], v[3];
  free_part(x, fixed, i, v);
  for (int d = 0; d < 3; ++d) s[d] = mass[i] * inv_dt2 * v[d];
  for (int j = krp[i]; j < krp[i + 1]; ++j) {
    int64_t c = kcol[j];
    if (fixed[c] == 7) continue;
    free_part(x, fixed, c, v);
    const double *B = kval + 9 * (int64_t)j;
    for (int r = 0; r < 3; ++r) s[r] += B[3 * r] * v[0] + B[3 * r + 1] * v[1] + B[3 * r + 2] * v[2];
  }
  if (hrp) {
    for (int j = hrp[i]; j < hrp[i + 1]; ++j) {
      int64_t c = hcol[j];
      if (fixed[c] == 7) continue;
      free_part(x, fixed, c, v);
      const double *B = hval + 9 * (int64_t)j;
      for (int r = 0; r < 3; ++r) s[r] += B[3 * r] * v[0] + B[3 * r + 1] * v[1] + B[3 * r + 2] * v[2];
    }
  }
  for (int d = 0; d < 3; ++d) y[3 * i + d] = (mi >> d) & 1 ? 0.0 : s[d];
}

__device__ inline bool inv3(const double *A, double *B) {
  double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
  double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  if (!(fabs(det) > 0.0)) return false;
  double id = 1.0 / det;
  B[0] = c00 * id;
  B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  B[3] = c01 * id;
  B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  B[6] = c02 * id;
  B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
  return true;
}

__global__ void k_jacobi(const int32_t *krp, const int32_t *kcol, const double *kval, const int32_t *hrp,
                         const int32_t *hcol, const double *hval, const double *mass, const uint8_t *fixed,
                         double inv_dt2, double *Pinv, int64_t V) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  double D[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int d = 0; d < 3; ++d) D[4 * d] = mass[i] * inv_dt2;
  for (int j = krp[i]; j < krp[i + 1]; ++j)
    if (kcol[j] == i)
      for (int z = 0; z < 9; ++z) D[z] += kval[9 * (int64_t)j + z];
  if (hrp)
    for (int j = hrp[i]; j < hrp[i + 1]; ++j)
      if (hcol[j] == i)
        for (int z = 0; z < 9; ++z) D[z] += hval[9 * (int64_t)j + z];
  // held components: identity rows/columns for the inverse, zeroed after
  const int m = fixed[i];
  for (int d = 0; d < 3; ++d)
    if ((m >> d) & 1)
      for (int k = 0; k < 3; ++k) D[3 * d + k] = D[3 * k + d] = (k == d) ? 1.0 : 0.0;
  double P[9];
  if (m == 7 || !inv3(D, P))
    for (int z = 0; z < 9; ++z) P[z] = 0.0;
  for (int d = 0; d < 3; ++d)
    if ((m >> d) & 1)
      for (int k = 0; k < 3; ++k) P[3 * d + k] = P[3 * k + d] = 0.0;
  for (int z = 0; z < 9; ++z) Pinv[9 * i + z] = P[z];
}

// partial sums of a.b over blocks of 1024 entries (fixed order)
__global__ void k_dot_partial(const double *a, const double *b, int64_t n, double *partial) {
  __shared__ double s[kT];
  int64_t base = (int64_t)blockIdx.x * 1024;
  double v = 0.0;
  for (int k = 0; k < 4; ++k) {
    int64_t j = base + k * kT + threadIdx.x;
    if (j < n) v += a[j] * b[j];
  }
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ void k_sum_partial(const double *a, int64_t n, double *partial) {
  __shared__ double s[kT];
  int64_t base = (int64_t)blockIdx.x * 1024;
  double v = 0.0;
  for (int k = 0; k < 4; ++k) {
    int64_t j = base + k * kT + threadIdx.x;
    if (j < n) v += a[j];
  }
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ void k_dot_final(const double *partial, int64_t nblk, double *out) {
  __shared__ double s[kT];
  double v = 0.0;
  for (int64_t j = threadIdx.x; j < nblk; j += kT) v += partial[j];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// z = Pinv r (per vertex 3x3)
__global__ void k_precond(const double *Pinv, const double *r, double *z, int64_t V) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  const double *P = Pinv + 9 * i;
  for (int a = 0; a < 3; ++a) z[3 * i + a] = P[3 * a] * r[3 * i] + P[3 * a + 1] * r[3 * i + 1] + P[3 * a + 2] * r[3 * i + 2];
}

// scalars: s[0] = rz, s[1] = pq, s[2] = rz_new, s[3] = rr, s[4] = bb
// x += (rz/pq) p ; r -= (rz/pq) q
__global__ void k_cg_update_xr(const double *s, double *x, double *r, const double *p, const double *q, int64_t n) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double alpha = s[1] != 0.0 ? s[0] / s[1] : 0.0;
  x[j] += alpha * p[j];
  r[j] -= alpha * q[j];
}

// p = z + (rz_new/rz) p ; then rz <- rz_new (one thread does it after use)
__global__ void k_cg_update_p(double *s, const double *z, double *p, int64_t n) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double beta = s[0] != 0.0 ? s[2] / s[0] : 0.0;
  p[j] = z[j] + beta * p[j];
}

__global__ void k_cg_roll(double *s) {
  if (threadIdx.x == 0 && blockIdx.x == 0) s[0] = s[2];
}

__global__ void k_copy_mask(const double *src, double *dst, const uint8_t *fixed, int64_t V, double scale) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  for (int d = 0; d < 3; ++d) dst[3 * i + d] = (fixed[i] >> d) & 1 ? 0.0 : scale * src[3 * i + d];
}

__global__ void k_zero(double *p, int64_t n) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) p[j] = 0.0;
}

// elastic + inertial energy terms per vertex and gradient:
//   g_i = m_i (x_i - xt_i)/dt^2 + (K (x - X))_i ; 0 in held components
//   e_i = 1/2 m_i |x_i - xt_i|^2 / dt^2 + 1/2 u_i . (K u)_i
__global__ void k_fem_grad(const int32_t *krp, const int32_t *kcol, const double *kval, const double *mass,
                           const uint8_t *fixed, double inv_dt2, const double *X, const double *x,
                           const double *xt, double *g, double *e, int64_t V) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  double ku[3] = {0, 0, 0};
  for (int j = krp[i]; j < krp[i + 1]; ++j) {
    int64_t c = kcol[j];
    const double *B = kval + 9 * (int64_t)j;
    double u[3] = {x[3 * c] - X[3 * c], x[3 * c + 1] - X[3 * c + 1], x[3 * c + 2] - X[3 * c + 2]};
    for (int r = 0; r < 3; ++r) ku[r] += B[3 * r] * u[0] + B[3 * r + 1] * u[1] + B[3 * r + 2] * u[2];
  }
  double ei = 0.0;
  for (int d = 0; d < 3; ++d) {
    double dv = x[3 * i + d] - xt[3 * i + d];
    double ui = x[3 * i + d] - X[3 * i + d];
    ei += 0.5 * mass[i] * inv_dt2 * dv * dv + 0.5 * ui * ku[d];
    if (g) g[3 * i + d] = (fixed[i] >> d) & 1 ? 0.0 : mass[i] * inv_dt2 * dv + ku[d];
  }
  e[i] = ei;
}

inline unsigned nb(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

struct FemPlan {
  size_t off = 0;
  char *base = nullptr;
  template <typename T>
  T *take(int64_t n) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += sizeof(T) * (size_t)(n > 0 ? n : 1);
    return p;
  }
};

struct FemTopo {
  std::vector<int32_t> rp, col, coff, clist;
};

void fem_topology(const int32_t *tets, int64_t n_tet, int64_t V, FemTopo &t) {
  std::vector<std::map<int32_t, std::vector<int32_t>>> rows(V);
  for (int64_t e = 0; e < n_tet; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) rows[tets[4 * e + a]][tets[4 * e + b]].push_back((int32_t)(e * 16 + a * 4 + b));
  t.rp.assign(V + 1, 0);
  for (int64_t i = 0; i < V; ++i) t.rp[i + 1] = t.rp[i] + (int32_t)rows[i].size();
  t.col.clear();
  t.coff.assign(1, 0);
  t.clist.clear();
  for (int64_t i = 0; i < V; ++i)
    for (auto &kv : rows[i]) {
      t.col.push_back(kv.first);
      for (int32_t c : kv.second) t.clist.push_back(c);
      t.coff.push_back((int32_t)t.clist.size());
    }
}

size_t fem_plan(int64_t V, int64_t n_tet, int64_t nnzb, int64_t ncontrib, char *base, FemDev *d, int64_t *nblk) {
  FemPlan p;
  p.base = base;
  FemDev t{};
  int64_t n = 3 * V;
  int64_t blocks = (n + 1023) / 1024;
  t.k_row_ptr = p.take<int32_t>(V + 1);
  t.k_col = p.take<int32_t>(nnzb);
  t.k_val = p.take<double>(9 * nnzb);
  t.c_off = p.take<int32_t>(nnzb + 1);
  t.c_list = p.take<int32_t>(ncontrib);
  t.mass = p.take<double>(V);
  t.fixed = p.take<uint8_t>(V);
  t.X = p.take<double>(3 * V);
  t.tets = p.take<int32_t>(4 * n_tet);
  t.Pinv = p.take<double>(9 * V);
  t.r = p.take<double>(n);
  t.z = p.take<double>(n);
  t.p = p.take<double>(n);
  t.q = p.take<double>(n);
  t.partial = p.take<double>(blocks);
  t.scal = p.take<double>(16);
  if (d) *d = t;
  if (nblk) *nblk = blocks;
  return p.off + 256;
}

void dot(gmcp_fem *f, const double *a, const double *b, double *out) {
  int64_t n = 3 * f->V;
  hipLaunchKernelGGL(k_dot_partial, dim3((unsigned)f->nblk), dim3(kT), 0, f->stream, a, b, n, f->d.partial);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kT), 0, f->stream, f->d.partial, f->nblk, out);
}

}  // namespace

extern "C" {

size_t gmcp_fem_workspace_size(const int32_t *tets, int64_t n_tet, int64_t n_vert) {
  if (!tets || n_tet <= 0 || n_vert <= 0) return 0;
  for (int64_t i = 0; i < 4 * n_tet; ++i)
    if (tets[i] < 0 || tets[i] >= n_vert) return 0;
  FemTopo t;
  fem_topology(tets, n_tet, n_vert, t);
  return fem_plan(n_vert, n_tet, (int64_t)t.col.size(), (int64_t)t.clist.size(), nullptr, nullptr, nullptr);
}

int gmcp_fem_create(gmcp_fem **out, const int32_t *tets, int64_t n_tet, int64_t n_vert, const double *X_rest,
                    double young, double poisson, double density, double dt, const int32_t *fixed,
                    int64_t n_fixed, void *workspace, size_t bytes, void *stream) {
  if (!out || !X_rest || !(young > 0) || !(poisson > -1 && poisson < 0.5) || !(density > 0) || !(dt > 0))
    return GMCP_E_ARG;
  *out = nullptr;
  size_t need = gmcp_fem_workspace_size(tets, n_tet, n_vert);
  if (need == 0 || bytes < need || !workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return GMCP_E_ARG;
  for (int64_t i = 0; i < n_fixed; ++i)
    if (fixed[i] < 0 || fixed[i] >= n_vert) return GMCP_E_ARG;
  FemTopo t;
  fem_topology(tets, n_tet, n_vert, t);
  gmcp_fem *f = new (std::nothrow) gmcp_fem();
  if (!f) return GMCP_E_ARG;
  f->stream = (hipStream_t)stream;
  f->V = n_vert;
  f->n_tet = n_tet;
  f->nnzb = (int64_t)t.col.size();
  f->mu = young / (2.0 * (1.0 + poisson));
  f->lambda = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson));
  f->rho = density;
  f->dt = dt;
  fem_plan(n_vert, n_tet, f->nnzb, (int64_t)t.clist.size(), (char *)workspace, &f->d, &f->nblk);
  // lumped mass: rho vol / 4 per tet vertex
  std::vector<double> mass(n_vert, 0.0);
  for (int64_t e = 0; e < n_tet; ++e) {
    const double *x0 = X_rest + 3 * (int64_t)tets[4 * e];
    double a[3], b[3], c[3];
    for (int d = 0; d < 3; ++d) {
      a[d] = X_rest[3 * (int64_t)tets[4 * e + 1] + d] - x0[d];
      b[d] = X_rest[3 * (int64_t)tets[4 * e + 2] + d] - x0[d];
      c[d] = X_rest[3 * (int64_t)tets[4 * e + 3] + d] - x0[d];
    }
    double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - b[0] * (a[1] * c[2] - a[2] * c[1]) +
                 c[0] * (a[1] * b[2] - a[2] * b[1]);
    for (int k = 0; k < 4; ++k) mass[tets[4 * e + k]] += density * fabs(det) / 24.0;
  }
  std::vector<uint8_t> fx(n_vert, 0);
  for (int64_t i = 0; i < n_fixed; ++i) fx[fixed[i]] = 7;
  hipError_t e = hipSuccess;
  auto up = [&](void *dst, const void *src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpy(dst, src, n, hipMemcpyHostToDevice);
  };
  up(f->d.k_row_ptr, t.rp.data(), sizeof(int32_t) * t.rp.size());
  up(f->d.k_col, t.col.data(), sizeof(int32_t) * t.col.size());
  up(f->d.c_off, t.coff.data(), sizeof(int32_t) * t.coff.size());
  up(f->d.c_list, t.clist.data(), sizeof(int32_t) * t.clist.size());
  up(f->d.mass, mass.data(), sizeof(double) * n_vert);
  up(f->d.fixed, fx.data(), n_vert);
  f->hfixed = fx;
  up(f->d.X, X_rest, sizeof(double) * 3 * n_vert);
  up(f->d.tets, tets, sizeof(int32_t) * 4 * n_tet);
  if (e != hipSuccess) {
    delete f;
    return GMCP_E_HIP;
  }
  hipLaunchKernelGGL(k_kvals, dim3(nb(f->nnzb)), dim3(kT), 0, f->stream, f->d.X, f->d.tets, f->d.c_off, f->d.c_list,
                     f->nnzb, f->mu, f->lambda, f->d.k_val);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(f->stream) != hipSuccess) {
    delete f;
    return GMCP_E_HIP;
  }
  *out = f;
  return GMCP_OK;
}

void gmcp_fem_destroy(gmcp_fem *f) { delete f; }

int gmcp_fem_constrain(gmcp_fem *f, const int32_t *verts, int64_t n, int mask) {
  if (!f || n < 0 || (n > 0 && !verts) || mask < 1 || mask > 7) return GMCP_E_ARG;
  for (int64_t i = 0; i < n; ++i)
    if (verts[i] < 0 || verts[i] >= f->V) return GMCP_E_ARG;
  for (int64_t i = 0; i < n; ++i) f->hfixed[verts[i]] |= (uint8_t)mask;
  if (hipStreamSynchronize(f->stream) != hipSuccess ||
      hipMemcpy(f->d.fixed, f->hfixed.data(), (size_t)f->V, hipMemcpyHostToDevice) != hipSuccess)
    return GMCP_E_HIP;
  return GMCP_OK;
}

int gmcp_fem_set_stream(gmcp_fem *f, void *stream) {
  if (!f) return GMCP_E_ARG;
  f->stream = (hipStream_t)stream;
  return GMCP_OK;
}

int64_t gmcp_fem_nnzb(const gmcp_fem *f) { return f ? f->nnzb : -1; }

int gmcp_fem_stiffness(gmcp_fem *f, int32_t *row_ptr, int32_t *col, double *val) {
  if (!f || !row_ptr || !col || !val) return GMCP_E_ARG;
  hipError_t e = hipMemcpyAsync(row_ptr, f->d.k_row_ptr, sizeof(int32_t) * (f->V + 1), hipMemcpyDeviceToDevice, f->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(col, f->d.k_col, sizeof(int32_t) * f->nnzb, hipMemcpyDeviceToDevice, f->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(val, f->d.k_val, sizeof(double) * 9 * f->nnzb, hipMemcpyDeviceToDevice, f->stream);
  return e == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

int gmcp_fem_energy(gmcp_fem *f, const double *x, const double *x_tilde, double *energy, double *grad) {
  if (!f || !x || !x_tilde || !energy) return GMCP_E_ARG;
  double inv_dt2 = 1.0 / (f->dt * f->dt);
  // per-vertex energies land in z[0..V), then a fixed-order sum
  hipLaunchKernelGGL(k_fem_grad, dim3(nb(f->V)), dim3(kT), 0, f->stream, f->d.k_row_ptr, f->d.k_col, f->d.k_val,
                     f->d.mass, f->d.fixed, inv_dt2, f->d.X, x, x_tilde, grad, f->d.z, f->V);
  hipLaunchKernelGGL(k_sum_partial, dim3((unsigned)((f->V + 1023) / 1024)), dim3(kT), 0, f->stream, f->d.z, f->V,
                     f->d.partial);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kT), 0, f->stream, f->d.partial, (f->V + 1023) / 1024, energy);
  return hipGetLastError() == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

int gmcp_fem_solve(gmcp_fem *f, const int32_t *h_row_ptr, const int32_t *h_col, const double *h_val,
                   const double *rhs, double *x, double rtol, int max_iter, int *iters, double *rel_res) {
  if (!f || !rhs || !x || max_iter <= 0 || !(rtol > 0)) return GMCP_E_ARG;
  if ((h_row_ptr != nullptr) != (h_col != nullptr) || (h_col != nullptr) != (h_val != nullptr)) return GMCP_E_ARG;
  hipStream_t s = f->stream;
  const int64_t V = f->V, n = 3 * V;
  const double inv_dt2 = 1.0 / (f->dt * f->dt);
  FemDev &d = f->d;
  hipLaunchKernelGGL(k_jacobi, dim3(nb(V)), dim3(kT), 0, s, d.k_row_ptr, d.k_col, d.k_val, h_row_ptr, h_col, h_val,
                     d.mass, d.fixed, inv_dt2, d.Pinv, V);
  // x = 0, r = b (fixed rows masked), z = P r, p = z, rz = r.z, bb = b.b
  hipLaunchKernelGGL(k_zero, dim3(nb(n)), dim3(kT), 0, s, x, n);
  hipLaunchKernelGGL(k_copy_mask, dim3(nb(V)), dim3(kT), 0, s, rhs, d.r, d.fixed, V, 1.0);
  hipLaunchKernelGGL(k_precond, dim3(nb(V)), dim3(kT), 0, s, d.Pinv, d.r, d.z, V);
  hipLaunchKernelGGL(k_copy_mask, dim3(nb(V)), dim3(kT), 0, s, d.z, d.p, d.fixed, V, 1.0);
  dot(f, d.r, d.z, d.scal + 0);
  dot(f, d.r, d.r, d.scal + 4);
  double host[8];
  if (hipMemcpyAsync(host, d.scal, sizeof(double) * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GMCP_E_HIP;
  const double bb = host[4];
  int it = 0;
  double rr = bb;
  if (bb > 0.0) {
    for (it = 0; it < max_iter;) {
      hipLaunchKernelGGL(k_apply, dim3(nb(V)), dim3(kT), 0, s, d.k_row_ptr, d.k_col, d.k_val, h_row_ptr, h_col,
                         h_val, d.mass, d.fixed, inv_dt2, d.p, d.q, V);
      dot(f, d.p, d.q, d.scal + 1);
      hipLaunchKernelGGL(k_cg_update_xr, dim3(nb(n)), dim3(kT), 0, s, d.scal, x, d.r, d.p, d.q, n);
      hipLaunchKernelGGL(k_precond, dim3(nb(V)), dim3(kT), 0, s, d.Pinv, d.r, d.z, V);
      dot(f, d.r, d.z, d.scal + 2);
      hipLaunchKernelGGL(k_cg_update_p, dim3(nb(n)), dim3(kT), 0, s, d.scal, d.z, d.p, n);
      hipLaunchKernelGGL(k_cg_roll, dim3(1), dim3(64), 0, s, d.scal);
      ++it;
      if (it % 8 == 0 || it == max_iter) {
        dot(f, d.r, d.r, d.scal + 3);
        if (hipMemcpyAsync(host, d.scal, sizeof(double) * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return GMCP_E_HIP;
        rr = host[3];
        if (!(rr == rr)) return GMCP_E_NONFINITE;
        if (rr <= rtol * rtol * bb) break;
      }
    }
  }
  if (iters) *iters = it;
  if (rel_res) *rel_res = bb > 0.0 ? sqrt(rr / bb) : 0.0;
  return hipGetLastError() == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

// y = A x (for checks): A = M/dt^2 + K + H, fixed rows 0
int gmcp_fem_apply(gmcp_fem *f, const int32_t *h_row_ptr, const int32_t *h_col, const double *h_val, const double *x,
                   double *y) {
  if (!f || !x || !y) return GMCP_E_ARG;
  hipLaunchKernelGGL(k_apply, dim3(nb(f->V)), dim3(kT), 0, f->stream, f->d.k_row_ptr, f->d.k_col, f->d.k_val,
                     h_row_ptr, h_col, h_val, f->d.mass, f->d.fixed, 1.0 / (f->dt * f->dt), x, y, f->V);
  return hipGetLastError() == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

}  // extern "C"
