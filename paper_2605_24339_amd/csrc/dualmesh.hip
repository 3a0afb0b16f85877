// Dual-mesh mapper (Sec. 3): visual vertices embedded on the simulation
// surface by nearest triangle, barycentric coordinates of the plane
// projection and a signed normal offset (Eqs. (bary_proj), (decomp),
// (gram)); per frame they follow the deformed triangles (Eq. (bary_interp)).
//
// k_embed: one thread per visual vertex, FP64.  Each block streams the
// simulation triangles through LDS in tiles of 256 (vertex, edges, unit
// normal, Gram entries and inverses, bounding sphere), and every thread
// scans them in ascending order keeping the strict minimum, so ties go to
// the smaller index.  A triangle whose bounding sphere lies farther than
// the best distance so far is skipped without the exact test (it cannot
// win); visual vertices that are adjacent in index order are usually
// adjacent in space, so whole waves skip together.
//
// k_update: one thread per visual vertex; three gathered simulation
// vertices (L2-resident for a surface of ~10^4-10^5 vertices), 32 B of
// mapping read and 12 B written per vertex in float.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/gmcp.h"
#include "../../include/gmcp_dualmesh.h"

namespace {

constexpr int kEmbedThreads = 256;

struct TriL {
  double a[3], e1[3], e2[3], n[3];
  double g11, g12, g22, inv_det, ig11, ig22, ie3;
  double c[3], rho;
};

__device__ inline double dot3(const double *x, const double *y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; }

// squared distance from p to triangle T (nearest point of the triangle)
__device__ inline double tri_dist2(const double p[3], const TriL &T) {
  double d[3] = {p[0] - T.a[0], p[1] - T.a[1], p[2] - T.a[2]};
  const double r1 = dot3(d, T.e1), r2 = dot3(d, T.e2);
  const double v = (T.g22 * r1 - T.g12 * r2) * T.inv_det;
  const double w = (T.g11 * r2 - T.g12 * r1) * T.inv_det;
  if (v >= 0.0 && w >= 0.0 && v + w <= 1.0) {
    const double dn = dot3(d, T.n);
    return dn * dn;
  }
  // nearest point on the boundary: edges a->b, a->c, b->c
  double best;
  {
    const double t = fmin(fmax(r1 * T.ig11, 0.0), 1.0);
    const double q0 = d[0] - t * T.e1[0], q1 = d[1] - t * T.e1[1], q2 = d[2] - t * T.e1[2];
    best = q0 * q0 + q1 * q1 + q2 * q2;
  }
  {
    const double t = fmin(fmax(r2 * T.ig22, 0.0), 1.0);
    const double q0 = d[0] - t * T.e2[0], q1 = d[1] - t * T.e2[1], q2 = d[2] - t * T.e2[2];
    best = fmin(best, q0 * q0 + q1 * q1 + q2 * q2);
  }
  {
    const double db[3] = {d[0] - T.e1[0], d[1] - T.e1[1], d[2] - T.e1[2]};
    const double e3[3] = {T.e2[0] - T.e1[0], T.e2[1] - T.e1[1], T.e2[2] - T.e1[2]};
    const double t = fmin(fmax(dot3(db, e3) * T.ie3, 0.0), 1.0);
    const double q0 = db[0] - t * e3[0], q1 = db[1] - t * e3[1], q2 = db[2] - t * e3[2];
    best = fmin(best, q0 * q0 + q1 * q1 + q2 * q2);
  }
  return best;
}

__global__ __launch_bounds__(kEmbedThreads) void k_embed(const double *__restrict__ P, int64_t N,
                                                         const double *__restrict__ V, const int32_t *__restrict__ F,
                                                         int64_t nT, int32_t *__restrict__ tri,
                                                         double *__restrict__ bary, double *__restrict__ delta,
                                                         double *__restrict__ dist2) {
  __shared__ TriL tl[kEmbedThreads];
  __shared__ int valid[kEmbedThreads];
  const int64_t i = (int64_t)blockIdx.x * kEmbedThreads + threadIdx.x;
  const bool live = i < N;
  double p[3] = {0.0, 0.0, 0.0};
  if (live)
    for (int k = 0; k < 3; ++k) p[k] = P[i * 3 + k];
  double best = INFINITY;
  int32_t bt = -1;
  for (int64_t t0 = 0; t0 < nT; t0 += kEmbedThreads) {
    __syncthreads();
    const int64_t t = t0 + threadIdx.x;
    int ok = 0;
    if (t < nT) {
      TriL &T = tl[threadIdx.x];
      double a[3], b[3], c[3];
      for (int k = 0; k < 3; ++k) {
        a[k] = V[(int64_t)F[t * 3 + 0] * 3 + k];
        b[k] = V[(int64_t)F[t * 3 + 1] * 3 + k];
        c[k] = V[(int64_t)F[t * 3 + 2] * 3 + k];
      }
      double e1[3], e2[3];
      for (int k = 0; k < 3; ++k) {
        e1[k] = b[k] - a[k];
        e2[k] = c[k] - a[k];
      }
      const double nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2],
                   nz = e1[0] * e2[1] - e1[1] * e2[0];
      const double nn = nx * nx + ny * ny + nz * nz;  // = Gram determinant
      ok = nn > 0.0 && isfinite(nn);
      const double inv_n = ok ? 1.0 / sqrt(nn) : 0.0;
      for (int k = 0; k < 3; ++k) {
        T.a[k] = a[k];
        T.e1[k] = e1[k];
        T.e2[k] = e2[k];
        T.c[k] = (a[k] + b[k] + c[k]) * (1.0 / 3.0);
      }
      T.n[0] = nx * inv_n;
      T.n[1] = ny * inv_n;
      T.n[2] = nz * inv_n;
      T.g11 = dot3(e1, e1);
      T.g12 = dot3(e1, e2);
      T.g22 = dot3(e2, e2);
      T.inv_det = ok ? 1.0 / (T.g11 * T.g22 - T.g12 * T.g12) : 0.0;
      const double e3[3] = {c[0] - b[0], c[1] - b[1], c[2] - b[2]};
      T.ig11 = ok ? 1.0 / T.g11 : 0.0;
      T.ig22 = ok ? 1.0 / T.g22 : 0.0;
      T.ie3 = ok ? 1.0 / dot3(e3, e3) : 0.0;
      double r = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double *q = k == 0 ? a : (k == 1 ? b : c);
        const double dx = q[0] - T.c[0], dy = q[1] - T.c[1], dz = q[2] - T.c[2];
        r = fmax(r, dx * dx + dy * dy + dz * dz);
      }
      T.rho = sqrt(r);
    }
    valid[threadIdx.x] = ok;
    __syncthreads();
    if (!live) continue;
    const int cnt = (int)((nT - t0) < kEmbedThreads ? (nT - t0) : kEmbedThreads);
    double sb = sqrt(best);
    for (int j = 0; j < cnt; ++j) {
      if (!valid[j]) continue;
      const TriL &T = tl[j];
      const double dx = p[0] - T.c[0], dy = p[1] - T.c[1], dz = p[2] - T.c[2];
      const double reach = (sb + T.rho) * (1.0 + 1e-12);
      if (dx * dx + dy * dy + dz * dz > reach * reach) continue;  // every point of T is farther than best
      const double d2 = tri_dist2(p, T);
      if (d2 < best) {
        best = d2;
        bt = (int32_t)(t0 + j);
        sb = sqrt(best);
      }
    }
  }
  if (!live) return;
  tri[i] = bt;
  if (dist2) dist2[i] = best;
  if (bt < 0) {
    for (int k = 0; k < 3; ++k) bary[i * 3 + k] = NAN;
    delta[i] = NAN;
    return;
  }
  // Eqs. (decomp), (gram) on the chosen triangle
  double a[3], e1[3], e2[3], d[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = V[(int64_t)F[(int64_t)bt * 3 + 0] * 3 + k];
    e1[k] = V[(int64_t)F[(int64_t)bt * 3 + 1] * 3 + k] - a[k];
    e2[k] = V[(int64_t)F[(int64_t)bt * 3 + 2] * 3 + k] - a[k];
    d[k] = p[k] - a[k];
  }
  const double g11 = dot3(e1, e1), g12 = dot3(e1, e2), g22 = dot3(e2, e2);
  const double r1 = dot3(d, e1), r2 = dot3(d, e2);
  const double det = g11 * g22 - g12 * g12;
  const double v = (g22 * r1 - g12 * r2) / det, w = (g11 * r2 - g12 * r1) / det;
  const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const double nl = sqrt(dot3(n, n));
  bary[i * 3 + 0] = 1.0 - v - w;
  bary[i * 3 + 1] = v;
  bary[i * 3 + 2] = w;
  delta[i] = dot3(d, n) / nl;
}

template <typename R>
__device__ inline R rsqrt_r(R x);
template <>
__device__ inline float rsqrt_r<float>(float x) {
  return rsqrtf(x);
}
template <>
__device__ inline double rsqrt_r<double>(double x) {
  return 1.0 / sqrt(x);
}

template <typename R>
__global__ __launch_bounds__(256) void k_update(const R *__restrict__ Vd, const int32_t *__restrict__ F,
                                                const int32_t *__restrict__ tri, const R *__restrict__ bary,
                                                const R *__restrict__ delta, int64_t N, R *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int64_t t = tri[i];
  const int64_t i0 = F[t * 3 + 0], i1 = F[t * 3 + 1], i2 = F[t * 3 + 2];
  const R ax = Vd[i0 * 3], ay = Vd[i0 * 3 + 1], az = Vd[i0 * 3 + 2];
  const R bx = Vd[i1 * 3], by = Vd[i1 * 3 + 1], bz = Vd[i1 * 3 + 2];
  const R cx = Vd[i2 * 3], cy = Vd[i2 * 3 + 1], cz = Vd[i2 * 3 + 2];
  const R e1x = bx - ax, e1y = by - ay, e1z = bz - az;
  const R e2x = cx - ax, e2y = cy - ay, e2z = cz - az;
  const R nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const R s = delta[i] * rsqrt_r<R>(nx * nx + ny * ny + nz * nz);
  const R u = bary[i * 3], v = bary[i * 3 + 1], w = bary[i * 3 + 2];
  out[i * 3 + 0] = u * ax + v * bx + w * cx + s * nx;
  out[i * 3 + 1] = u * ay + v * by + w * cy + s * ny;
  out[i * 3 + 2] = u * az + v * bz + w * cz + s * nz;
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

extern "C" {

int gmcp_dualmesh_embed(const double *P, int64_t N, const double *V, const int32_t *F, int64_t nT, int32_t *tri,
                        double *bary, double *delta, double *dist2, void *stream) {
  if (N < 0 || nT < 0) return GMCP_E_ARG;
  if (N == 0) return GMCP_OK;
  if (nT == 0 || !P || !V || !F || !tri || !bary || !delta) return GMCP_E_ARG;
  hipLaunchKernelGGL(k_embed, dim3(nblocks(N, kEmbedThreads)), dim3(kEmbedThreads), 0, (hipStream_t)stream, P, N, V,
                     F, nT, tri, bary, delta, dist2);
  return hipGetLastError() == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

int gmcp_dualmesh_update(const void *Vd, const int32_t *F, const int32_t *tri, const void *bary, const void *delta,
                         int64_t N, void *out, uint32_t flags, void *stream) {
  if (N < 0) return GMCP_E_ARG;
  if (N == 0) return GMCP_OK;
  if (!Vd || !F || !tri || !bary || !delta || !out) return GMCP_E_ARG;
  if (flags & GMCP_F64)
    hipLaunchKernelGGL(k_update<double>, dim3(nblocks(N, 256)), dim3(256), 0, (hipStream_t)stream,
                       (const double *)Vd, F, tri, (const double *)bary, (const double *)delta, N, (double *)out);
  else
    hipLaunchKernelGGL(k_update<float>, dim3(nblocks(N, 256)), dim3(256), 0, (hipStream_t)stream, (const float *)Vd,
                       F, tri, (const float *)bary, (const float *)delta, N, (float *)out);
  return hipGetLastError() == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

}  // extern "C"
