// Step bound for a search direction dx:
//   linearised gap, Eqs. (ccd) and (global_ccd), over the selected samples
//   of the last assembly, and additive CCD (Li, Kaufman, Jiang 2021) over
//   swept (sample point, master triangle) pairs found with a grid over the
//   master triangles' swept boxes.
// Both reduce with a float atomic-min on the bit pattern of positive floats
// (order-independent, hence deterministic).  Positions in the CCD are taken
// relative to the sample point's start, so float32 keeps small distances.
#include "common.h"

namespace gmcp {

namespace {

constexpr int kThreads = 256;
constexpr int kAccdMaxIter = 1 << 14;

template <typename R> __device__ inline float to_float_down(R v);
template <> __device__ inline float to_float_down<float>(float v) { return v; }
template <> __device__ inline float to_float_down<double>(double v) { return __double2float_rd(v); }

// Per-environment minimum of a >= 0 (uint order of non-negative floats is
// float order).  Waves reduce by shuffles; a block whose waves all hold one
// environment issues a single atomic.  Optionally the waves' counts (wcount,
// held by lane 0) are summed into *count with one atomic per block.  Every
// thread of the block must call.
__device__ inline void env_min(uint32_t *bits, int env, float a, int lane, unsigned long long wcount = 0,
                               unsigned long long *count = nullptr) {
  __shared__ int wenv[kThreads / kWave];
  __shared__ float wmin[kThreads / kWave];
  __shared__ unsigned long long wcnt[kThreads / kWave];
  const int w = threadIdx.x / kWave;
  uint64_t vm = __ballot(env >= 0);
  int e0 = vm ? __shfl(env, __ffsll((unsigned long long)vm) - 1, kWave) : -1;
  bool uniform = __all(env < 0 || env == e0);
  float m = (env >= 0 && uniform) ? a : INFINITY;
  for (int o = 32; o > 0; o >>= 1) m = fminf(m, __shfl_xor(m, o, kWave));
  if (!uniform && env >= 0 && a < INFINITY) atomicMin(&bits[env], __float_as_uint(a));
  if (lane == 0) {
    wenv[w] = uniform ? e0 : -1;
    wmin[w] = m;
    wcnt[w] = wcount;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int nw = blockDim.x / kWave;
  if (count) {
    unsigned long long c = 0;
    for (int v = 0; v < nw; ++v) c += wcnt[v];
    if (c) atomicAdd(count, c);
  }
  for (int v = 0; v < nw; ++v) {
    if (wenv[v] < 0) continue;
    float mm = wmin[v];
    for (int u = v + 1; u < nw; ++u)
      if (wenv[u] == wenv[v]) {
        mm = fminf(mm, wmin[u]);
        wenv[u] = -1;
      }
    if (mm < INFINITY) atomicMin(&bits[wenv[v]], __float_as_uint(mm));
  }
}

// Eq. (ccd): alpha_k = 0.9 g_k / (-grad g_k . dx) for grad g_k . dx < 0.
// One wave per work tile (the narrow phase's Morton tiles) with selected
// samples - the tiles the narrow phase listed, or every tile (list ==
// nullptr, clipped samples): lane (j, r0) takes records r0, r0 + nq, ... of
// the tile's triangle j (contiguous per triangle), so the triangle's normal
// and slave displacements are shared loads and the wave belongs to one
// environment (one atomic per tile).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_ccd_linear(const Rec<R> *__restrict__ rec, const DevStatus *st,
                                                          int64_t cap_active, const Tile *__restrict__ tiles,
                                                          int n_tiles, const int32_t *__restrict__ list,
                                                          const int32_t *__restrict__ count,
                                                          const int32_t *__restrict__ s_order,
                                                          const int32_t *__restrict__ tri_roff,
                                                          const int32_t *__restrict__ tri_rcnt,
                                                          const R *__restrict__ tri_nrm,
                                                          const int32_t *__restrict__ ts,
                                                          const int32_t *__restrict__ tm,
                                                          const EnvInfo *__restrict__ env,
                                                          const double *__restrict__ rule, const R *__restrict__ dxs,
                                                          const R *__restrict__ dxm, uint32_t *bits) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nlist = (int64_t)st->n_active > cap_active ? 0 : (list ? *count : n_tiles);
  // the wave's running minimum of environment ew (flushed when the
  // environment changes; the last one goes through the block reduction)
  int ew = -1;
  float aw = INFINITY;
  for (int64_t li = (int64_t)blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave; li < nlist;
       li += (int64_t)gridDim.x * (kThreads / kWave)) {
    const int tile_id = list ? list[li] : (int)li;
    float a = INFINITY;
    const Tile tl = tiles[tile_id];
    const int e = tl.env;
    if (e != ew) {
      for (int o = 32; o > 0; o >>= 1) aw = fminf(aw, __shfl_xor(aw, o, kWave));
      if (lane == 0 && ew >= 0 && aw < INFINITY) atomicMin(&bits[ew], __float_as_uint(aw));
      ew = e;
      aw = INFINITY;
    }
    const int j = lane / tl.nq, r0 = lane - j * tl.nq;
    if (j < tl.count) {
      const int T = s_order[tl.first + j];
      // a triangle's records: nq of them with whole-triangle samples, any
      // number with clipped mortar samples
      const int rcnt = tri_rcnt[T], roff = tri_roff[T];
      for (int r = r0; r < rcnt; r += tl.nq) {
        const Rec<R> rc = rec[roff + r];
        const R *n = tri_nrm + 3 * (int64_t)T;
        const R bs[3] = {R(1) - rc.s1 - rc.s2, rc.s1, rc.s2};
        const R bm[3] = {rc.b0, rc.b1, rc.b2};
        R gd = 0;
        for (int k = 0; k < 3; ++k) {
          const R *d = dxs + 3 * (int64_t)ts[3 * (int64_t)T + k];
          gd -= bs[k] * (n[0] * d[0] + n[1] * d[1] + n[2] * d[2]);
        }
        if (dxm)
          for (int m = 0; m < 3; ++m) {
            const R *d = dxm + 3 * (int64_t)tm[3 * (int64_t)rc.M + m];
            gd += bm[m] * (n[0] * d[0] + n[1] * d[1] + n[2] * d[2]);
          }
        if (gd < R(0)) a = fminf(a, to_float_down<R>(R(0.9) * rc.g / (-gd)));
      }
    }
    aw = fminf(aw, a);
  }
  env_min(bits, ew, aw, lane);
}

// squared distance from the origin-relative point p to triangle (a, b, c):
// closest point by Voronoi regions of the vertices, edges and face (the
// published closest-point-on-triangle method: C. Ericson, Real-Time
// Collision Detection, Morgan Kaufmann 2005, Sec. 5.1.5)
template <typename R>
__device__ inline R pt_tri_dist2(const R p[3], const R a[3], const R b[3], const R c[3]) {
  R ab[3], ac[3], ap[3];
  for (int d = 0; d < 3; ++d) {
    ab[d] = b[d] - a[d];
    ac[d] = c[d] - a[d];
    ap[d] = p[d] - a[d];
  }
  auto dot = [](const R *x, const R *y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
  R q[3];
  R d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= R(0) && d2 <= R(0)) {
    for (int d = 0; d < 3; ++d) q[d] = a[d];
  } else {
    R bp[3];
    for (int d = 0; d < 3; ++d) bp[d] = p[d] - b[d];
    R d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= R(0) && d4 <= d3) {
      for (int d = 0; d < 3; ++d) q[d] = b[d];
    } else {
      R vc = d1 * d4 - d3 * d2;
      if (vc <= R(0) && d1 >= R(0) && d3 <= R(0)) {
        R v = d1 / (d1 - d3);
        for (int d = 0; d < 3; ++d) q[d] = a[d] + v * ab[d];
      } else {
        R cp[3];
        for (int d = 0; d < 3; ++d) cp[d] = p[d] - c[d];
        R d5 = dot(ab, cp), d6 = dot(ac, cp);
        if (d6 >= R(0) && d5 <= d6) {
          for (int d = 0; d < 3; ++d) q[d] = c[d];
        } else {
          R vb = d5 * d2 - d1 * d6;
          if (vb <= R(0) && d2 >= R(0) && d6 <= R(0)) {
            R w = d2 / (d2 - d6);
            for (int d = 0; d < 3; ++d) q[d] = a[d] + w * ac[d];
          } else {
            R va = d3 * d6 - d5 * d4;
            if (va <= R(0) && (d4 - d3) >= R(0) && (d5 - d6) >= R(0)) {
              R w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
              for (int d = 0; d < 3; ++d) q[d] = b[d] + w * (c[d] - b[d]);
            } else {
              R den = R(1) / (va + vb + vc);
              R v = vb * den, w = vc * den;
              for (int d = 0; d < 3; ++d) q[d] = a[d] + ab[d] * v + ac[d] * w;
            }
          }
        }
      }
    }
  }
  R r[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
  return dot(r, r);
}

// additive CCD, thickness 0, separation ratio s, horizon 1: the point starts
// at the origin (coordinates are relative to it)
template <typename R>
__device__ inline R accd(const R dp[3], const R a0[3], const R da[3], const R b0[3], const R db[3], const R c0[3],
                         const R dc[3], R s) {
  R mean[3], up[3], ua[3], ub[3], uc[3];
  for (int d = 0; d < 3; ++d) {
    mean[d] = R(0.25) * (dp[d] + da[d] + db[d] + dc[d]);
    up[d] = dp[d] - mean[d];
    ua[d] = da[d] - mean[d];
    ub[d] = db[d] - mean[d];
    uc[d] = dc[d] - mean[d];
  }
  auto nrm = [](const R *v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); };
  R l = nrm(up) + fmax(nrm(ua), fmax(nrm(ub), nrm(uc)));
  if (!(l > R(0))) return R(1);
  R p[3] = {0, 0, 0}, a[3], b[3], c[3];
  for (int d = 0; d < 3; ++d) {
    a[d] = a0[d];
    b[d] = b0[d];
    c[d] = c0[d];
  }
  R dist = sqrt(pt_tri_dist2(p, a, b, c));
  if (!(dist > R(0))) return R(0);
  R gmin = s * dist, t = 0, step = (R(1) - s) * dist / l;
  for (int it = 0; it < kAccdMaxIter; ++it) {
    for (int d = 0; d < 3; ++d) {
      p[d] += step * up[d];
      a[d] += step * ua[d];
      b[d] += step * ub[d];
      c[d] += step * uc[d];
    }
    dist = sqrt(pt_tri_dist2(p, a, b, c));
    if (t > R(0) && dist < gmin) break;
    t += step;
    if (t > R(1)) return R(1);
    step = R(0.9) * dist / l;
  }
  return t;
}

__device__ inline int cell_coord(const GridEnv &g, float x, int d) {
  float f = (x - g.lo[d]) * g.inv_h;
  int n = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
  int c = (int)floorf(f);
  return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// swept box of slave triangle T over dx (float, with a few ulps of slack):
// it covers the swept box of every sample point of T
__device__ inline void slack_box(float a, float b, float &lo, float &hi) {
  const float mn = fminf(a, b), mx = fmaxf(a, b);
  lo = mn - fabsf(mn) * 4e-7f - 1e-30f;
  hi = mx + fabsf(mx) * 4e-7f + 1e-30f;
}
template <typename R>
__device__ inline void swept_tri_box(const R *xs, const R *dxs, const int64_t v[3], float tlo[3], float thi[3]) {
  for (int d = 0; d < 3; ++d) {
    float lo = INFINITY, hi = -INFINITY;
    for (int k = 0; k < 3; ++k) {
      float l, h;
      slack_box((float)xs[3 * v[k] + d], (float)(xs[3 * v[k] + d] + dxs[3 * v[k] + d]), l, h);
      lo = fminf(lo, l);
      hi = fmaxf(hi, h);
    }
    tlo[d] = lo;
    thi[d] = hi;
  }
}

__device__ inline bool box_in_grid(const GridEnv &g, const float lo[3], const float hi[3]) {
  const float ext[3] = {g.nx * g.h, g.ny * g.h, g.nz * g.h};
  for (int d = 0; d < 3; ++d)
    if (hi[d] < g.lo[d] || lo[d] > g.lo[d] + ext[d]) return false;
  return true;
}

// Thread per slave triangle (Morton order): lists the work tiles with a
// triangle whose swept box meets an occupied cell of the swept grid.  Only
// they can have swept pairs (every sample point's swept box lies inside its
// triangle's), and they are usually few, so the CCD kernel walks this list
// instead of every tile.  A tile is listed once: its first triangle to
// claim the tile's flag appends it (the CCD kernel clears the flags of the
// tiles it walks).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_ccd_pre(const R *__restrict__ xs, const R *__restrict__ dxs,
                                                       const int32_t *__restrict__ ts,
                                                       const int32_t *__restrict__ s_order,
                                                       const int32_t *__restrict__ s_env,
                                                       const EnvInfo *__restrict__ env,
                                                       const GridEnv *__restrict__ grid, int64_t Ts,
                                                       const int32_t *__restrict__ cell_start, int64_t cap_items,
                                                       int64_t total_cells, int32_t *__restrict__ tflag,
                                                       int32_t *__restrict__ list, int32_t *__restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  bool active = false;
  int64_t t = -1;
  int tile = -1;
  if (i < Ts && cell_start[total_cells] <= cap_items) {
    t = s_order[i];
    const int e = s_env[t];
    const GridEnv g = grid[e];
    tile = env[e].tile0 + (int)((i - env[e].st0) / (kWave / env[e].nq));  // tiles cover the env's positions
    if (g.valid) {
      const int64_t v[3] = {ts[3 * t], ts[3 * t + 1], ts[3 * t + 2]};
      float lo[3], hi[3];
      swept_tri_box<R>(xs, dxs, v, lo, hi);
      if (box_in_grid(g, lo, hi)) {
        int c0[3], c1[3];
        for (int d = 0; d < 3; ++d) {
          c0[d] = cell_coord(g, lo[d], d);
          c1[d] = cell_coord(g, hi[d], d);
        }
        const int64_t ncell = (int64_t)(c1[0] - c0[0] + 1) * (c1[1] - c0[1] + 1) * (c1[2] - c0[2] + 1);
        if (ncell > 4096) {
          active = true;  // too many cells to check here: the CCD kernel decides
        } else {
          const int64_t base = env[e].cell0;
          // the (y, z) rows of the box, 8 at a time (their loads in flight
          // together); a row's x-run of cells is contiguous
          const int ny = c1[1] - c0[1] + 1, nrow = ny * (c1[2] - c0[2] + 1);
          int ry = 0, rz = 0;  // row r0 + k as (y, z) offsets, stepped (no divisions)
          for (int r0 = 0; r0 < nrow && !active; r0 += 8) {
            int32_t hi_s[8], lo_s[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const int r = r0 + k;
              hi_s[k] = lo_s[k] = 0;
              const int64_t row = base + ((int64_t)(c0[2] + rz) * g.ny + c0[1] + ry) * g.nx;
              if (++ry == ny) {
                ry = 0;
                ++rz;
              }
              if (r < nrow) {
                hi_s[k] = cell_start[row + c1[0] + 1];
                lo_s[k] = cell_start[row + c0[0]];
              }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) active = active || hi_s[k] > lo_s[k];
          }
        }
      }
    }
  }
  // the tile's first claim appends it: wave ballots, block prefix in LDS,
  // one atomic per block
  if (active) active = atomicExch(&tflag[tile], 1) == 0;
  __shared__ int wq[kThreads / kWave], qb;
  const int w = threadIdx.x / kWave;
  const uint64_t m = __ballot(active);
  if (lane == 0) wq[w] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int sum = 0;
    for (int k = 0; k < kThreads / kWave; ++k) {
      const int c0 = wq[k];
      wq[k] = sum;
      sum += c0;
    }
    qb = sum ? atomicAdd(count, sum) : 0;
  }
  __syncthreads();
  if (active) list[qb + wq[w] + __popcll(m & ((1ull << lane) - 1))] = tile;
}


// One wave per listed work tile (k_ccd_pre), lane = (slave triangle j, rule
// point q) as in the narrow phase.  The lanes of a triangle first gather,
// from the grid cells its swept box covers, the master triangles whose
// swept boxes overlap it (each once: the cell holding the lower corner of
// the overlap), into an LDS slice; then every lane tests its own point's
// swept box against that list, and the overlaps go through a per-wave queue
// that runs additive CCD on 64 pairs at a time.  A triangle whose list
// overflows its slice walks the cells point by point instead.
constexpr int kAccdPool = 1024;  // LDS list entries per wave, split over the tile's triangles

template <typename R>
__global__ __launch_bounds__(kThreads) void k_ccd_accd(
    const R *__restrict__ xs, const R *__restrict__ xm, const R *__restrict__ dxs, const R *__restrict__ dxm,
    const int32_t *__restrict__ ts, const int32_t *__restrict__ tm, const Tile *__restrict__ tiles,
    const int32_t *__restrict__ list, const int32_t *__restrict__ count, int32_t *__restrict__ tflag,
    const int32_t *__restrict__ s_order, const EnvInfo *__restrict__ env, const double *__restrict__ rule,
    const GridEnv *__restrict__ grid, const int32_t *__restrict__ cell_start, const int32_t *__restrict__ items,
    const float4 *__restrict__ smbox, int64_t cap_items, int64_t total_cells, uint32_t *bits, DevStatus *st) {
  __shared__ int32_t plist[kThreads / kWave][kAccdPool];
  __shared__ int32_t pcnt[kThreads / kWave][kWave];
  __shared__ int32_t qpt[kThreads / kWave][2 * kWave], qm[kThreads / kWave][2 * kWave];  // pair queue
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const bool grid_ok = cell_start[total_cells] <= cap_items;
  const int64_t nlist = *count;
  // the wave's running minimum of environment ew (flushed when the
  // environment changes; the last one goes through the block reduction)
  // and its pair count
  int ew = -1;
  float aw = INFINITY;
  unsigned long long npairs = 0;
  // the waves walk the listed tiles (k_ccd_pre); each tile's flag is
  // cleared once it is done, ready for the next call
  for (int64_t li = (int64_t)blockIdx.x * (kThreads / kWave) + w; li < nlist;
       li += (int64_t)gridDim.x * (kThreads / kWave)) {
    const int tile_id = list[li];
    if (!grid_ok) {  // nothing to test against: only the flag
      if (lane == 0) tflag[tile_id] = 0;
      continue;
    }
    wave_sync();  // the previous tile's LDS reads are done
    float amin = INFINITY;
    const Tile tl = tiles[tile_id];
    const int e = tl.env;
    if (e != ew) {
      for (int o = 32; o > 0; o >>= 1) aw = fminf(aw, __shfl_xor(aw, o, kWave));
      if (lane == 0 && ew >= 0 && aw < INFINITY) atomicMin(&bits[ew], __float_as_uint(aw));
      ew = e;
      aw = INFINITY;
    }
    const int j = lane / tl.nq, q = lane - j * tl.nq;
    const bool live = j < tl.count;
    const int64_t T = live ? s_order[tl.first + j] : 0;
    const EnvInfo &ev = env[e];
    const GridEnv g = grid[e];
    const int slice = kAccdPool / (tl.count > 0 ? tl.count : 1);
    const int64_t base = ev.cell0;
    const float ext[3] = {g.nx * g.h, g.ny * g.h, g.nz * g.h};
    auto inside_grid = [&](const float lo[3], const float hi[3]) {
      for (int d = 0; d < 3; ++d)
        if (hi[d] < g.lo[d] || lo[d] > g.lo[d] + ext[d]) return false;
      return true;
    };
    int64_t v[3] = {0, 0, 0};
    float tlo[3], thi[3];
    if (live) {
      for (int k = 0; k < 3; ++k) v[k] = ts[3 * T + k];
      swept_tri_box<R>(xs, dxs, v, tlo, thi);  // covers every point's swept box
    }
    // ---- gather the triangle's swept candidates into its LDS slice
    if (live && q == 0) pcnt[w][j] = 0;
    wave_sync();
    if (live && g.valid && inside_grid(tlo, thi)) {
      int c0[3], c1[3];
      for (int d = 0; d < 3; ++d) {
        c0[d] = cell_coord(g, tlo[d], d);
        c1[d] = cell_coord(g, thi[d], d);
      }
      for (int z = c0[2]; z <= c1[2]; ++z)
        for (int y = c0[1]; y <= c1[1]; ++y)
          for (int x = c0[0]; x <= c1[0]; ++x) {
            const int64_t cell = base + ((int64_t)z * g.ny + y) * g.nx + x;
            const int i1 = cell_start[cell + 1];
            for (int i = cell_start[cell] + q; i < i1; i += tl.nq) {
              const int M = items[i];
              const float4 ma = smbox[3 * (int64_t)M], mb = smbox[3 * (int64_t)M + 1];
              if (ma.x > thi[0] || mb.x < tlo[0] || ma.y > thi[1] || mb.y < tlo[1] || ma.z > thi[2] ||
                  mb.z < tlo[2])
                continue;
              if (cell_coord(g, fmaxf(ma.x, tlo[0]), 0) != x || cell_coord(g, fmaxf(ma.y, tlo[1]), 1) != y ||
                  cell_coord(g, fmaxf(ma.z, tlo[2]), 2) != z)
                continue;
              const int slot = atomicAdd(&pcnt[w][j], 1);
              if (slot < slice) plist[w][j * slice + slot] = M;
            }
          }
    }
    wave_sync();
    // the point's start (relative frame) and displacement, and its swept box
    const bool pt_ok = live && g.valid;
    R s0[3] = {0, 0, 0}, dp[3] = {0, 0, 0}, off[3] = {0, 0, 0};
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    if (pt_ok) {
      const double *rq = rule + ((ev.rule_n - 1) * 16 + q) * 3;
      const R bs[3] = {R(1) - (R)rq[0] - (R)rq[1], (R)rq[0], (R)rq[1]};
      for (int d = 0; d < 3; ++d) {
        s0[d] = xs[3 * v[0] + d];
        off[d] = bs[1] * (xs[3 * v[1] + d] - s0[d]) + bs[2] * (xs[3 * v[2] + d] - s0[d]);
        dp[d] = bs[0] * dxs[3 * v[0] + d] + bs[1] * dxs[3 * v[1] + d] + bs[2] * dxs[3 * v[2] + d];
      }
      for (int d = 0; d < 3; ++d) {
        const R p0 = s0[d] + off[d];
        slack_box((float)p0, (float)(p0 + dp[d]), lo[d], hi[d]);
      }
    }
    auto boxes_meet = [&](int M) {
      const float4 ma = smbox[3 * (int64_t)M], mb = smbox[3 * (int64_t)M + 1];
      return !(ma.x > hi[0] || mb.x < lo[0] || ma.y > hi[1] || mb.y < lo[1] || ma.z > hi[2] || mb.z < lo[2]);
    };
    // additive CCD of a point (given by its frame) against master triangle M
    auto run = [&](int M, const R ps0[3], const R poff[3], const R pdp[3]) {
      R A[3], B[3], C[3], dA[3], dB[3], dC[3];
      const int64_t w0 = tm[3 * (int64_t)M], w1 = tm[3 * (int64_t)M + 1], w2 = tm[3 * (int64_t)M + 2];
      for (int d = 0; d < 3; ++d) {
        A[d] = (xm[3 * w0 + d] - ps0[d]) - poff[d];
        B[d] = (xm[3 * w1 + d] - ps0[d]) - poff[d];
        C[d] = (xm[3 * w2 + d] - ps0[d]) - poff[d];
        dA[d] = dxm ? dxm[3 * w0 + d] : R(0);
        dB[d] = dxm ? dxm[3 * w1 + d] : R(0);
        dC[d] = dxm ? dxm[3 * w2 + d] : R(0);
      }
      amin = fminf(amin, to_float_down<R>(accd<R>(pdp, A, dA, B, dB, C, dC, R(0.1))));
    };
    // The wave's (point, master triangle) overlaps from the LDS lists are
    // queued in LDS and run 64 at a time, one pair per lane, so a point with
    // many overlaps does not hold the rest of the wave; each lane fetches the
    // queued point's frame from the point's lane by shuffles.  The minimum
    // does not depend on which lane runs a pair.
    const int n = pt_ok ? pcnt[w][j] : 0;
    const bool walk = n > slice;  // list overflowed: this point walks its own cells below
    const int nl = walk ? 0 : n;
    int maxn = nl;
    for (int o = 32; o > 0; o >>= 1) maxn = max(maxn, __shfl_xor(maxn, o, kWave));
    auto drain = [&](int first, int count) {  // every lane calls (the shuffles)
      const bool act = lane < count;
      const int p = act ? qpt[w][first + lane] : lane;
      const int M = act ? qm[w][first + lane] : 0;
      R ps0[3], poff[3], pdp[3];
      for (int d = 0; d < 3; ++d) {
        ps0[d] = __shfl(s0[d], p, kWave);
        poff[d] = __shfl(off[d], p, kWave);
        pdp[d] = __shfl(dp[d], p, kWave);
      }
      if (act) run(M, ps0, poff, pdp);
    };
    const uint64_t one = 1;
    int qn = 0;  // queued pairs (wave-uniform), < kWave between rounds
    for (int r = 0; r < maxn; ++r) {
      int M = 0;
      bool hit = false;
      if (r < nl) {
        M = plist[w][j * slice + r];
        hit = boxes_meet(M);
      }
      const uint64_t hm = __ballot(hit);
      if (hit) {
        const int pos = qn + __popcll(hm & ((one << lane) - 1));
        qpt[w][pos] = lane;
        qm[w][pos] = M;
        ++npairs;
      }
      qn += __popcll(hm);
      if (qn >= kWave) {
        wave_sync();
        qn -= kWave;
        drain(qn, kWave);
        wave_sync();  // the drained entries are read before the next round overwrites them
      }
    }
    wave_sync();
    if (qn > 0) drain(0, qn);
    if (walk && inside_grid(lo, hi)) {  // overflow: walk the point's own cells
      int c0[3], c1[3];
      for (int d = 0; d < 3; ++d) {
        c0[d] = cell_coord(g, lo[d], d);
        c1[d] = cell_coord(g, hi[d], d);
      }
      for (int z = c0[2]; z <= c1[2]; ++z)
        for (int y = c0[1]; y <= c1[1]; ++y)
          for (int x = c0[0]; x <= c1[0]; ++x) {
            const int64_t cell = base + ((int64_t)z * g.ny + y) * g.nx + x;
            for (int i = cell_start[cell]; i < cell_start[cell + 1]; ++i) {
              const int M = items[i];
              const float4 ma = smbox[3 * (int64_t)M];
              if (cell_coord(g, fmaxf(ma.x, lo[0]), 0) != x || cell_coord(g, fmaxf(ma.y, lo[1]), 1) != y ||
                  cell_coord(g, fmaxf(ma.z, lo[2]), 2) != z)
                continue;
              if (!boxes_meet(M)) continue;
              ++npairs;
              run(M, s0, off, dp);
            }
          }
    }
    aw = fminf(aw, amin);
    if (lane == 0) tflag[tile_id] = 0;
  }
  // pair count: wave sums, one atomic per block (with the minimum)
  unsigned long long tot = npairs;
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, kWave);
  env_min(bits, ew, aw, lane, tot, &st->n_swept);
}

template <typename R>
__global__ void k_alpha_final(const uint32_t *bits, int n_env, R *alpha) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_env) return;
  float a = __uint_as_float(bits[e]);
  // shrink the float bound so it never exceeds the exact one
  float r = a < 1.0f ? a * (1.0f - 1.0f / 8192.0f) : 1.0f;
  alpha[e] = (R)r;
}


}  // namespace

template <typename R>
hipError_t launch_ccd_swept(gmcp_ctx *c, const R *xs, const R *xm, const R *dxs, const R *dxm) {
  Buffers &b = c->b;
  hipStream_t s = c->stream;
  StageInit si;
  si.which = 4;
  si.box = b.sbox;
  si.alpha = b.alpha_bits;
  si.zero[0] = b.scount;
  si.nzero[0] = 1;
  hipError_t e = stage_init(c, si);
  if (e != hipSuccess) return e;
  prof_mark(c, ST_CCD_GRID, 0);
  e = build_grid<R>(c, xs, xm, dxs, dxm, true);
  prof_mark(c, ST_CCD_GRID, 1);
  if (e != hipSuccess) return e;
  prof_mark(c, ST_CCD_ACCD, 0);
  // the tile-list walk uses a fixed grid (the list is usually short; its
  // length is known on the device only)
  const unsigned accd_blocks = (unsigned)std::max<int64_t>(
      1, std::min<int64_t>((c->n_tiles + kThreads / kWave - 1) / (kThreads / kWave), 2048));
  if (c->n_tiles) {
    hipLaunchKernelGGL(k_ccd_pre<R>, dim3((unsigned)((c->Ts + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, xs,
                       dxs, c->ts, b.s_order, b.s_env, b.env, b.sgrid, c->Ts, b.scell_start, c->caps.grid_items,
                       c->total_cells, b.tflag, b.slist, b.scount);
    hipLaunchKernelGGL(k_ccd_accd<R>, dim3(accd_blocks), dim3(kThreads), 0, s, xs, xm, dxs, dxm, c->ts, c->tm,
                       b.tiles, b.slist, b.scount, b.tflag, b.s_order, b.env, b.rule, b.sgrid, b.scell_start,
                       b.sitems, b.smbox, c->caps.grid_items, c->total_cells, b.alpha_bits, b.status);
  }
  prof_mark(c, ST_CCD_ACCD, 1);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_ccd_finish(gmcp_ctx *c, const R *dxs, const R *dxm, R *alpha) {
  Buffers &b = c->b;
  hipStream_t s = c->stream;
  prof_mark(c, ST_CCD_LINEAR, 0);
  // a fixed grid walks the tiles with selected samples (their number is
  // known on the device only); clipped samples: every tile
  const unsigned lin_blocks = (unsigned)std::max<int64_t>(
      1, std::min<int64_t>((c->n_tiles + kThreads / kWave - 1) / (kThreads / kWave), 4096));
  if (c->n_tiles)
    hipLaunchKernelGGL(k_ccd_linear<R>, dim3(lin_blocks), dim3(kThreads), 0, s, (const Rec<R> *)b.rec, b.status,
                       c->caps.active, b.tiles, (int)c->n_tiles, c->mortar ? nullptr : b.atile, b.atile_cnt, b.s_order,
                       b.tri_roff, b.tri_rcnt, (const R *)b.tri_nrm, c->ts, c->tm, b.env, b.rule, dxs, dxm,
                       b.alpha_bits);
  prof_mark(c, ST_CCD_LINEAR, 1);
  hipLaunchKernelGGL(k_alpha_final<R>, dim3((c->n_env + 63) / 64), dim3(64), 0, s, b.alpha_bits, c->n_env, alpha);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_ccd(gmcp_ctx *c, const R *xs, const R *xm, const R *dxs, const R *dxm, R *alpha) {
  hipError_t e = launch_ccd_swept<R>(c, xs, xm, dxs, dxm);
  if (e != hipSuccess) return e;
  return launch_ccd_finish<R>(c, dxs, dxm, alpha);
}

template hipError_t launch_ccd<float>(gmcp_ctx *, const float *, const float *, const float *, const float *,
                                      float *);
template hipError_t launch_ccd<double>(gmcp_ctx *, const double *, const double *, const double *, const double *,
                                       double *);
template hipError_t launch_ccd_swept<float>(gmcp_ctx *, const float *, const float *, const float *, const float *);
template hipError_t launch_ccd_swept<double>(gmcp_ctx *, const double *, const double *, const double *,
                                             const double *);
template hipError_t launch_ccd_finish<float>(gmcp_ctx *, const float *, const float *, float *);
template hipError_t launch_ccd_finish<double>(gmcp_ctx *, const double *, const double *, double *);

}  // namespace gmcp
