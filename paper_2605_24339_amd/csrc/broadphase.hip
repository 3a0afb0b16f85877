// Broad phase: per-environment uniform grid over the master triangles,
// queried with the support prism of every slave triangle.
//
// Grid domain of an environment: the slave surface's box grown by eps_max
// (a master triangle outside it cannot be reached by any sample's support
// segment).  Cells are numbered x-fastest inside the environment's slice of
// the cell array.  Every master triangle is counted into each cell its box
// touches (atomic counts), the counts are scanned into cell starts, and a
// second pass places the triangle ids (the counters return to zero, ready
// for the next call).  The support prism of a slave triangle is covered by
// thin slabs along its normal, whose boxes are far tighter than the box of
// the whole (slanted) prism; candidates found in several cells or slabs are
// merged in an LDS hash set and each list is written sorted, so candidate
// lists are deterministic.
#include "common.h"

namespace gmcp {

namespace {

constexpr int kThreads = 256;

template <typename R>
__device__ inline void load3(const R *x, int64_t v, float o[3]) {
  o[0] = (float)x[3 * v];
  o[1] = (float)x[3 * v + 1];
  o[2] = (float)x[3 * v + 2];
}

// outward rounding margin for float boxes of (possibly double) coordinates
__device__ inline float grow(float v) { return fabsf(v) * 4e-7f + 1e-30f; }

// slave surface box per environment (swept: union of x and x + dx): thread
// per slave vertex on a slave triangle (the union of the triangles' vertex
// boxes, read coalesced); large blocks, so that few blocks meet at each
// environment's six words
constexpr int kBoxThreads = 1024;

template <typename R>
__global__ __launch_bounds__(kBoxThreads) void k_slave_box(const R *__restrict__ xs, const R *__restrict__ dxs,
                                                         const int32_t *__restrict__ s_venv, int64_t Vs,
                                                         uint32_t *box, int32_t *zero_a, int32_t *zero_b,
                                                         uint32_t *epoch) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0) {  // counters of the kernels that follow (nullable), and the broad phase's epoch
    if (zero_a) *zero_a = 0;
    if (zero_b) *zero_b = 0;
    if (epoch) *epoch += 1u;
  }
  int lane = threadIdx.x & (kWave - 1);
  int env = v < Vs ? s_venv[v] : -1;
  bool ok = env >= 0;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (ok) {
    float p[3];
    load3(xs, v, p);
    for (int d = 0; d < 3; ++d) {  // fminf / fmaxf: a NaN coordinate leaves the box as it is
      lo[d] = fminf(lo[d], p[d] - grow(p[d]));
      hi[d] = fmaxf(hi[d], p[d] + grow(p[d]));
    }
    if (dxs) {
      for (int d = 0; d < 3; ++d) {
        float q = (float)(xs[3 * v + d] + dxs[3 * v + d]);
        lo[d] = fminf(lo[d], q - grow(q));
        hi[d] = fmaxf(hi[d], q + grow(q));
      }
    }
  }
  // environments are contiguous in vertex order: most blocks hold one,
  // which then takes a single set of atomics
  __shared__ int benv[kBoxThreads / kWave];
  __shared__ float bbox[kBoxThreads / kWave][6];
  const int w = threadIdx.x / kWave;
  uint64_t vm = __ballot(ok);
  int e0 = vm ? __shfl(env, __ffsll((unsigned long long)vm) - 1, kWave) : -1;
  bool uniform = __all(!ok || env == e0);
  if (uniform) {
    for (int d = 0; d < 3; ++d) {
      float a = lo[d], b = hi[d];
      for (int o = 32; o > 0; o >>= 1) {
        a = fminf(a, __shfl_xor(a, o, kWave));
        b = fmaxf(b, __shfl_xor(b, o, kWave));
      }
      lo[d] = a;
      hi[d] = b;
    }
  } else if (ok) {
    for (int d = 0; d < 3; ++d) {
      atomicMin(&box[6 * env + d], float_to_ordered(lo[d]));
      atomicMax(&box[6 * env + 3 + d], float_to_ordered(hi[d]));
    }
  }
  if (lane == 0) {
    benv[w] = uniform ? e0 : -2;  // -1: no triangle, -2: already flushed
    for (int d = 0; d < 3; ++d) {
      bbox[w][d] = lo[d];
      bbox[w][3 + d] = hi[d];
    }
  }
  __syncthreads();
  const int nw = blockDim.x / kWave;
  bool same = true;
  for (int v = 0; v < nw; ++v)
    if (benv[v] != -1 && benv[v] != benv[0]) same = false;
  if (same) {  // one environment (the common case): six threads, one component each
    const int d = threadIdx.x;
    if (d >= 6 || benv[0] < 0) return;
    float a = bbox[0][d];
    for (int v = 1; v < nw; ++v)
      if (benv[v] >= 0) a = d < 3 ? fminf(a, bbox[v][d]) : fmaxf(a, bbox[v][d]);
    if (d < 3) atomicMin(&box[6 * benv[0] + d], float_to_ordered(a));
    else atomicMax(&box[6 * benv[0] + d], float_to_ordered(a));
    return;
  }
  if (threadIdx.x != 0) return;  // several environments: each uniform wave's box on its own
  for (int v = 0; v < nw; ++v) {
    if (benv[v] < 0) continue;
    for (int d = 0; d < 3; ++d) {
      atomicMin(&box[6 * benv[v] + d], float_to_ordered(bbox[v][d]));
      atomicMax(&box[6 * benv[v] + 3 + d], float_to_ordered(bbox[v][3 + d]));
    }
  }
}

// grid geometry of environment e: domain = box grown by `pad`, cell size
// from the caller (cell > 0) or max(eps_max / 4, cbrt(volume / budget)),
// enlarged until the cell count fits the environment's budget
__device__ inline GridEnv grid_of(const EnvInfo &v, const uint32_t *__restrict__ box, int e, int swept) {
  GridEnv g;
  float lo[3], hi[3];
  bool empty = false;
  float pad = swept ? 0.0f : (float)v.dhat * 1.0001f;
  for (int d = 0; d < 3; ++d) {
    lo[d] = ordered_to_float(box[6 * e + d]);
    hi[d] = ordered_to_float(box[6 * e + 3 + d]);
    if (!(lo[d] <= hi[d])) empty = true;
    lo[d] -= pad;
    hi[d] += pad;
  }
  if (empty || v.cell_budget <= 0 || v.st1 == v.st0) {
    g.valid = 0;
    g.nx = g.ny = g.nz = 1;
    g.h = 1.0f;
    g.inv_h = 1.0f;
    for (int d = 0; d < 3; ++d) g.lo[d] = 0.0f;
    return g;
  }
  double ext[3] = {hi[0] - (double)lo[0], hi[1] - (double)lo[1], hi[2] - (double)lo[2]};
  double span = fmax(ext[0], fmax(ext[1], ext[2]));
  double vol = fmax(ext[0], span * 1e-3) * fmax(ext[1], span * 1e-3) * fmax(ext[2], span * 1e-3);
  double h = v.cell > 0.0 ? v.cell : fmax(v.dhat * 0.25, cbrt(vol / (double)v.cell_budget));
  if (!(h > span * 1e-6)) h = span * 1e-6 + 1e-30;
  int64_t n[3], tot = 1;
  for (int it = 0; it < 200; ++it) {
    tot = 1;
    for (int d = 0; d < 3; ++d) {
      n[d] = (int64_t)(ext[d] / h) + 1;
      tot *= n[d];
    }
    if (tot <= v.cell_budget) break;
    h *= 1.05 * cbrt((double)tot / (double)v.cell_budget);
  }
  g.valid = tot <= v.cell_budget && n[0] < (1 << 30) && n[1] < (1 << 30) && n[2] < (1 << 30);
  g.h = (float)h;
  g.inv_h = (float)(1.0 / h);
  g.nx = (int)n[0];
  g.ny = (int)n[1];
  g.nz = (int)n[2];
  for (int d = 0; d < 3; ++d) g.lo[d] = lo[d];
  return g;
}

__device__ inline int cell_coord(const GridEnv &g, float x, int d) {
  float f = (x - g.lo[d]) * g.inv_h;
  int n = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
  int c = (int)floorf(f);
  return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

__device__ inline bool box_hits_grid(const GridEnv &g, const float lo[3], const float hi[3]) {
  float ext[3] = {g.nx * g.h, g.ny * g.h, g.nz * g.h};
  for (int d = 0; d < 3; ++d)
    if (hi[d] < g.lo[d] || lo[d] > g.lo[d] + ext[d]) return false;
  return true;
}

// Thread per master triangle (and per environment): the environments'
// grids from their slave boxes (thread e writes grid[e]; every triangle's
// thread derives its own environment's grid, so no separate launch is
// needed), master triangle boxes (and unit normals), static or swept over
// dx, and the count of the grid cells each box covers (placement:
// k_grid_insert)
template <typename R>
__global__ __launch_bounds__(kThreads) void k_master_boxes(const R *__restrict__ xm, const R *__restrict__ dxm,
                                                            const int32_t *__restrict__ tm, int64_t Tm,
                                                            float4 *__restrict__ mbox,
                                                            const int32_t *__restrict__ m_env,
                                                            const EnvInfo *__restrict__ env,
                                                            const uint32_t *__restrict__ box, GridEnv *grid,
                                                            int n_env, int swept, int32_t *__restrict__ cell_cnt) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_env) grid[t] = grid_of(env[t], box, (int)t, swept);
  if (t >= Tm) return;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  R p[3][3];
  for (int j = 0; j < 3; ++j) {
    int64_t v = tm[3 * t + j];
    for (int d = 0; d < 3; ++d) {
      p[j][d] = xm[3 * v + d];
      float f = (float)p[j][d];
      lo[d] = fminf(lo[d], f - grow(f));
      hi[d] = fmaxf(hi[d], f + grow(f));
      if (dxm) {
        float q = (float)(p[j][d] + dxm[3 * v + d]);
        lo[d] = fminf(lo[d], q - grow(q));
        hi[d] = fmaxf(hi[d], q + grow(q));
      }
    }
  }
  R f1[3], f2[3];
  for (int d = 0; d < 3; ++d) {
    f1[d] = p[1][d] - p[0][d];
    f2[d] = p[2][d] - p[0][d];
  }
  R N[3] = {f1[1] * f2[2] - f1[2] * f2[1], f1[2] * f2[0] - f1[0] * f2[2], f1[0] * f2[1] - f1[1] * f2[0]};
  R len = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
  R inv = len > R(0) ? R(1) / len : R(0);
  mbox[3 * t + 0] = make_float4(lo[0], lo[1], lo[2], 0.0f);
  mbox[3 * t + 1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
  mbox[3 * t + 2] = make_float4((float)(N[0] * inv), (float)(N[1] * inv), (float)(N[2] * inv), 0.0f);
  const int e = m_env[t];
  const GridEnv g = grid_of(env[e], box, e, swept);
  if (!g.valid || !box_hits_grid(g, lo, hi)) return;
  int c0[3], c1[3];
  for (int d = 0; d < 3; ++d) {
    c0[d] = cell_coord(g, lo[d], d);
    c1[d] = cell_coord(g, hi[d], d);
  }
  const int64_t base = env[e].cell0;
  for (int z = c0[2]; z <= c1[2]; ++z)
    for (int y = c0[1]; y <= c1[1]; ++y)
      for (int x = c0[0]; x <= c1[0]; ++x) atomicAdd(&cell_cnt[base + ((int64_t)z * g.ny + y) * g.nx + x], 1);
}

// place the master ids in their cells after the count and its scan (the
// counters return to zero); same cell ranges as the count
__global__ __launch_bounds__(kThreads) void k_grid_insert(const float4 *__restrict__ mbox,
                                                           const int32_t *__restrict__ m_env,
                                                           const EnvInfo *__restrict__ env,
                                                           const GridEnv *__restrict__ grid, int64_t Tm,
                                                           int32_t *__restrict__ cell_cnt,
                                                           const int32_t *__restrict__ cell_start,
                                                           int32_t *__restrict__ items, int64_t cap_items,
                                                           int64_t total_cells, DevStatus *st) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Tm) return;
  // the overflow is reported by thread 0 whatever its own triangle does
  const int64_t total = cell_start[total_cells];
  const bool fits = total <= cap_items;
  if (!fits && t == 0) {
    atomicMax(&st->need_items, (unsigned long long)total);
    atomicCAS(&st->code, 0, GMCP_E_CAPACITY);
  }
  int e = m_env[t];
  GridEnv g = grid[e];
  if (!g.valid) return;
  float4 a = mbox[3 * t], b = mbox[3 * t + 1];
  float lo[3] = {a.x, a.y, a.z}, hi[3] = {b.x, b.y, b.z};
  if (!box_hits_grid(g, lo, hi)) return;
  int c0[3], c1[3];
  for (int d = 0; d < 3; ++d) {
    c0[d] = cell_coord(g, lo[d], d);
    c1[d] = cell_coord(g, hi[d], d);
  }
  const int64_t base = env[e].cell0;
  // the box's cells four at a time: their atomics in flight together (the
  // cell coordinates stepped x-fastest, no divisions)
  const int nxy = (c1[0] - c0[0] + 1) * (c1[1] - c0[1] + 1);
  const int ncell = nxy * (c1[2] - c0[2] + 1);
  int x = c0[0], y = c0[1], z = c0[2];
  for (int i0 = 0; i0 < ncell; i0 += 4) {
    int64_t cell[4];
    int slot[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cell[k] = base + ((int64_t)z * g.ny + y) * g.nx + x;
      if (++x > c1[0]) {
        x = c0[0];
        if (++y > c1[1]) {
          y = c0[1];
          ++z;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      slot[k] = i0 + k < ncell ? cell_start[cell[k]] + atomicSub(&cell_cnt[cell[k]], 1) - 1 : -1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (fits && slot[k] >= 0) items[slot[k]] = (int32_t)t;
  }
}

constexpr int kQueryWaves = kThreads / kWave;
constexpr int kQuerySet = 512;   // distinct candidates per slave triangle (LDS set)
constexpr int kQuerySmall = 64;       // the first set a triangle tries
constexpr int kQuerySmallProbe = 16;  // probes before it moves to the full set
constexpr int kMaxSlabs = 64;

// a / b for 0 <= a and 1 <= b (both below 2^24): a float quotient, then
// corrected to the exact integer one (a fraction of an integer division's cost)
__device__ inline int div_small(int a, int b) {
  int q = (int)__fdividef((float)a, (float)b);
  while (q > 0 && q * b > a) --q;
  while ((q + 1) * b <= a) ++q;
  return q;
}

// box of the prism slab {p + t n : p in T, t0 <= t <= t1}
__device__ inline void slab_box(const float tlo[3], const float thi[3], const float n[3], float t0, float t1,
                                float margin, float lo[3], float hi[3]) {
  for (int d = 0; d < 3; ++d) {
    float a = fminf(t0 * n[d], t1 * n[d]), b = fmaxf(t0 * n[d], t1 * n[d]);
    lo[d] = tlo[d] + a - margin;
    hi[d] = thi[d] + b + margin;
  }
}

// Thread per slave triangle (Morton order): the slave frame check
// (degenerate / non-finite triangles go to the status word, with the same
// criterion as the narrow phase), the box of the whole support prism
// {p + t n : p in T, |t| <= dhat} and the number of (master triangle, cell)
// incidences in the grid cells it covers.  Triangles with none get an empty
// candidate list at once; the others are appended to the query list that
// the per-triangle wave kernel walks.  The prism box is widened by a few
// ulps so that it covers the union of the query's slab boxes.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_query_pre(const R *__restrict__ xs, const int32_t *__restrict__ ts,
                                                         const int32_t *__restrict__ s_order,
                                                         const int32_t *__restrict__ s_env,
                                                         const EnvInfo *__restrict__ env,
                                                         const GridEnv *__restrict__ grid, int64_t Ts,
                                                         const int32_t *__restrict__ cell_start, int64_t cap_items,
                                                         int64_t total_cells, int32_t *__restrict__ cand_cnt,
                                                         int32_t *__restrict__ qlist, float4 *__restrict__ qrec,
                                                         int32_t *__restrict__ qcount, uint32_t *__restrict__ box,
                                                         int n_env, DevStatus *st, const uint32_t *__restrict__ epoch,
                                                         uint32_t *__restrict__ tile_act,
                                                         int32_t *__restrict__ tri_npair, int32_t *__restrict__ tri_rcnt,
                                                         int32_t *__restrict__ tri_poff, int32_t *__restrict__ tri_roff) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  if (i < n_env)  // the slave boxes were read by the grid kernels: empty them for the next call
    for (int d = 0; d < 3; ++d) {
      box[6 * i + d] = 0xffffffffu;  // min: largest ordered value
      box[6 * i + 3 + d] = 0u;       // max: smallest ordered value
    }
  bool active = false;
  int64_t t = -1;
  float4 fr[3];  // the listed triangle's frame for the query kernel
  if (i < Ts) {
    t = s_order[i];
    R p[3][3], e1[3], e2[3];
    for (int j = 0; j < 3; ++j) {
      const int64_t v = ts[3 * t + j];
      for (int d = 0; d < 3; ++d) p[j][d] = xs[3 * v + d];
    }
    const R *s0 = p[0];
    for (int d = 0; d < 3; ++d) {
      e1[d] = p[1][d] - s0[d];
      e2[d] = p[2][d] - s0[d];
    }
    const R c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const R len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    const R ref = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2] + e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    const bool finite = isfinite(len) && isfinite(ref) && isfinite(s0[0]) && isfinite(s0[1]) && isfinite(s0[2]);
    if (!finite) {
      set_error(st, GMCP_E_NONFINITE, (unsigned long long)t);
    } else if (!(len > R(1e-14) * ref)) {
      set_error(st, GMCP_E_DEGENERATE, (unsigned long long)t);
    } else if (cell_start[total_cells] <= cap_items) {
      const int e = s_env[t];
      const GridEnv g = grid[e];
      const float eps = (float)env[e].dhat;
      // the frame the query starts from: unit normal and vertex box (float,
      // grown outward)
      float tlo[3], thi[3], n[3];
      for (int d = 0; d < 3; ++d) {
        n[d] = (float)(c[d] / len);
        const float lo_d = fminf(fminf((float)p[0][d], (float)p[1][d]), (float)p[2][d]);
        const float hi_d = fmaxf(fmaxf((float)p[0][d], (float)p[1][d]), (float)p[2][d]);
        tlo[d] = lo_d - grow(lo_d);
        thi[d] = hi_d + grow(hi_d);
      }
      if (g.valid) {
        fr[0] = make_float4(tlo[0], tlo[1], tlo[2], __int_as_float((int)t));
        fr[1] = make_float4(thi[0], thi[1], thi[2], __int_as_float(e));
        fr[2] = make_float4(n[0], n[1], n[2], 0.0f);
        float lo[3], hi[3];
        const float ew = eps * (1.0f + 1e-5f);
        slab_box(tlo, thi, n, -ew, ew, 4.0f * eps * 1e-6f, lo, hi);
        if (box_hits_grid(g, lo, hi)) {
          int c0[3], c1[3];
          for (int d = 0; d < 3; ++d) {
            c0[d] = cell_coord(g, lo[d], d);
            c1[d] = cell_coord(g, hi[d], d);
          }
          const int64_t ncell = (int64_t)(c1[0] - c0[0] + 1) * (c1[1] - c0[1] + 1) * (c1[2] - c0[2] + 1);
          if (ncell > 4096) {
            active = true;  // too many cells to count here: let the wave kernel decide
          } else {
            const int64_t base = env[e].cell0;
            // the (y, z) rows of the box, 8 at a time so that their loads are
            // in flight together; a row's x-run of cells is contiguous
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
    if (!active) {
      // no candidates: the assembly's per-triangle outputs are empty, and a
      // work tile with no listed triangle is skipped by the narrow phase
      cand_cnt[t] = 0;
      tri_npair[t] = 0;
      tri_rcnt[t] = 0;
      tri_poff[t] = 0;
      tri_roff[t] = 0;
    } else {
      const EnvInfo &ev = env[s_env[t]];
      tile_act[ev.tile0 + (int)((i - ev.st0) / (kWave / ev.nq))] = *epoch;
    }
  }
  // list appends: wave ballots, block prefix in LDS, one atomic per block
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
    qb = sum ? atomicAdd(qcount, sum) : 0;
  }
  __syncthreads();
  if (active) {
    const int slot = qb + wq[w] + __popcll(m & ((1ull << lane) - 1));
    qlist[slot] = (int32_t)t;
    for (int k = 0; k < 3; ++k) qrec[3 * (int64_t)slot + k] = fr[k];
  }
}

// One wave per slave triangle.  The support prism (|t| <= eps_max along n_T)
// is covered by up to 64 slabs about one cell thick; the lanes split the
// cells of all slab boxes, test each master triangle in them (box overlap
// with the slab box, facing test with slack) and insert it into an LDS hash
// set, which removes the duplicates of overlapping cells and slabs.
// One pass: the set is compacted, sorted in LDS and written to a scratch
// list at an offset allocated from the block's share of the scratch (the
// content of a triangle's list does not depend on the order); k_cand_move
// then places every list at its CSR offset, so the candidate CSR is the
// same on every run.
template <typename R>
__device__ __forceinline__ void query_body(const R *__restrict__ xs, const int32_t *__restrict__ ts,
                                                     const int32_t *__restrict__ s_order,
                                                     const int32_t *__restrict__ s_env,
                                                     const EnvInfo *__restrict__ env,
                                                     const GridEnv *__restrict__ grid, int64_t Ts,
                                                     const int32_t *__restrict__ cell_start,
                                                     const int32_t *__restrict__ items,
                                                     const float4 *__restrict__ mbox, int32_t *__restrict__ cand_cnt,
                                                     int32_t *__restrict__ tmp_off, int32_t *__restrict__ cand_tmp,
                                                     int64_t cap_cand,
                                                     int64_t cap_items, int64_t total_cells,
                                                     const int32_t *__restrict__ qlist,
                                                     const float4 *__restrict__ qrec,
                                                     const int32_t *__restrict__ qcount,
                                                     int32_t *__restrict__ cand_blk, DevStatus *st) {
  __shared__ int32_t set[kQueryWaves][kQuerySet];
  __shared__ int32_t dense[kQueryWaves][kQuerySet];
  __shared__ int2 imark[kQueryWaves][kWave];  // per round of 64 incidences: where each item's incidences start
  __shared__ int blk_req;  // candidates requested by this block's triangles (LDS atomics)
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  // (blocks take list entries in dispatch order: an XCD-by-XCD mapping of
  // the list measured slower on the single indentation and no faster on
  // the batch)
  const int lblk = blockIdx.x;
  const int64_t nlist = *qcount;
  if (cell_start[total_cells] > cap_items) {  // grid incomplete
    for (int64_t li = (int64_t)lblk * kQueryWaves + w; li < nlist; li += (int64_t)gridDim.x * kQueryWaves)
      if (lane == 0) cand_cnt[qlist[li]] = 0;
    if (threadIdx.x == 0) cand_blk[blockIdx.x] = 0;
    return;
  }
  // the scratch is split evenly over the blocks; a block allocates its
  // triangles' lists from its own share with LDS atomics (no global
  // contention); a list that does not fit is dropped and the need reported
  const int64_t share = cap_cand / gridDim.x;
  if (threadIdx.x == 0) blk_req = 0;
  __syncthreads();
  // the waves walk the query list (triangles whose prism meets occupied
  // cells) with the frames the prepass stored: one load instead of the
  // chain triangle -> vertex ids -> positions (loading the next entry's
  // frame ahead measured slower: the registers it holds cause spills)
  for (int64_t li = (int64_t)lblk * kQueryWaves + w; li < nlist; li += (int64_t)gridDim.x * kQueryWaves) {
    const float4 f0 = qrec[3 * li], f1 = qrec[3 * li + 1], f2 = qrec[3 * li + 2];
    [&] {
  wave_sync();  // the previous triangle's LDS reads are done
  const int64_t t = __float_as_int(f0.w);
  const int e = __float_as_int(f1.w);
  const GridEnv g = grid[e];
  const float eps = (float)env[e].dhat;
  const float tlo[3] = {f0.x, f0.y, f0.z}, thi[3] = {f1.x, f1.y, f1.z}, n[3] = {f2.x, f2.y, f2.z};
  const bool ok = g.valid;
  const int S = ok ? max(1, min(kMaxSlabs, (int)ceilf(2.0f * eps / g.h))) : 0;
  const float dt = 2.0f * eps / (float)max(S, 1);
  const float margin = eps * 1e-6f;
  // lane s < S: cell range of slab s
  int c0[3] = {0, 0, 0}, c1[3] = {-1, -1, -1}, ncs = 0;
  if (lane < S) {
    float lo[3], hi[3];
    slab_box(tlo, thi, n, -eps + lane * dt, -eps + (lane + 1) * dt, margin, lo, hi);
    if (box_hits_grid(g, lo, hi)) {
      for (int d = 0; d < 3; ++d) {
        c0[d] = cell_coord(g, lo[d], d);
        c1[d] = cell_coord(g, hi[d], d);
      }
      ncs = (c1[0] - c0[0] + 1) * (c1[1] - c0[1] + 1) * (c1[2] - c0[2] + 1);
    }
  }
  const int incl = wave_incl_add(ncs);
  const int work = __shfl(incl, kWave - 1, kWave);
  const int64_t base = env[e].cell0;
  // the candidate set starts small (most triangles have a few candidates:
  // a short set is cheap to clear and compact); a triangle whose insertions
  // probe too far walks its cells again with the full set
  int tsz = kQuerySmall;
  bool full;
  for (;;) {
    for (int k = lane; k < tsz; k += kWave) set[w][k] = -1;
    wave_sync();
    full = false;
    const int max_probe = tsz == kQuerySet ? kQuerySet : kQuerySmallProbe;
    // the (slab, cell) items are taken 64 at a time; their master-triangle
    // incidences are flattened over the lanes (exclusive prefix of the cell
    // sizes in LDS, binary search per incidence), so a crowded cell does not
    // serialise on one lane
    for (int w0 = 0; w0 < work; w0 += kWave) {
      const int wi = w0 + lane;
      int s = 0;
      for (int z = 0; z < S; ++z) s += __shfl(incl, z, kWave) <= wi;  // slab holding item wi
      s = min(s, kWave - 1);
      const int sc0x = __shfl(c0[0], s, kWave), sc0y = __shfl(c0[1], s, kWave), sc0z = __shfl(c0[2], s, kWave);
      const int sc1x = __shfl(c1[0], s, kWave), sc1y = __shfl(c1[1], s, kWave);
      const int sstart = __shfl(incl - ncs, s, kWave);
      int cs = 0, cn = 0;
      if (wi < work) {
        const int nxr = sc1x - sc0x + 1, nyr = sc1y - sc0y + 1;
        const int li = wi - sstart;
        const int q1 = div_small(li, nxr), q2 = div_small(q1, nyr);
        const int x = sc0x + (li - q1 * nxr), y = sc0y + (q1 - q2 * nyr), zc = sc0z + q2;
        const int64_t cell = base + ((int64_t)zc * g.ny + y) * g.nx + x;
        cs = cell_start[cell];
        cn = cell_start[cell + 1] - cs;
      }
      const int ci = wave_incl_add(cn);
      const int tot = __shfl(ci, kWave - 1, kWave);
      const int pfx = ci - cn;  // the lane's first incidence
      // incidences 64 per round, one per lane; the owner of incidence f is
      // the item whose range [pfx, pfx + cn) holds it: every item with
      // incidences marks the lane of its first one in LDS (its cell offset
      // less its prefix, and its slab), a ballot of the marks gives the
      // highest mark at or below each lane, and a lane before the round's
      // first mark continues the previous round's last item - two round
      // trips instead of a six-step binary search over the prefixes
      int carry_off = 0, carry_sl = 0;
      for (int f0 = 0; f0 < tot; f0 += kWave) {
        wave_sync();  // the previous round's mark reads are done
        imark[w][lane] = make_int2(0, -1);
        if (cn > 0 && pfx >= f0 && pfx < f0 + kWave) imark[w][pfx - f0] = make_int2(cs - pfx, s);
        wave_sync();
        const int2 mk = imark[w][lane];
        const uint64_t le = __ballot(mk.y >= 0) & ((2ull << lane) - 1);  // marks at lanes 0..lane
        const int pos = le ? 63 - __builtin_clzll(le) : 0;
        int off = __shfl(mk.x, pos, kWave), sl = __shfl(mk.y, pos, kWave);
        if (!le) {
          off = carry_off;
          sl = carry_sl;
        }
        carry_off = __builtin_amdgcn_readlane(off, kWave - 1);  // uniform: scalar registers
        carry_sl = __builtin_amdgcn_readlane(sl, kWave - 1);
        const int f = f0 + lane;
        if (f >= tot) continue;
        const int j = off + f;
        float lo[3], hi[3];
        slab_box(tlo, thi, n, -eps + sl * dt, -eps + (sl + 1) * dt, margin, lo, hi);
        const int M = items[j];
        const float4 a = mbox[3 * (int64_t)M], b = mbox[3 * (int64_t)M + 1];
        if (a.x > hi[0] || b.x < lo[0] || a.y > hi[1] || b.y < lo[1] || a.z > hi[2] || b.z < lo[2]) continue;
        const float4 nm = mbox[3 * (int64_t)M + 2];
        // facing test with slack: the narrow phase takes the exact decision
        if (n[0] * nm.x + n[1] * nm.y + n[2] * nm.z >= 1e-5f) continue;
        uint32_t h = ((uint32_t)M * 2654435761u) & (uint32_t)(tsz - 1);
        int probe = 0;
        for (; probe < max_probe; ++probe) {
          const int prev = atomicCAS(&set[w][h], -1, M);
          if (prev == -1 || prev == M) break;
          h = (h + 1) & (uint32_t)(tsz - 1);
        }
        if (probe == max_probe) full = true;
      }
    }
    if (!__any(full) || tsz == kQuerySet) break;
    tsz = kQuerySet;
    wave_sync();  // the small set's accesses are done before the full one is cleared
  }
  if (__any(full)) {
    if (lane == 0) {
      atomicCAS(&st->code, 0, GMCP_E_CAPACITY);
      atomicMin(&st->index, (unsigned long long)t);
      cand_cnt[t] = 0;
    }
    return;
  }
  wave_sync();
  int nu = 0;
  for (int k0 = 0; k0 < tsz; k0 += kWave) {
    int k = k0 + lane;
    bool used = k < tsz && set[w][k] >= 0;
    uint64_t m = __ballot(used);
    if (used) dense[w][nu + __popcll(m & ((1ull << lane) - 1))] = set[w][k];
    nu += __popcll(m);
  }
  int off = 0;
  if (lane == 0) {
    off = nu ? atomicAdd(&blk_req, nu) : 0;
    const bool fits = (int64_t)off + nu <= share;
    cand_cnt[t] = fits ? nu : 0;
    tmp_off[t] = (int32_t)(blockIdx.x * share + off);
    if (!fits) off = -1;
  }
  off = __shfl(off, 0, kWave);
  wave_sync();
  if (off < 0) return;  // dropped (capacity reported below)
  int32_t *l = cand_tmp + blockIdx.x * share + off;
  for (int k = lane; k < nu; k += kWave) {  // rank sort: ids are unique
    int v = dense[w][k], r = 0;
    for (int m = 0; m < nu; ++m) r += dense[w][m] < v;
    l[r] = v;
  }
  wave_sync();  // the set is reused by the wave's next triangle
    }();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    cand_blk[blockIdx.x] = blk_req;  // summed by gmcp_status
    if ((int64_t)blk_req > share) {
      atomicMax(&st->need_cand, (unsigned long long)blk_req * gridDim.x);
      atomicCAS(&st->code, 0, GMCP_E_CAPACITY);
    }
  }
}

// float: seven waves per SIMD (72 registers); double as compiled
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(7))) void k_query_f32(
    const float *__restrict__ xs, const int32_t *__restrict__ ts, const int32_t *__restrict__ s_order,
    const int32_t *__restrict__ s_env, const EnvInfo *__restrict__ env, const GridEnv *__restrict__ grid, int64_t Ts,
    const int32_t *__restrict__ cell_start, const int32_t *__restrict__ items, const float4 *__restrict__ mbox,
    int32_t *__restrict__ cand_cnt, int32_t *__restrict__ tmp_off, int32_t *__restrict__ cand_tmp, int64_t cap_cand,
    int64_t cap_items, int64_t total_cells, const int32_t *__restrict__ qlist, const float4 *__restrict__ qrec,
    const int32_t *__restrict__ qcount, int32_t *__restrict__ cand_blk, DevStatus *st) {
  query_body<float>(xs, ts, s_order, s_env, env, grid, Ts, cell_start, items, mbox, cand_cnt, tmp_off, cand_tmp,
                    cap_cand, cap_items, total_cells, qlist, qrec, qcount, cand_blk, st);
}
__global__ __launch_bounds__(kThreads) void k_query_f64(
    const double *__restrict__ xs, const int32_t *__restrict__ ts, const int32_t *__restrict__ s_order,
    const int32_t *__restrict__ s_env, const EnvInfo *__restrict__ env, const GridEnv *__restrict__ grid, int64_t Ts,
    const int32_t *__restrict__ cell_start, const int32_t *__restrict__ items, const float4 *__restrict__ mbox,
    int32_t *__restrict__ cand_cnt, int32_t *__restrict__ tmp_off, int32_t *__restrict__ cand_tmp, int64_t cap_cand,
    int64_t cap_items, int64_t total_cells, const int32_t *__restrict__ qlist, const float4 *__restrict__ qrec,
    const int32_t *__restrict__ qcount, int32_t *__restrict__ cand_blk, DevStatus *st) {
  query_body<double>(xs, ts, s_order, s_env, env, grid, Ts, cell_start, items, mbox, cand_cnt, tmp_off, cand_tmp,
                    cap_cand, cap_items, total_cells, qlist, qrec, qcount, cand_blk, st);
}

// Each listed triangle's sorted list, from its scratch offset to its CSR
// offset (one wave per list entry of the query list).
__global__ __launch_bounds__(kThreads) void k_cand_move(const int32_t *__restrict__ qlist,
                                                         const int32_t *__restrict__ qcount,
                                                         const int32_t *__restrict__ cand_cnt,
                                                         const int32_t *__restrict__ tmp_off,
                                                         const int32_t *__restrict__ cand_off,
                                                         const int32_t *__restrict__ cand_tmp,
                                                         int32_t *__restrict__ cand) {
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int64_t nlist = *qcount;
  for (int64_t li = (int64_t)blockIdx.x * kQueryWaves + w; li < nlist; li += (int64_t)gridDim.x * kQueryWaves) {
    const int t = qlist[li];
    const int n = cand_cnt[t], src = tmp_off[t], dst = cand_off[t];
    for (int k = lane; k < n; k += kWave) cand[dst + k] = cand_tmp[src + k];
  }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

template <typename R>
hipError_t build_grid(gmcp_ctx *c, const R *xs, const R *xm, const R *dxs, const R *dxm, bool swept) {
  Buffers &b = c->b;
  uint32_t *box = swept ? b.sbox : b.box;
  GridEnv *grid = swept ? b.sgrid : b.grid;
  int32_t *cnt = swept ? b.scell_cnt : b.cell_cnt;
  int32_t *start = swept ? b.scell_start : b.cell_start;
  int32_t *items = swept ? b.sitems : b.items;
  float4 *mbox = swept ? b.smbox : b.mbox;
  hipStream_t s = c->stream;
  // the boxes are empty here: the swept ones from the caller's stage_init,
  // the static ones from the previous query prepass (or creation); the
  // slave-box kernel also zeroes the broad phase's two list counters
  if (c->Ts)
    hipLaunchKernelGGL(k_slave_box<R>, dim3((unsigned)((c->Vs + kBoxThreads - 1) / kBoxThreads)),
                       dim3(kBoxThreads), 0, s, xs, swept ? dxs : nullptr, b.s_venv, c->Vs, box,
                       swept ? nullptr : b.qcount, swept ? nullptr : b.cand_cnt + c->Ts, swept ? nullptr : b.epoch);
  const int64_t nmb = std::max<int64_t>(c->Tm, c->n_env);
  if (nmb)
    hipLaunchKernelGGL(k_master_boxes<R>, dim3(nblk(nmb)), dim3(kThreads), 0, s, xm, swept ? dxm : nullptr, c->tm,
                       c->Tm, mbox, b.m_env, b.env, box, grid, c->n_env, swept ? 1 : 0, cnt);
  hipError_t e = scan_exclusive(c, cnt, start, c->total_cells + 1, swept, grid);
  if (e != hipSuccess) return e;
  if (c->Tm)
    hipLaunchKernelGGL(k_grid_insert, dim3(nblk(c->Tm)), dim3(kThreads), 0, s, mbox, b.m_env, b.env, grid, c->Tm,
                       cnt, start, items, c->caps.grid_items, c->total_cells, b.status);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_broadphase(gmcp_ctx *c, const R *xs, const R *xm) {
  Buffers &b = c->b;
  hipStream_t s = c->stream;
  hipError_t e = hipSuccess;
  if (!c->Ts) {  // no slave triangle: nothing below resets these
    StageInit si;
    si.which = 1;
    si.box = b.box;
    si.zero[0] = b.qcount;
    si.nzero[0] = 1;
    si.zero[1] = b.cand_cnt + c->Ts;
    si.nzero[1] = 1;
    if ((e = stage_init(c, si)) != hipSuccess) return e;
  }
  prof_mark(c, ST_GRID, 0);
  e = build_grid<R>(c, xs, xm, nullptr, nullptr, false);
  prof_mark(c, ST_GRID, 1);
  if (e != hipSuccess) return e;
  prof_mark(c, ST_QUERY_PRE, 0);
  if (c->Ts)
    hipLaunchKernelGGL(k_query_pre<R>, dim3(nblk(std::max<int64_t>(c->Ts, c->n_env))), dim3(kThreads), 0, s, xs, c->ts,
                       b.s_order, b.s_env, b.env, b.grid, c->Ts, b.cell_start, c->caps.grid_items, c->total_cells,
                       b.cand_cnt, b.qlist, b.qrec, b.qcount, b.box, c->n_env, b.status, b.epoch, b.tile_act,
                       b.tri_npair, b.tri_rcnt, b.tri_poff, b.tri_roff);
  prof_mark(c, ST_QUERY_PRE, 1);
  // the wave kernels walk the query list with a fixed grid, all of it
  // resident at once
  if (c->query_grid_max == 0)
    c->query_grid_max = std::min<int64_t>(kQueryBlocks, sizeof(R) == 4 ? resident_blocks(c, k_query_f32, kThreads, 0)
                                                                      : resident_blocks(c, k_query_f64, kThreads, 0));
  const int64_t qmax = c->tune.query_blocks > 0 ? c->tune.query_blocks : c->query_grid_max;
  const int64_t qb = std::min<int64_t>((c->Ts + kQueryWaves - 1) / kQueryWaves, qmax);
  const dim3 qgrid((unsigned)(qb > 0 ? qb : 1));
  prof_mark(c, ST_QUERY_COUNT, 0);
  c->query_blocks = c->Ts ? (int)qgrid.x : 0;
  if (c->Ts)
  {
    if constexpr (sizeof(R) == 4)
      hipLaunchKernelGGL(k_query_f32, qgrid, dim3(kThreads), 0, s, xs, c->ts, b.s_order, b.s_env, b.env, b.grid, c->Ts,
                       b.cell_start, b.items, b.mbox, b.cand_cnt, b.cand_tmp_off, b.cand_tmp, c->caps.candidates,
                       c->caps.grid_items, c->total_cells, b.qlist, b.qrec, b.qcount, b.cand_blk, b.status);
    else
      hipLaunchKernelGGL(k_query_f64, qgrid, dim3(kThreads), 0, s, xs, c->ts, b.s_order, b.s_env, b.env, b.grid, c->Ts,
                       b.cell_start, b.items, b.mbox, b.cand_cnt, b.cand_tmp_off, b.cand_tmp, c->caps.candidates,
                       c->caps.grid_items, c->total_cells, b.qlist, b.qrec, b.qcount, b.cand_blk, b.status);
  }
  prof_mark(c, ST_QUERY_COUNT, 1);
  // the narrow phase reads every list where the query wrote it (count and
  // scratch offset per triangle); the candidate CSR is built only for export
  return hipGetLastError();
}

hipError_t build_candidate_csr(gmcp_ctx *c) {
  Buffers &b = c->b;
  hipError_t e = scan_exclusive(c, b.cand_cnt, b.cand_off, c->Ts + 1);
  if (e != hipSuccess) return e;
  const int64_t qb = (c->Ts + kQueryWaves - 1) / kQueryWaves;
  const dim3 qgrid((unsigned)(qb < kQueryBlocks ? (qb > 0 ? qb : 1) : kQueryBlocks));
  if (c->Ts)
    hipLaunchKernelGGL(k_cand_move, qgrid, dim3(kThreads), 0, c->stream, b.qlist, b.qcount, b.cand_cnt,
                       b.cand_tmp_off, b.cand_off, b.cand_tmp, b.cand);
  return hipGetLastError();
}

template hipError_t build_grid<float>(gmcp_ctx *, const float *, const float *, const float *, const float *, bool);
template hipError_t build_grid<double>(gmcp_ctx *, const double *, const double *, const double *, const double *,
                                       bool);
template hipError_t launch_broadphase<float>(gmcp_ctx *, const float *, const float *);
template hipError_t launch_broadphase<double>(gmcp_ctx *, const double *, const double *);

}  // namespace gmcp
