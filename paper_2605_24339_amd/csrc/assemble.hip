// GMCP assembly: narrow phase, barrier, per-triangle / per-pair sums, BSR
// scatter, gradient, energy; plus the Hessian-vector product and the
// per-sample export that reuse the same intermediate sums.
//
// Work decomposition of the narrow phase (the hot loop): one wave64 per work
// tile of up to 64/(n*n) slave triangles, Morton-ordered; lane = one sample.
// Each round, every lane stages one candidate master triangle of its own
// slave triangle into LDS - pair-local edge vectors relative to the slave
// triangle's first vertex, the facing denominator and the inverse Gram
// matrix of Eq. (gram) - and then every lane tests all staged candidates of
// its triangle (an LDS broadcast among the triangle's lanes).  Geometric
// quantities are formed as differences of nearby points only, never from
// absolute sample positions, so float32 keeps the small gaps accurate.
//
// Reductions are deterministic: per triangle and per pair in lane order,
// per BSR row by per-column sums in a canonical contribution order, per
// master triangle over pairs sorted by slave triangle.
#include "common.h"

namespace gmcp {

namespace {

constexpr int kThreads = 256;

template <typename R> struct CandL {
  R d0[3], f1[3], f2[3], N[3];
  R g11, g12, g22, inv_den;
  int32_t M;
};

template <typename R> struct SampL {
  int32_t M;
  R c1, c2, b0, b1, b2;
};

__device__ inline int sym3(int a, int b) {  // 00 01 02 11 12 22
  if (a > b) { int t = a; a = b; b = t; }
  return a == 0 ? b : (a == 1 ? 2 + b : 5);
}

template <typename R> __device__ inline R hermite(R x, R delta) {
  if (x <= R(0)) return R(0);
  if (x >= delta) return R(1);
  R t = x / delta;
  return t * t * (R(3) - R(2) * t);
}

template <typename R> __device__ inline R log1p_r(R x);
template <> __device__ inline float log1p_r<float>(float x) { return log1pf(x); }
template <> __device__ inline double log1p_r<double>(double x) { return log1p(x); }

template <typename R>
struct NarrowArgs {
  const R *xs, *xm;
  const int32_t *ts, *tm;
  const Tile *tiles;
  int n_tiles;
  const int32_t *s_order, *samp_off;
  const EnvInfo *env;
  const double *rule;
  const R *area;
  const int32_t *cand_off, *cand;
  int64_t Ts, cap_cand;
  const R *g_ref, *dgap;
  Rec<R> *rec;
  int64_t cap_active;
  R *tri_nrm, *tri_sum;
  int32_t *tri_npair, *tri_poff, *tri_roff, *tri_rcnt;
  Pair<R> *pair;
  int64_t cap_pairs;
  double *tile_E;
  DevStatus *st;
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_narrow(NarrowArgs<R> a) {
  __shared__ CandL<R> sc[kTilePerBlock][kWave];
  __shared__ SampL<R> ss[kTilePerBlock][kWave];
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int tile_id = xcd_block(blockIdx.x, gridDim.x) * kTilePerBlock + w;
  if (tile_id >= a.n_tiles) return;  // waves are independent: no block barrier below
  if (a.cand_off[a.Ts] > a.cap_cand) return;
  const Tile tl = a.tiles[tile_id];
  const EnvInfo &ev = a.env[tl.env];
  const int nq = tl.nq;
  const int j = lane / nq, q = lane - j * nq;
  const bool valid = j < tl.count;
  const int T = valid ? a.s_order[tl.first + j] : 0;
  const R dhat = (R)ev.dhat, kappa = (R)ev.kappa, deltaT = (R)ev.delta_T;

  // ---- slave frame: first vertex, edges, unit normal (A2)
  R s0[3] = {0, 0, 0}, e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0}, n[3] = {0, 0, 1};
  bool degen = false;
  if (valid) {
    int v0 = a.ts[3 * T], v1 = a.ts[3 * T + 1], v2 = a.ts[3 * T + 2];
    for (int d = 0; d < 3; ++d) {
      s0[d] = a.xs[3 * (int64_t)v0 + d];
      e1[d] = a.xs[3 * (int64_t)v1 + d] - s0[d];
      e2[d] = a.xs[3 * (int64_t)v2 + d] - s0[d];
    }
    R c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    R len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    R ref = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2] + e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    bool finite = isfinite(len) && isfinite(ref) && isfinite(s0[0]) && isfinite(s0[1]) && isfinite(s0[2]);
    if (!finite) {
      if (q == 0) set_error(a.st, GMCP_E_NONFINITE, (unsigned long long)T);
      degen = true;
    } else if (!(len > R(1e-14) * ref)) {
      if (q == 0) set_error(a.st, GMCP_E_DEGENERATE, (unsigned long long)T);
      degen = true;
    } else {
      for (int d = 0; d < 3; ++d) n[d] = c[d] / len;
    }
  }
  const int k = valid ? a.samp_off[T] + q : 0;
  const double *rq = a.rule + ((ev.rule_n - 1) * 16 + q) * 3;
  const R xi = (R)rq[0], eta = (R)rq[1], wq = (R)rq[2];
  const R ps[3] = {xi * e1[0] + eta * e2[0], xi * e1[1] + eta * e2[1], xi * e1[2] + eta * e2[2]};
  R eps = dhat;
  if (valid && a.g_ref) eps = fmin(R(0.9) * a.g_ref[k], dhat);

  const int cbeg = (valid && !degen) ? a.cand_off[T] : 0;
  const int ccnt = (valid && !degen) ? a.cand_off[T + 1] - cbeg : 0;
  int maxc = ccnt;
  for (int o = 32; o > 0; o >>= 1) maxc = max(maxc, __shfl_xor(maxc, o, kWave));

  // ---- candidate loop (A4)
  int bM = -1;
  R bt = 0, bb0 = 0, bb1 = 0, bb2 = 0;
  bool pen = false;
  for (int base = 0; base < maxc; base += nq) {
    CandL<R> cl;
    cl.M = -1;
    int ci = base + q;
    if (ci < ccnt) {
      int M = a.cand[cbeg + ci];
      int64_t m0 = a.tm[3 * (int64_t)M], m1 = a.tm[3 * (int64_t)M + 1], m2 = a.tm[3 * (int64_t)M + 2];
      R p0[3], f1[3], f2[3];
      for (int d = 0; d < 3; ++d) {
        R x0 = a.xm[3 * m0 + d];
        p0[d] = x0 - s0[d];
        f1[d] = a.xm[3 * m1 + d] - x0;
        f2[d] = a.xm[3 * m2 + d] - x0;
      }
      R N[3] = {f1[1] * f2[2] - f1[2] * f2[1], f1[2] * f2[0] - f1[0] * f2[2], f1[0] * f2[1] - f1[1] * f2[0]};
      R den = n[0] * N[0] + n[1] * N[1] + n[2] * N[2];
      R a11 = f1[0] * f1[0] + f1[1] * f1[1] + f1[2] * f1[2];
      R a12 = f1[0] * f2[0] + f1[1] * f2[1] + f1[2] * f2[2];
      R a22 = f2[0] * f2[0] + f2[1] * f2[1] + f2[2] * f2[2];
      R det = a11 * a22 - a12 * a12;
      if (den < R(0) && det > R(0)) {
        R id = R(1) / det;
        cl.M = M;
        for (int d = 0; d < 3; ++d) {
          cl.d0[d] = p0[d];
          cl.f1[d] = f1[d];
          cl.f2[d] = f2[d];
          cl.N[d] = N[d];
        }
        cl.g11 = a22 * id;
        cl.g12 = -a12 * id;
        cl.g22 = a11 * id;
        cl.inv_den = R(1) / den;
      }
    }
    sc[w][lane] = cl;
    wave_sync();
    int nc = min(nq, ccnt - base);
    for (int c = 0; c < nc; ++c) {
      const CandL<R> &e = sc[w][j * nq + c];
      if (e.M < 0) continue;
      R dv[3] = {e.d0[0] - ps[0], e.d0[1] - ps[1], e.d0[2] - ps[2]};  // m0 - x_s,k
      R t = (e.N[0] * dv[0] + e.N[1] * dv[1] + e.N[2] * dv[2]) * e.inv_den;
      R r[3] = {t * n[0] - dv[0], t * n[1] - dv[1], t * n[2] - dv[2]};  // x_m,k - m0
      R r1 = r[0] * e.f1[0] + r[1] * e.f1[1] + r[2] * e.f1[2];
      R r2 = r[0] * e.f2[0] + r[1] * e.f2[1] + r[2] * e.f2[2];
      R b1 = e.g11 * r1 + e.g12 * r2, b2 = e.g12 * r1 + e.g22 * r2;
      R b0 = R(1) - b1 - b2;
      if (b0 < R(0) || b1 < R(0) || b2 < R(0)) continue;
      if (t > R(0) && t < eps) {
        if (bM < 0 || t < bt || (t == bt && e.M < bM)) {
          bM = e.M;
          bt = t;
          bb0 = b0;
          bb1 = b1;
          bb2 = b2;
        }
      } else if (t > -eps && t <= R(0)) {
        pen = true;
      }
    }
    wave_sync();
  }
  if (pen) set_error(a.st, GMCP_E_PENETRATION, (unsigned long long)k);

  // ---- barrier, weight, sample scalars (A5)
  const bool sel = valid && bM >= 0;
  R g = 0, c1 = 0, c2 = 0, pr = 0;
  double E = 0.0;
  if (sel) {
    g = bt;
    if (a.dgap) g += a.dgap[k];
    if (!(g > R(0))) {
      set_error(a.st, GMCP_E_PENETRATION, (unsigned long long)k);
    } else if (g < eps) {
      R gam = deltaT > R(0) ? hermite(fmin(bb0, fmin(bb1, bb2)), deltaT) : R(1);
      R wk = R(2) * a.area[T] * wq;
      R dd = g - eps;
      R L = log1p_r<R>(dd / eps);  // ln(g / eps), accurate near the support edge
      R B = -dd * dd * L;
      R B1 = -R(2) * dd * L - dd * dd / g;
      R B2 = -R(2) * L - R(4) * dd / g + dd * dd / (g * g);
      R kw = kappa * wk * gam;
      E = (double)(kw * B);
      c1 = kw * B1;
      c2 = fmax(kw * B2, R(0));  // PSD projection of the rank-one block
      pr = -kappa * gam * B1;
    }
  }

  // ---- energy of the tile (fixed butterfly order)
  for (int o = 32; o > 0; o >>= 1) E += __shfl_xor(E, o, kWave);
  if (lane == 0) a.tile_E[tile_id] = E;

  SampL<R> me;
  me.M = sel ? bM : -1;
  me.c1 = c1;
  me.c2 = c2;
  me.b0 = bb0;
  me.b1 = bb1;
  me.b2 = bb2;
  ss[w][lane] = me;
  wave_sync();

  // ---- per slave triangle sums (A6): ss[6] = sum c2 bs_a bs_b, gs[3] = sum c1 bs_a
  const uint64_t one = 1;
  const uint64_t trimask = valid ? (((one << nq) - 1) << (j * nq)) : 0;
  const uint64_t selmask = __ballot(sel);
  const bool tri_active = (selmask & trimask) != 0;
  if (valid && tri_active) {
    for (int v = q; v < 9; v += nq) {
      R acc = 0;
      int ia, ib;
      if (v < 6) {
        const int A[6] = {0, 0, 0, 1, 1, 2}, B[6] = {0, 1, 2, 1, 2, 2};
        ia = A[v];
        ib = B[v];
      } else {
        ia = v - 6;
        ib = -1;
      }
      for (int i = 0; i < nq; ++i) {
        const SampL<R> &o = ss[w][j * nq + i];
        if (o.M < 0) continue;
        const double *ri = a.rule + ((ev.rule_n - 1) * 16 + i) * 3;
        R bs[3] = {R(1) - (R)ri[0] - (R)ri[1], (R)ri[0], (R)ri[1]};
        acc += ib >= 0 ? o.c2 * bs[ia] * bs[ib] : o.c1 * bs[ia];
      }
      a.tri_sum[9 * (int64_t)T + v] = acc;
    }
    if (q == 0)
      for (int d = 0; d < 3; ++d) a.tri_nrm[3 * (int64_t)T + d] = n[d];
  }

  // ---- selected-sample records (wave prefix + one atomic per wave)
  const int nsel = __popcll(selmask);
  const int rpre = __popcll(selmask & ((one << lane) - 1));
  unsigned long long rbase = 0;
  if (lane == 0 && nsel) rbase = atomicAdd(&a.st->n_active, (unsigned long long)nsel);
  rbase = __shfl(rbase, 0, kWave);
  const bool rec_ok = rbase + nsel <= (unsigned long long)a.cap_active;
  if (nsel && !rec_ok && lane == 0) atomicCAS(&a.st->code, 0, GMCP_E_CAPACITY);
  if (sel && rec_ok) {
    Rec<R> r;
    r.k = k;
    r.M = bM;
    r.T = T;
    r.q = q;
    r.g = g;
    r.b0 = bb0;
    r.b1 = bb1;
    r.b2 = bb2;
    r.c1 = c1;
    r.c2 = c2;
    r.p = pr;
    r.pad = 0;
    a.rec[rbase + rpre] = r;
  }

  // ---- contact pairs: one per distinct master triangle of a slave triangle
  bool leader = false;
  int rank = 0;
  if (sel) {
    leader = true;
    for (int i = 0; i < q; ++i)
      if (ss[w][j * nq + i].M == bM) {
        leader = false;
        break;
      }
  }
  const uint64_t leadmask = __ballot(leader);
  if (leader) {
    for (int i = 0; i < nq; ++i) {
      const SampL<R> &o = ss[w][j * nq + i];
      if (((leadmask >> (j * nq + i)) & 1) && o.M < bM) ++rank;
    }
  }
  const int npair_w = __popcll(leadmask);
  unsigned long long pbase = 0;
  if (lane == 0 && npair_w) pbase = atomicAdd(&a.st->n_pairs, (unsigned long long)npair_w);
  pbase = __shfl(pbase, 0, kWave);
  const bool pair_ok = pbase + npair_w <= (unsigned long long)a.cap_pairs;
  if (npair_w && !pair_ok && lane == 0) atomicCAS(&a.st->code, 0, GMCP_E_CAPACITY);
  const int tri_pre = valid ? __popcll(leadmask & ((one << (j * nq)) - 1)) : 0;
  if (valid && q == 0) {
    a.tri_npair[T] = __popcll(leadmask & trimask);
    a.tri_poff[T] = (int32_t)(pbase + tri_pre);
    a.tri_rcnt[T] = __popcll(selmask & trimask);
    a.tri_roff[T] = (int32_t)(rbase + __popcll(selmask & ((one << (j * nq)) - 1)));
  }
  if (leader && pair_ok) {
    Pair<R> p;
    p.T = T;
    p.M = bM;
    for (int z = 0; z < 6; ++z) p.mm[z] = 0;
    for (int z = 0; z < 9; ++z) p.sm[z] = 0;
    for (int z = 0; z < 3; ++z) p.gm[z] = 0;
    for (int i = 0; i < nq; ++i) {
      const SampL<R> &o = ss[w][j * nq + i];
      if (o.M != bM) continue;
      const double *ri = a.rule + ((ev.rule_n - 1) * 16 + i) * 3;
      R bs[3] = {R(1) - (R)ri[0] - (R)ri[1], (R)ri[0], (R)ri[1]};
      R bm[3] = {o.b0, o.b1, o.b2};
      p.mm[0] += o.c2 * bm[0] * bm[0];
      p.mm[1] += o.c2 * bm[0] * bm[1];
      p.mm[2] += o.c2 * bm[0] * bm[2];
      p.mm[3] += o.c2 * bm[1] * bm[1];
      p.mm[4] += o.c2 * bm[1] * bm[2];
      p.mm[5] += o.c2 * bm[2] * bm[2];
      for (int s = 0; s < 3; ++s)
        for (int m = 0; m < 3; ++m) p.sm[3 * s + m] -= o.c2 * bs[s] * bm[m];
      for (int m = 0; m < 3; ++m) p.gm[m] += o.c1 * bm[m];
    }
    a.pair[pbase + tri_pre + rank] = p;
  }
}

// ---------------------------------------------------- pairs by master tri
// pass 0: count pairs per master triangle; pass 1: place (slave triangle,
// pair) keys into the buckets in arrival order (counters return to zero)
template <typename R>
__global__ void k_pair_bucket(const Pair<R> *__restrict__ pair, const DevStatus *st, int64_t cap_pairs,
                              int32_t *__restrict__ mp_cnt, const int32_t *__restrict__ mp_off,
                              long long *__restrict__ mp_key, int pass) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t np = (int64_t)st->n_pairs;
  if (np > cap_pairs || p >= np) return;
  int M = pair[p].M;
  if (pass == 0) {
    atomicAdd(&mp_cnt[M], 1);
  } else {
    int slot = mp_off[M] + atomicSub(&mp_cnt[M], 1) - 1;
    mp_key[slot] = ((long long)pair[p].T << 32) | (long long)p;
  }
}

// deterministic order inside each bucket: every key is ranked among its
// bucket's keys (slave triangle, unique per bucket) and written in place
template <typename R>
__global__ void k_bucket_rank(const Pair<R> *__restrict__ pair, const int32_t *__restrict__ mp_off,
                              const long long *__restrict__ mp_key, int32_t *__restrict__ mp_list,
                              const DevStatus *st, int64_t cap_pairs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t np = (int64_t)st->n_pairs;
  if (np > cap_pairs || i >= np) return;
  long long key = mp_key[i];
  int M = pair[key & 0xffffffffLL].M;
  int b = mp_off[M], e = mp_off[M + 1], r = 0;
  for (int j = b; j < e; ++j) r += mp_key[j] < key;
  mp_list[b + r] = (int32_t)(key & 0xffffffffLL);
}

template <typename R>
struct RowArgs {
  const int32_t *ts, *tm;
  int64_t Vs, V;
  bool kinematic;
  const int32_t *s_vt_off, *s_vt, *m_vt_off, *m_vt;
  const int32_t *tri_npair, *tri_poff;
  const R *tri_sum, *tri_nrm;
  const Pair<R> *pair;
  const int32_t *mp_off, *mp_list;
  const DevStatus *st_r;
  DevStatus *st;
  int64_t cap_pairs;
  int32_t *row_cnt;
  const int32_t *row_ptr;
  int32_t *col;
  R *val;
  int64_t cap_nnzb;
  R *grad;   // nullable: written by the writing pass (pass 1) or alone (pass 2)
};

constexpr int kRowWaves = 2;

// slot of column `col` in an open-addressing table of `slots` (power of 2)
__device__ inline int row_slot(int32_t *key, int slots, int32_t col, bool *full) {
  uint32_t h = ((uint32_t)col * 2654435761u) & (uint32_t)(slots - 1);
  for (int probe = 0; probe < slots; ++probe) {
    int32_t prev = atomicCAS(&key[h], -1, col);
    if (prev == -1 || prev == col) return (int)h;
    h = (h + 1) & (uint32_t)(slots - 1);
  }
  *full = true;
  return -1;
}

// One wave per BSR row.  pass 0 counts the distinct columns, pass 1 writes
// them, pass 2 only computes the gradient row.  The row's contributions
// (column, coef, slave triangle whose normal n_T it carries; block =
// coef n_T n_T^T) are enumerated in a canonical order - source by source,
// sources in adjacency order - and their columns inserted into an LDS hash
// set.  In pass 1 the contributions are also kept in LDS (rows longer than
// kRowEnt re-walk their sources instead); each lane then owns one distinct
// column and sums its contributions in the canonical order, so the float
// sums are the same on every run.  Columns are ranked and written ascending.
constexpr int kRowEnt = 512;

template <typename R, int PASS>
__global__ __launch_bounds__(kWave *kRowWaves) void k_rows(RowArgs<R> a, int slots) {
  constexpr int pass = PASS;
  extern __shared__ __align__(16) unsigned char smem[];
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const size_t per_wave = (size_t)slots * 8 + (pass == 1 ? (size_t)kRowEnt * (8 + sizeof(R)) : 0);
  int32_t *key = reinterpret_cast<int32_t *>(smem + (size_t)w * per_wave);
  int32_t *dense = key + slots;
  int32_t *ecol = dense + slots;
  int32_t *etri = ecol + kRowEnt;
  R *ecoef = reinterpret_cast<R *>(etri + kRowEnt);
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + w;
  if (row >= a.V) return;
  if ((int64_t)a.st_r->n_pairs > a.cap_pairs) {
    if (pass == 0 && lane == 0) a.row_cnt[row] = 0;
    return;
  }
  if (pass == 1 && (int64_t)a.row_ptr[a.V] > a.cap_nnzb) return;
  const bool slave = row < a.Vs;
  const int64_t vid = slave ? row : row - a.Vs;
  const int sb = slave ? a.s_vt_off[vid] : a.m_vt_off[vid];
  const int se = slave ? a.s_vt_off[vid + 1] : a.m_vt_off[vid + 1];

  // contributions of one source (incident triangle), in canonical order
  auto src_count = [&](int src) -> int {
    int t = (slave ? a.s_vt[src] : a.m_vt[src]) >> 2;
    if (slave) {
      int np = a.tri_npair[t];
      return np > 0 ? 3 + (a.kinematic ? 0 : 3 * np) : 0;
    }
    return 6 * (a.mp_off[t + 1] - a.mp_off[t]);
  };
  auto visit_src = [&](int src, auto &&visit) {
    int ent = slave ? a.s_vt[src] : a.m_vt[src];
    int t = ent >> 2, corner = ent & 3;
    if (slave) {
      if (a.tri_npair[t] == 0) return;
      const R *S = a.tri_sum + 9 * (int64_t)t;
      for (int b = 0; b < 3; ++b) visit(a.ts[3 * (int64_t)t + b], S[sym3(corner, b)], t);
      if (!a.kinematic) {
        int pb = a.tri_poff[t], np = a.tri_npair[t];
        for (int p = pb; p < pb + np; ++p) {
          const Pair<R> &P = a.pair[p];
          for (int m = 0; m < 3; ++m) visit((int32_t)(a.Vs + a.tm[3 * (int64_t)P.M + m]), P.sm[3 * corner + m], t);
        }
      }
    } else {
      for (int i = a.mp_off[t]; i < a.mp_off[t + 1]; ++i) {
        const Pair<R> &P = a.pair[a.mp_list[i]];
        for (int m = 0; m < 3; ++m)
          visit((int32_t)(a.Vs + a.tm[3 * (int64_t)t + m]), P.mm[sym3(corner, m)], P.T);
        for (int s = 0; s < 3; ++s) visit(a.ts[3 * (int64_t)P.T + s], P.sm[3 * s + corner], P.T);
      }
    }
  };

  int n_ent = 0;
  for (int src = sb + lane; src < se; src += kWave) n_ent += src_count(src);
  for (int o = 32; o > 0; o >>= 1) n_ent += __shfl_xor(n_ent, o, kWave);
  if (pass != 0 && a.grad) {
    // gradient row: slave a: sum_T -gs[T][a] n_T; master j: sum over the
    // pairs of its master triangles of gm[j] n_T (lane partials, fixed-order
    // butterfly)
    R gr[3] = {0, 0, 0};
    for (int src = sb + lane; src < se; src += kWave) {
      int ent = slave ? a.s_vt[src] : a.m_vt[src];
      int t = ent >> 2, corner = ent & 3;
      if (slave) {
        if (a.tri_npair[t] == 0) continue;
        R cf = -a.tri_sum[9 * (int64_t)t + 6 + corner];
        const R *nn = a.tri_nrm + 3 * (int64_t)t;
        for (int d = 0; d < 3; ++d) gr[d] += cf * nn[d];
      } else {
        for (int i = a.mp_off[t]; i < a.mp_off[t + 1]; ++i) {
          const Pair<R> &P = a.pair[a.mp_list[i]];
          const R *nn = a.tri_nrm + 3 * (int64_t)P.T;
          for (int d = 0; d < 3; ++d) gr[d] += P.gm[corner] * nn[d];
        }
      }
    }
    for (int d = 0; d < 3; ++d)
      for (int o = 32; o > 0; o >>= 1) gr[d] += __shfl_xor(gr[d], o, kWave);
    if (lane == 0)
      for (int d = 0; d < 3; ++d) a.grad[3 * row + d] = gr[d];
  }
  if (pass == 2) return;
  if (n_ent == 0) {
    if (pass == 0 && lane == 0) a.row_cnt[row] = 0;
    return;
  }
  int tsz = 64;
  while (tsz < 2 * n_ent && tsz < slots) tsz <<= 1;
  for (int i = lane; i < tsz; i += kWave) key[i] = -1;
  wave_sync();
  const bool stash = pass == 1 && n_ent <= kRowEnt;
  bool full = false;
  int run = 0;
  for (int s0 = sb; s0 < se; s0 += kWave) {
    const int src = s0 + lane;
    const int cnt = src < se ? src_count(src) : 0;
    int incl = cnt;
    for (int d = 1; d < kWave; d <<= 1) {
      int v = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += v;
    }
    int o = run + incl - cnt;
    if (src < se)
      visit_src(src, [&](int32_t col, R cf, int t) {
        if (row_slot(key, tsz, col, &full) < 0) return;
        if (stash) {
          ecol[o] = col;
          etri[o] = t;
          ecoef[o] = cf;
        }
        ++o;
      });
    run += __shfl(incl, kWave - 1, kWave);
  }
  if (__any(full)) {
    if (lane == 0) {
      atomicMax(&a.st->need_row, (unsigned long long)(2 * slots));
      atomicCAS(&a.st->code, 0, GMCP_E_CAPACITY);
      if (pass == 0) a.row_cnt[row] = 0;
    }
    return;
  }
  wave_sync();
  int nuniq = 0;
  for (int i0 = 0; i0 < tsz; i0 += kWave) {
    int i = i0 + lane;
    bool used = i < tsz && key[i] >= 0;
    uint64_t m = __ballot(used);
    if (used) dense[nuniq + __popcll(m & ((1ull << lane) - 1))] = key[i];
    nuniq += __popcll(m);
  }
  if (pass == 0) {
    if (lane == 0) a.row_cnt[row] = nuniq;
    return;
  }
  wave_sync();
  for (int u = lane; u < nuniq; u += kWave) {
    const int32_t c = dense[u];
    int r = 0;
    for (int m = 0; m < nuniq; ++m) r += dense[m] < c;
    R v[6] = {0, 0, 0, 0, 0, 0};
    auto add = [&](int32_t col, R cf, int t) {
      if (col != c) return;
      const R *nn = a.tri_nrm + 3 * (int64_t)t;
      v[0] += cf * nn[0] * nn[0];
      v[1] += cf * nn[0] * nn[1];
      v[2] += cf * nn[0] * nn[2];
      v[3] += cf * nn[1] * nn[1];
      v[4] += cf * nn[1] * nn[2];
      v[5] += cf * nn[2] * nn[2];
    };
    if (stash) {
      for (int e = 0; e < n_ent; ++e) add(ecol[e], ecoef[e], etri[e]);
    } else {
      for (int src = sb; src < se; ++src) visit_src(src, add);
    }
    const int64_t dst = (int64_t)a.row_ptr[row] + r;
    a.col[dst] = c;
    R *ov = a.val + 9 * dst;
    ov[0] = v[0]; ov[1] = v[1]; ov[2] = v[2];
    ov[3] = v[1]; ov[4] = v[3]; ov[5] = v[4];
    ov[6] = v[2]; ov[7] = v[4]; ov[8] = v[5];
  }
}


// gradient row by row: slave a: sum_T -gs[T][a] n_T; master j: sum over
// the pairs of its master triangles (sorted by slave triangle) gm[j] n_T
// MODE 0: gradient (tri_sum gs, Pair::gm); MODE 1: HVP (hv_tri, hv_pair)
template <typename R, int MODE>
__global__ __launch_bounds__(kThreads) void k_grad(RowArgs<R> a, const R *__restrict__ hv_tri,
                                                    const R *__restrict__ hv_pair, R *__restrict__ out) {
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= a.V) return;
  R g[3] = {0, 0, 0};
  if ((int64_t)a.st_r->n_pairs <= a.cap_pairs) {
    if (row < a.Vs) {
      for (int s = a.s_vt_off[row]; s < a.s_vt_off[row + 1]; ++s) {
        int ent = a.s_vt[s], t = ent >> 2, corner = ent & 3;
        if (a.tri_npair[t] == 0) continue;
        R cf = -(MODE == 0 ? a.tri_sum[9 * (int64_t)t + 6 + corner] : hv_tri[3 * (int64_t)t + corner]);
        const R *nn = a.tri_nrm + 3 * (int64_t)t;
        for (int d = 0; d < 3; ++d) g[d] += cf * nn[d];
      }
    } else {
      int64_t vid = row - a.Vs;
      for (int s = a.m_vt_off[vid]; s < a.m_vt_off[vid + 1]; ++s) {
        int ent = a.m_vt[s], t = ent >> 2, corner = ent & 3;
        for (int i = a.mp_off[t]; i < a.mp_off[t + 1]; ++i) {
          int p = a.mp_list[i];
          R cf = MODE == 0 ? a.pair[p].gm[corner] : hv_pair[3 * (int64_t)p + corner];
          const R *nn = a.tri_nrm + 3 * (int64_t)a.pair[p].T;
          for (int d = 0; d < 3; ++d) g[d] += cf * nn[d];
        }
      }
    }
  }
  for (int d = 0; d < 3; ++d) out[3 * row + d] = g[d];
}

template <typename R>
__global__ void k_energy(const double *__restrict__ tile_E, const EnvInfo *__restrict__ env, R *energy) {
  __shared__ double part[256];
  int e = blockIdx.x;
  double s = 0.0;
  for (int t = env[e].tile0 + threadIdx.x; t < env[e].tile1; t += blockDim.x) s += tile_E[t];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) energy[e] = (R)part[0];
}

__global__ void k_finish_counts(const int32_t *row_ptr, int64_t V, DevStatus *st, int64_t cap_nnzb) {
  if (threadIdx.x || blockIdx.x) return;
  long long nnzb = row_ptr[V];
  st->nnzb = (unsigned long long)nnzb;
  if (nnzb > cap_nnzb) atomicCAS(&st->code, 0, GMCP_E_CAPACITY);
}

template <typename R>
__global__ void k_rest_area(const R *__restrict__ x, const int32_t *__restrict__ ts, int64_t Ts, R *area,
                            const int32_t *__restrict__ samp_off, const int32_t *__restrict__ s_env,
                            const EnvInfo *__restrict__ env, const double *__restrict__ rule, R *weights) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Ts) return;
  R p[3][3];
  for (int j = 0; j < 3; ++j)
    for (int d = 0; d < 3; ++d) p[j][d] = x[3 * (int64_t)ts[3 * t + j] + d];
  R e1[3], e2[3];
  for (int d = 0; d < 3; ++d) {
    e1[d] = p[1][d] - p[0][d];
    e2[d] = p[2][d] - p[0][d];
  }
  R c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  R A = R(0.5) * sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  area[t] = A;
  if (weights) {
    const EnvInfo &ev = env[s_env[t]];
    for (int q = 0; q < ev.nq; ++q)
      weights[samp_off[t] + q] = R(2) * A * (R)rule[((ev.rule_n - 1) * 16 + q) * 3 + 2];
  }
}

template <typename R>
__global__ void k_fill_r(R *p, R v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

template <typename R>
__global__ void k_export(const Rec<R> *__restrict__ rec, const DevStatus *st, int64_t cap_active, int32_t *M,
                         R *g, R *bm, R *c1, R *c2, R *p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t na = (int64_t)st->n_active;
  if (na > cap_active || i >= na) return;
  Rec<R> r = rec[i];
  if (M) M[r.k] = r.M;
  if (g) g[r.k] = r.g;
  if (bm) {
    bm[3 * (int64_t)r.k] = r.b0;
    bm[3 * (int64_t)r.k + 1] = r.b1;
    bm[3 * (int64_t)r.k + 2] = r.b2;
  }
  if (c1) c1[r.k] = r.c1;
  if (c2) c2[r.k] = r.c2;
  if (p) p[r.k] = r.p;
}

// HVP, step 1: per slave triangle, s_k = c2 (grad g_k . v_x + v_d[k]);
// out_d[k] = s_k; triangle sums s_k bs_a; pair sums s_k bm_j
template <typename R>
__global__ void k_hvp_tri(const Rec<R> *__restrict__ rec, const int32_t *__restrict__ tri_roff,
                          const int32_t *__restrict__ tri_rcnt, const int32_t *__restrict__ tri_npair,
                          const int32_t *__restrict__ tri_poff, const Pair<R> *__restrict__ pair,
                          const R *__restrict__ tri_nrm, const int32_t *__restrict__ ts,
                          const int32_t *__restrict__ tm, const int32_t *__restrict__ s_env,
                          const EnvInfo *__restrict__ env, const double *__restrict__ rule, int64_t Ts, int64_t Vs,
                          bool kinematic, const R *__restrict__ vx, const R *__restrict__ vd, R *__restrict__ od,
                          R *__restrict__ hv_tri, R *__restrict__ hv_pair, const DevStatus *st, int64_t cap_active,
                          int64_t cap_pairs) {
  int64_t T = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (T >= Ts) return;
  if ((int64_t)st->n_active > cap_active || (int64_t)st->n_pairs > cap_pairs) return;
  int rc = tri_rcnt[T];
  if (rc == 0) return;
  int rb = tri_roff[T];
  const R *nn = tri_nrm + 3 * T;
  const EnvInfo &ev = env[s_env[T]];
  R vs[3];
  for (int a = 0; a < 3; ++a) {
    const R *v = vx + 3 * (int64_t)ts[3 * T + a];
    vs[a] = nn[0] * v[0] + nn[1] * v[1] + nn[2] * v[2];
  }
  R ht[3] = {0, 0, 0};
  int pb = tri_poff[T], np = tri_npair[T];
  for (int p = pb; p < pb + np; ++p) {
    const Pair<R> &P = pair[p];
    R vm[3];
    for (int m = 0; m < 3; ++m) {
      if (kinematic) {
        vm[m] = 0;
        continue;
      }
      const R *v = vx + 3 * (Vs + tm[3 * (int64_t)P.M + m]);
      vm[m] = nn[0] * v[0] + nn[1] * v[1] + nn[2] * v[2];
    }
    R hp[3] = {0, 0, 0};
    for (int i = rb; i < rb + rc; ++i) {
      const Rec<R> &r = rec[i];
      if (r.M != P.M) continue;
      const double *rq = rule + ((ev.rule_n - 1) * 16 + r.q) * 3;
      R bs[3] = {R(1) - (R)rq[0] - (R)rq[1], (R)rq[0], (R)rq[1]};
      R bm[3] = {r.b0, r.b1, r.b2};
      R dot = -(bs[0] * vs[0] + bs[1] * vs[1] + bs[2] * vs[2]) + bm[0] * vm[0] + bm[1] * vm[1] + bm[2] * vm[2];
      if (vd) dot += vd[r.k];
      R s = r.c2 * dot;
      if (od) od[r.k] = s;
      for (int q = 0; q < 3; ++q) {
        ht[q] += s * bs[q];
        hp[q] += s * bm[q];
      }
    }
    for (int q = 0; q < 3; ++q) hv_pair[3 * (int64_t)p + q] = hp[q];
  }
  for (int q = 0; q < 3; ++q) hv_tri[3 * T + q] = ht[q];
}

inline unsigned nblk(int64_t n, int t = kThreads) { return (unsigned)((n + t - 1) / t); }

template <typename R>
RowArgs<R> row_args(gmcp_ctx *c, const gmcp_bsr *H) {
  Buffers &b = c->b;
  RowArgs<R> ra;
  ra.ts = c->ts;
  ra.tm = c->tm;
  ra.Vs = c->Vs;
  ra.V = c->V;
  ra.kinematic = c->kinematic;
  ra.s_vt_off = b.s_vt_off;
  ra.s_vt = b.s_vt;
  ra.m_vt_off = b.m_vt_off;
  ra.m_vt = b.m_vt;
  ra.tri_npair = b.tri_npair;
  ra.tri_poff = b.tri_poff;
  ra.tri_sum = (const R *)b.tri_sum;
  ra.tri_nrm = (const R *)b.tri_nrm;
  ra.pair = (const Pair<R> *)b.pair;
  ra.mp_off = b.mp_off;
  ra.mp_list = b.mp_list;
  ra.st_r = b.status;
  ra.st = b.status;
  ra.cap_pairs = c->caps.pairs;
  ra.row_cnt = b.row_cnt;
  ra.row_ptr = H ? H->row_ptr : nullptr;
  ra.col = H ? H->col : nullptr;
  ra.val = H ? (R *)H->val : nullptr;
  ra.cap_nnzb = H ? H->cap_nnzb : 0;
  ra.grad = nullptr;
  return ra;
}

}  // namespace

template <typename R>
hipError_t launch_rest_area(gmcp_ctx *c, const R *x_rest, R *weights) {
  if (!c->Ts) return hipSuccess;
  hipLaunchKernelGGL(k_rest_area<R>, dim3(nblk(c->Ts)), dim3(kThreads), 0, c->stream, x_rest, c->ts, c->Ts,
                     (R *)c->b.area, c->b.samp_off, c->b.s_env, c->b.env, c->b.rule, weights);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_assemble(gmcp_ctx *c, const R *xs, const R *xm, const R *g_ref, const R *dgap, R *energy,
                           R *grad, const gmcp_bsr *H) {
  Buffers &b = c->b;
  hipStream_t s = c->stream;
  hipError_t e = reset_status(c, 2);
  if (e != hipSuccess) return e;
  NarrowArgs<R> na;
  na.xs = xs;
  na.xm = xm;
  na.ts = c->ts;
  na.tm = c->tm;
  na.tiles = b.tiles;
  na.n_tiles = (int)c->n_tiles;
  na.s_order = b.s_order;
  na.samp_off = b.samp_off;
  na.env = b.env;
  na.rule = b.rule;
  na.area = (const R *)b.area;
  na.cand_off = b.cand_off;
  na.cand = b.cand;
  na.Ts = c->Ts;
  na.cap_cand = c->caps.candidates;
  na.g_ref = g_ref;
  na.dgap = dgap;
  na.rec = (Rec<R> *)b.rec;
  na.cap_active = c->caps.active;
  na.tri_nrm = (R *)b.tri_nrm;
  na.tri_sum = (R *)b.tri_sum;
  na.tri_npair = b.tri_npair;
  na.tri_poff = b.tri_poff;
  na.tri_roff = b.tri_roff;
  na.tri_rcnt = b.tri_rcnt;
  na.pair = (Pair<R> *)b.pair;
  na.cap_pairs = c->caps.pairs;
  na.tile_E = b.tile_E;
  na.st = b.status;
  prof_mark(c, ST_NARROW, 0);
  if (c->n_tiles)
    hipLaunchKernelGGL(k_narrow<R>, dim3(nblk(c->n_tiles, kTilePerBlock)), dim3(kThreads), 0, s, na);
  prof_mark(c, ST_NARROW, 1);
  hipLaunchKernelGGL(k_energy<R>, dim3(c->n_env), dim3(256), 0, s, b.tile_E, b.env, energy);
  // bucket pairs by master triangle (needed for master rows and the HVP)
  const Pair<R> *pr = (const Pair<R> *)b.pair;
  unsigned pb = nblk(c->caps.pairs);
  prof_mark(c, ST_BUCKET, 0);
  hipLaunchKernelGGL(k_pair_bucket<R>, dim3(pb), dim3(kThreads), 0, s, pr, b.status, c->caps.pairs, b.mp_cnt,
                     b.mp_off, b.mp_key, 0);
  e = scan_exclusive(c, b.mp_cnt, b.mp_off, c->Tm + 1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pair_bucket<R>, dim3(pb), dim3(kThreads), 0, s, pr, b.status, c->caps.pairs, b.mp_cnt,
                     b.mp_off, b.mp_key, 1);
  hipLaunchKernelGGL(k_bucket_rank<R>, dim3(pb), dim3(kThreads), 0, s, pr, b.mp_off, b.mp_key, b.mp_list, b.status,
                     c->caps.pairs);
  prof_mark(c, ST_BUCKET, 1);
  RowArgs<R> ra = row_args<R>(c, H);
  ra.grad = grad;
  if (grad && !H) {  // gradient alone: the row kernel's gradient-only pass
    prof_mark(c, ST_GRAD, 0);
    hipLaunchKernelGGL((k_rows<R, 2>), dim3((unsigned)((c->V + kRowWaves - 1) / kRowWaves)), dim3(kWave * kRowWaves),
                       0, s, ra, 64);
    prof_mark(c, ST_GRAD, 1);
  }
  if (H) {
    // per wave: distinct-column set and list (8 B per slot, <= 1024 slots),
    // plus the row's contributions in the writing pass (<= kRowEnt)
    int slots = 64;
    while (slots < c->caps.row_entries && slots < 1024) slots <<= 1;
    const int nw = kRowWaves;
    unsigned rb = (unsigned)((c->V + nw - 1) / nw);
    size_t lds0 = (size_t)nw * slots * 8, lds1 = (size_t)nw * ((size_t)slots * 8 + (size_t)kRowEnt * (8 + sizeof(R)));
    e = fill_i32(c, b.row_cnt + c->V, 0, 1);
    if (e != hipSuccess) return e;
    prof_mark(c, ST_ROWS_COUNT, 0);
    hipLaunchKernelGGL((k_rows<R, 0>), dim3(rb), dim3(kWave * nw), lds0, s, ra, slots);
    prof_mark(c, ST_ROWS_COUNT, 1);
    e = scan_exclusive(c, b.row_cnt, H->row_ptr, c->V + 1);
    if (e != hipSuccess) return e;
    prof_mark(c, ST_ROWS_FILL, 0);
    hipLaunchKernelGGL((k_rows<R, 1>), dim3(rb), dim3(kWave * nw), lds1, s, ra, slots);
    prof_mark(c, ST_ROWS_FILL, 1);
    hipLaunchKernelGGL(k_finish_counts, dim3(1), dim3(64), 0, s, H->row_ptr, c->V, b.status, H->cap_nnzb);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_hvp(gmcp_ctx *c, const R *vx, const R *vd, R *ox, R *od) {
  Buffers &b = c->b;
  hipStream_t s = c->stream;
  if (od) hipLaunchKernelGGL(k_fill_r<R>, dim3(nblk(c->Ns) > 4096 ? 4096 : nblk(c->Ns)), dim3(kThreads), 0, s, od,
                             R(0), c->Ns);
  if (c->Ts)
    hipLaunchKernelGGL(k_hvp_tri<R>, dim3(nblk(c->Ts)), dim3(kThreads), 0, s, (const Rec<R> *)b.rec, b.tri_roff,
                       b.tri_rcnt, b.tri_npair, b.tri_poff, (const Pair<R> *)b.pair, (const R *)b.tri_nrm, c->ts,
                       c->tm, b.s_env, b.env, b.rule, c->Ts, c->Vs, c->kinematic, vx, vd, od, (R *)b.hv_tri,
                       (R *)b.hv_pair, b.status, c->caps.active, c->caps.pairs);
  RowArgs<R> ra = row_args<R>(c, nullptr);
  hipLaunchKernelGGL((k_grad<R, 1>), dim3(nblk(c->V)), dim3(kThreads), 0, s, ra, (const R *)b.hv_tri,
                     (const R *)b.hv_pair, ox);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_sample_results(gmcp_ctx *c, int32_t *M, R *g, R *bm, R *c1, R *c2, R *p) {
  hipStream_t s = c->stream;
  unsigned nb = nblk(c->Ns) > 4096 ? 4096 : nblk(c->Ns);
  if (!c->Ns) return hipSuccess;
  if (M && fill_i32(c, M, -1, c->Ns) != hipSuccess) return hipGetLastError();
  if (g) hipLaunchKernelGGL(k_fill_r<R>, dim3(nb), dim3(kThreads), 0, s, g, R(0), c->Ns);
  if (bm) hipLaunchKernelGGL(k_fill_r<R>, dim3(nb), dim3(kThreads), 0, s, bm, R(0), 3 * c->Ns);
  if (c1) hipLaunchKernelGGL(k_fill_r<R>, dim3(nb), dim3(kThreads), 0, s, c1, R(0), c->Ns);
  if (c2) hipLaunchKernelGGL(k_fill_r<R>, dim3(nb), dim3(kThreads), 0, s, c2, R(0), c->Ns);
  if (p) hipLaunchKernelGGL(k_fill_r<R>, dim3(nb), dim3(kThreads), 0, s, p, R(0), c->Ns);
  hipLaunchKernelGGL(k_export<R>, dim3(nblk(c->caps.active)), dim3(kThreads), 0, s, (const Rec<R> *)c->b.rec,
                     c->b.status, c->caps.active, M, g, bm, c1, c2, p);
  return hipGetLastError();
}

#define GMCP_INST(R)                                                                                            \
  template hipError_t launch_rest_area<R>(gmcp_ctx *, const R *, R *);                                          \
  template hipError_t launch_assemble<R>(gmcp_ctx *, const R *, const R *, const R *, const R *, R *, R *,      \
                                         const gmcp_bsr *);                                                     \
  template hipError_t launch_hvp<R>(gmcp_ctx *, const R *, const R *, R *, R *);                                \
  template hipError_t launch_sample_results<R>(gmcp_ctx *, int32_t *, R *, R *, R *, R *, R *);
GMCP_INST(float)
GMCP_INST(double)

}  // namespace gmcp
