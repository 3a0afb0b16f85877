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
  R s1, s2;  // the rule point (slave barycentrics 1 - s1 - s2, s1, s2)
};

template <typename R> union NarrowSlot {
  CandL<R> c;
  SampL<R> s;
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
  const int32_t *cand_cnt, *cand_pos, *cand;  // per slave triangle: list length and offset in cand
  int64_t Ts, cap_cand;
  const R *g_ref, *dgap;
  Rec<R> *rec;
  int64_t cap_active;
  R *tri_nrm, *tri_sum;
  int32_t *tri_npair, *tri_poff, *tri_roff, *tri_rcnt;
  Pair<R> *pair;
  int64_t cap_pairs;
  int32_t *mp_cnt;  // pairs per master triangle (counted where the pairs are written)
  int32_t *atile, *atile_cnt;  // tiles with selected samples (read by the linearised step bound)
  const uint32_t *tile_act, *epoch;  // nullable: tiles the last broad phase listed (others have no candidates)
  double *tile_E;
  DevStatus *st;
  bool features;                                   // clipped samples: edge and point samples too
  const int32_t *m_opp, *m_vt_off, *m_vt;          // master edge neighbours, vertex adjacency
};

// Narrow phase: one wave per work tile, kNarrowWaves tiles per block.  The
// records and pairs of a block are allocated together (wave counts in LDS,
// one pair of atomics per block), so every wave of a block passes through
// that allocation exactly once, whatever its tile holds.
template <typename R> constexpr int narrow_waves() { return sizeof(R) == 4 ? 8 : 4; }

template <typename R>
__device__ __forceinline__ void narrow_body(const NarrowArgs<R> &a) {
  constexpr int kNW = narrow_waves<R>();
  // a wave's staged candidates and, once its candidate loop is done, its
  // sample records share one LDS slot per lane (more resident blocks)
  __shared__ NarrowSlot<R> nl[kNW][kWave];
  __shared__ unsigned int alloc_r[kNW], alloc_p[kNW], alloc_t[kNW];
  __shared__ unsigned long long alloc_rb, alloc_pb;
  __shared__ int alloc_tb;
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  // the block's allocation: every wave calls it once (two block barriers);
  // a wave with records also takes a slot of the active-tile list
  int tslot = -1;
  auto allocate = [&](int nrec, int npair, unsigned long long &rb, unsigned long long &pb) {
    if (lane == 0) {
      alloc_r[w] = (unsigned)nrec;
      alloc_p[w] = (unsigned)npair;
      alloc_t[w] = nrec > 0 ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long tr = 0, tp = 0;
      unsigned tt = 0;
      for (int i = 0; i < kNW; ++i) {
        const unsigned r0 = alloc_r[i], p0 = alloc_p[i], t0 = alloc_t[i];
        alloc_r[i] = (unsigned)tr;
        alloc_p[i] = (unsigned)tp;
        alloc_t[i] = tt;
        tr += r0;
        tp += p0;
        tt += t0;
      }
      alloc_rb = tr ? atomicAdd(&a.st->n_active, tr) : 0;
      alloc_pb = tp ? atomicAdd(&a.st->n_pairs, tp) : 0;
      alloc_tb = (tt && a.atile) ? atomicAdd(a.atile_cnt, (int)tt) : 0;
    }
    __syncthreads();
    rb = alloc_rb + alloc_r[w];
    pb = alloc_pb + alloc_p[w];
    if (nrec > 0) tslot = alloc_tb + (int)alloc_t[w];
  };
  const int tile_id = xcd_block(blockIdx.x, gridDim.x) * kNW + w;
  if (tile_id >= a.n_tiles) {
    unsigned long long rb, pb;
    allocate(0, 0, rb, pb);
    return;
  }
  // a tile none of whose triangles the broad phase listed has no candidates
  // (the broad phase emptied their per-triangle outputs): one load decides
  if (a.tile_act && a.tile_act[tile_id] != *a.epoch) {
    if (lane == 0) a.tile_E[tile_id] = 0.0;
    unsigned long long rb, pb;
    allocate(0, 0, rb, pb);
    return;
  }
  const Tile tl = a.tiles[tile_id];
  const EnvInfo &ev = a.env[tl.env];
  const int nq = tl.nq;
  const int j = lane / nq, q = lane - j * nq;
  const bool valid = j < tl.count;
  const int T = valid ? a.s_order[tl.first + j] : 0;
  const R dhat = (R)ev.dhat, kappa = (R)ev.kappa, deltaT = (R)ev.delta_T;

  // ---- a tile without candidates selects nothing: empty bookkeeping only
  // (the broad phase has already checked its triangles' frames)
  {
    int cn = valid ? a.cand_cnt[T] : 0;
    for (int o = 32; o > 0; o >>= 1) cn = max(cn, __shfl_xor(cn, o, kWave));
    if (cn == 0) {
      if (valid && q == 0) {
        a.tri_npair[T] = 0;
        a.tri_rcnt[T] = 0;
        a.tri_poff[T] = 0;
        a.tri_roff[T] = 0;
      }
      if (lane == 0) a.tile_E[tile_id] = 0.0;
      unsigned long long rb, pb;
      allocate(0, 0, rb, pb);
      return;
    }
  }

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

  const int ccnt = (valid && !degen) ? a.cand_cnt[T] : 0;
  const int cbeg = ccnt > 0 ? a.cand_pos[T] : 0;
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
    nl[w][lane].c = cl;
    wave_sync();
    int nc = min(nq, ccnt - base);
    for (int c = 0; c < nc; ++c) {
      const CandL<R> &e = nl[w][j * nq + c].c;
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
  R g = 0, c1 = 0, c2 = 0, pr = 0, kw = 0;
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
      kw = kappa * wk * gam;
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
  me.s1 = xi;
  me.s2 = eta;
  nl[w][lane].s = me;
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
        const SampL<R> &o = nl[w][j * nq + i].s;
        if (o.M < 0) continue;
        R bs[3] = {R(1) - o.s1 - o.s2, o.s1, o.s2};
        acc += ib >= 0 ? o.c2 * bs[ia] * bs[ib] : o.c1 * bs[ia];
      }
      a.tri_sum[9 * (int64_t)T + v] = acc;
    }
    if (q == 0)
      for (int d = 0; d < 3; ++d) a.tri_nrm[3 * (int64_t)T + d] = n[d];
  }

  // ---- contact pairs: one per distinct master triangle of a slave triangle
  bool leader = false;
  int rank = 0;
  if (sel) {
    leader = true;
    for (int i = 0; i < q; ++i)
      if (nl[w][j * nq + i].s.M == bM) {
        leader = false;
        break;
      }
  }
  const uint64_t leadmask = __ballot(leader);
  if (leader) {
    for (int i = 0; i < nq; ++i) {
      const SampL<R> &o = nl[w][j * nq + i].s;
      if (((leadmask >> (j * nq + i)) & 1) && o.M < bM) ++rank;
    }
  }
  const int npair_w = __popcll(leadmask);

  // ---- records and pairs: wave prefixes, one block allocation
  const int nsel = __popcll(selmask);
  const int rpre = __popcll(selmask & ((one << lane) - 1));
  unsigned long long rbase, pbase;
  allocate(nsel, npair_w, rbase, pbase);
  const bool rec_ok = rbase + nsel <= (unsigned long long)a.cap_active;
  if (nsel && !rec_ok && lane == 0) atomicCAS(&a.st->code, 0, GMCP_E_CAPACITY);
  if (lane == 0 && tslot >= 0 && a.atile) a.atile[tslot] = tile_id;
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
    r.eps = eps;
    r.s1 = xi;
    r.s2 = eta;
    r.kwg = kw;
    r.pad = 0;
    a.rec[rbase + rpre] = r;
  }

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
    for (int m = 0; m < 3; ++m) p.mv[m] = a.tm[3 * (int64_t)bM + m];
    for (int z = 0; z < 6; ++z) p.mm[z] = 0;
    for (int z = 0; z < 9; ++z) p.sm[z] = 0;
    for (int z = 0; z < 3; ++z) p.gm[z] = 0;
    for (int i = 0; i < nq; ++i) {
      const SampL<R> &o = nl[w][j * nq + i].s;
      if (o.M != bM) continue;
      R bs[3] = {R(1) - o.s1 - o.s2, o.s1, o.s2};
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
    atomicAdd(&a.mp_cnt[bM], 1);
  }
}

// float: six waves per SIMD (80 registers), three blocks of 8 waves per CU
__global__ __launch_bounds__(kWave * 8) __attribute__((amdgpu_waves_per_eu(6))) void k_narrow_f32(
    NarrowArgs<float> a) {
  narrow_body<float>(a);
}
__global__ __launch_bounds__(kWave * 4) void k_narrow_f64(NarrowArgs<double> a) { narrow_body<double>(a); }

// ----------------------------------------------------------- mortar samples
// Clipped mortar face samples (Sec. 4.1, face samples): for a slave
// triangle T and an opposing candidate master triangle M, M is projected
// along n_T onto T's plane, expressed in T's barycentric pair (u, v) (T is
// the reference triangle u, v >= 0, u + v <= 1), clipped by T
// (Sutherland-Hodgman in LDS, at most 6 vertices), fan-triangulated from
// its first vertex, and every sub-triangle carries the n x n rule.  Sample:
// beta^s = (1 - u - v, u, v), beta^m = barycentric coordinates of the point
// in the projected master triangle, gap g = sum_j beta^m_j h_j with h_j the
// master vertices' heights above T's plane (= n_T . (x_m - x_s), Eq. (gap)),
// weight w = 2 A_sub W_q with A_sub the sub-triangle's share of T's rest
// area.  One wave per work tile, the tile's triangles in turn, candidate
// pairs in chunks of 64: a lane projects and clips one pair, then the
// chunk's (pair, sub-triangle, rule point) items are spread over the lanes.
// A counting pass sizes the triangle's records and pairs (one allocation,
// so they stay contiguous and in candidate order), a writing pass
// recomputes and writes them.  Per triangle and per pair sums, energy:
// fixed lane orders, segmented scans and butterflies.
constexpr int kMortarChunks = 8;  // candidates per slave triangle <= 512 (the broad phase's set)

template <typename R>
struct MortarPair {   // one (T, M) pair, projected into T's (u, v) coordinates
  R q[3][2];          // projected master vertices
  R h[3];             // master vertex heights above T's plane
  R qi[2][2];         // inverse of [q1 - q0, q2 - q0]
  R len[3];           // master edge lengths, edge k = (vertex k, vertex k+1)
  bool opposing;      // n_T . N_M < 0 (q, h, len are set)
  bool ok;            // face overlap possible (opposing, in the band, not edge-on)
};

template <typename R>
__device__ inline MortarPair<R> mortar_pair(const NarrowArgs<R> &a, int M, const R s0[3], const R e1[3],
                                            const R e2[3], const R n[3], R gi11, R gi12, R gi22, R eps) {
  MortarPair<R> P;
  P.ok = false;
  P.opposing = false;
  R p[3][3];
  for (int j = 0; j < 3; ++j) {
    const int64_t v = a.tm[3 * (int64_t)M + j];
    for (int d = 0; d < 3; ++d) p[j][d] = a.xm[3 * v + d] - s0[d];
  }
  R f1[3], f2[3];
  for (int d = 0; d < 3; ++d) {
    f1[d] = p[1][d] - p[0][d];
    f2[d] = p[2][d] - p[0][d];
  }
  const R N[3] = {f1[1] * f2[2] - f1[2] * f2[1], f1[2] * f2[0] - f1[0] * f2[2], f1[0] * f2[1] - f1[1] * f2[0]};
  if (!(n[0] * N[0] + n[1] * N[1] + n[2] * N[2] < R(0))) return P;  // not opposing
  P.opposing = true;
  for (int k = 0; k < 3; ++k) {
    const int k1 = k == 2 ? 0 : k + 1;
    const R dx = p[k1][0] - p[k][0], dy = p[k1][1] - p[k][1], dz = p[k1][2] - p[k][2];
    P.len[k] = sqrt(dx * dx + dy * dy + dz * dz);
  }
  R hmin = INFINITY, hmax = -INFINITY;
  for (int j = 0; j < 3; ++j) {
    P.h[j] = n[0] * p[j][0] + n[1] * p[j][1] + n[2] * p[j][2];
    hmin = fmin(hmin, P.h[j]);
    hmax = fmax(hmax, P.h[j]);
    const R r1 = p[j][0] * e1[0] + p[j][1] * e1[1] + p[j][2] * e1[2];
    const R r2 = p[j][0] * e2[0] + p[j][1] * e2[1] + p[j][2] * e2[2];
    P.q[j][0] = gi11 * r1 + gi12 * r2;
    P.q[j][1] = gi12 * r1 + gi22 * r2;
  }
  if (!(hmin < eps && hmax > -eps)) return P;  // every gap beyond the support band
  const R a00 = P.q[1][0] - P.q[0][0], a01 = P.q[2][0] - P.q[0][0];
  const R a10 = P.q[1][1] - P.q[0][1], a11 = P.q[2][1] - P.q[0][1];
  const R det = a00 * a11 - a01 * a10;
  if (!(fabs(det) > R(1e-14))) return P;  // master edge-on to the slave plane
  const R id = R(1) / det;
  P.qi[0][0] = a11 * id;
  P.qi[0][1] = -a01 * id;
  P.qi[1][0] = -a10 * id;
  P.qi[1][1] = a00 * id;
  P.ok = true;
  return P;
}

// Sutherland-Hodgman clip of the projected master triangle by the reference
// triangle (at most 6 vertices); the polygon lives in LDS (lane-minor),
// returns its vertex count
template <typename R>
__device__ inline int mortar_clip(const MortarPair<R> &P, R (*buf)[6][2][kWave], int lane) {
  int cnt = 3;
  for (int j = 0; j < 3; ++j) {
    buf[0][j][0][lane] = P.q[j][0];
    buf[0][j][1][lane] = P.q[j][1];
  }
  int src = 0;
  for (int plane = 0; plane < 3; ++plane) {
    int out = 0;
    const int dst = src ^ 1;
    for (int i = 0; i < cnt; ++i) {
      const int i1 = i + 1 == cnt ? 0 : i + 1;
      const R pu = buf[src][i][0][lane], pv = buf[src][i][1][lane];
      const R qu = buf[src][i1][0][lane], qv = buf[src][i1][1][lane];
      const R fp = plane == 0 ? pu : (plane == 1 ? pv : R(1) - pu - pv);
      const R fq = plane == 0 ? qu : (plane == 1 ? qv : R(1) - qu - qv);
      // a convex polygon gains at most one vertex per half-plane (6 in
      // all); the cap only guards rounding-made non-convex inputs
      if (fp >= R(0)) {
        if (out < 6) {
          buf[dst][out][0][lane] = pu;
          buf[dst][out][1][lane] = pv;
          ++out;
        }
        if (fq < R(0) && out < 6) {
          const R t = fp / (fp - fq);
          buf[dst][out][0][lane] = pu + (qu - pu) * t;
          buf[dst][out][1][lane] = pv + (qv - pv) * t;
          ++out;
        }
      } else if (fq >= R(0) && out < 6) {
        const R t = fp / (fp - fq);
        buf[dst][out][0][lane] = pu + (qu - pu) * t;
        buf[dst][out][1][lane] = pv + (qv - pv) * t;
        ++out;
      }
    }
    cnt = out;
    src = dst;
    if (cnt == 0) break;
  }
  if (src != 0)  // leave the result in buffer 0
    for (int i = 0; i < cnt; ++i) {
      buf[0][i][0][lane] = buf[1][i][0][lane];
      buf[0][i][1][lane] = buf[1][i][1][lane];
    }
  return cnt;
}

// parameter interval [t0, t1] of qa + t (qb - qa), t in [0, 1], inside the
// reference triangle (Liang-Barsky); false if empty
template <typename R>
__device__ inline bool clip_seg(const R qa[2], const R qb[2], R &t0, R &t1) {
  t0 = R(0);
  t1 = R(1);
  for (int f = 0; f < 3; ++f) {
    const R fa = f == 0 ? qa[0] : (f == 1 ? qa[1] : R(1) - qa[0] - qa[1]);
    const R fb = f == 0 ? qb[0] : (f == 1 ? qb[1] : R(1) - qb[0] - qb[1]);
    const R d = fb - fa;
    if (d == R(0)) {
      if (fa < R(0)) return false;
      continue;
    }
    const R t = -fa / d;
    if (d > R(0)) t0 = fmax(t0, t);
    else t1 = fmin(t1, t);
  }
  return t1 > t0;
}

template <typename R>
__device__ __forceinline__ void mortar_body(const NarrowArgs<R> &a) {
  __shared__ R poly[2][6][2][kWave];                   // clip buffers (lane-minor); see fr below
  __shared__ uint64_t maskbuf[kMortarChunks][kWave];   // accepted face samples of each lane's pair
  __shared__ uint32_t fmaskbuf[kMortarChunks][kWave];  // accepted edge (bit 4k + j) / point (bit 12 + k) samples
  __shared__ uint8_t oflag[kMortarChunks * kWave];     // candidate i of the triangle is opposing
  __shared__ uint64_t accw[kWave];                     // accepted face items of a chunk, 64 per word
  __shared__ int32_t istart[kWave + 1];                // first face item of each candidate lane of a chunk
  __shared__ int32_t rstart[kWave];                    // first record of each candidate lane (from the triangle's)
  __shared__ int32_t candM[kWave];                     // master triangle of each candidate lane
  __shared__ R pacc[18][kWave];                        // each candidate lane's pair sums (mm 6, sm 9, gm 3)
  const int lane = threadIdx.x;
  const int tile_id = xcd_block(blockIdx.x, gridDim.x);
  if (tile_id >= a.n_tiles) return;
  const Tile tl = a.tiles[tile_id];
  const EnvInfo &ev = a.env[tl.env];
  const R dhat = (R)ev.dhat, kappa = (R)ev.kappa, deltaT = (R)ev.delta_T;
  const R kappa_e = (R)ev.kappa_e, kappa_p = (R)ev.kappa_p, delta_e = (R)ev.delta_e;
  const int nq = ev.nq, ng = ev.rule_n;
  const double *rule = a.rule + (ev.rule_n - 1) * 16 * 3;
  const double *gl = a.rule + kGaussOff + (ev.rule_n - 1) * 4 * 2;
  const bool features = a.features;
  R(*buf)[6][2][kWave] = poly;
  // once a lane's clip is done its column of buffer 1 is free: it holds the
  // pair's frame there, fr[z][lane] = q0 (2), qi (4), h (3)
  R(*fr)[kWave] = reinterpret_cast<R(*)[kWave]>(&poly[1][0][0][0]);
  double E = 0.0;
  const uint64_t below = (1ull << lane) - 1;
  for (int j = 0; j < tl.count; ++j) {
    const int T = a.s_order[tl.first + j];
    const int cn = a.cand_cnt[T], cb = cn > 0 ? a.cand_pos[T] : 0;
    // support radius of the triangle's samples, Eq. (adaptive_eps): in this
    // mode the reference gaps are one per slave triangle
    const R eps = a.g_ref ? fmin(R(0.9) * a.g_ref[T], dhat) : dhat;
    // slave frame
    R s0[3], e1[3], e2[3], n[3];
    {
      const int64_t v0 = a.ts[3 * (int64_t)T], v1 = a.ts[3 * (int64_t)T + 1], v2 = a.ts[3 * (int64_t)T + 2];
      for (int d = 0; d < 3; ++d) {
        s0[d] = a.xs[3 * v0 + d];
        e1[d] = a.xs[3 * v1 + d] - s0[d];
        e2[d] = a.xs[3 * v2 + d] - s0[d];
      }
    }
    const R c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const R len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    const R g11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    const R g12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
    const R g22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    const bool good = cn > 0 && isfinite(len) && len > R(1e-14) * (g11 + g22);
    if (cn > 0 && !good && lane == 0)
      set_error(a.st, isfinite(len) ? GMCP_E_DEGENERATE : GMCP_E_NONFINITE, (unsigned long long)T);
    if (!good) {
      if (lane == 0) {
        a.tri_npair[T] = 0;
        a.tri_rcnt[T] = 0;
        a.tri_poff[T] = 0;
        a.tri_roff[T] = 0;
      }
      continue;
    }
    for (int d = 0; d < 3; ++d) n[d] = c[d] / len;
    const R gdet = g11 * g22 - g12 * g12;
    const R gi11 = g22 / gdet, gi12 = -g12 / gdet, gi22 = g11 / gdet;
    const R area = a.area[T];
    const int nchunk = (cn + kWave - 1) / kWave;
    auto pair_of = [&](int M) { return mortar_pair(a, M, s0, e1, e2, n, gi11, gi12, gi22, eps); };

    // ---- feature ownership: an edge or vertex belongs to the smallest-index
    // opposing candidate master triangle that contains it.  The counting
    // pass searches the triangle's candidate ids in LDS (the pair sums'
    // array, which only the writing pass uses)
    int32_t *cids = reinterpret_cast<int32_t *>(&pacc[0][0]);
    static_assert(sizeof(pacc) >= sizeof(int32_t) * kMortarChunks * kWave, "candidate ids fit the pair sums");
    if (features) {
      wave_sync();
      for (int ci = lane; ci < cn && ci < kMortarChunks * kWave; ci += kWave) {
        const int M = a.cand[cb + ci];
        cids[ci] = M;
        oflag[ci] = pair_of(M).opposing ? 1 : 0;
      }
      wave_sync();
    }
    auto cand_opposing = [&](int t) -> bool {
      int lo = 0, hi = cn < kMortarChunks * kWave ? cn : kMortarChunks * kWave;
      const int end = hi;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cids[mid] < t) lo = mid + 1;
        else hi = mid;
      }
      return lo < end && cids[lo] == t && oflag[lo];
    };
    auto owns_edge = [&](int M, int k) -> bool {
      const int o = a.m_opp[3 * (int64_t)M + k];
      return o < 0 || o > M || !cand_opposing(o);
    };
    auto owns_vertex = [&](int M, int k) -> bool {
      const int v = a.tm[3 * (int64_t)M + k];
      for (int i = a.m_vt_off[v]; i < a.m_vt_off[v + 1]; ++i) {  // incident triangles, ascending
        const int t = a.m_vt[i] >> 2;
        if (t == M) return true;
        if (cand_opposing(t)) return false;
      }
      return true;
    };
    // edge / point samples of an opposing pair: bit 4k + j (edge k, Gauss
    // point j), bit 12 + k (vertex k)
    auto feature_mask = [&](const MortarPair<R> &P, int M, bool &pen_) -> uint32_t {
      uint32_t fm = 0;
      for (int k = 0; k < 3; ++k) {
        const int k1 = k == 2 ? 0 : k + 1;
        if (!(fmin(P.h[k], P.h[k1]) < eps && fmax(P.h[k], P.h[k1]) > -eps)) continue;
        R t0, t1;
        if (!clip_seg(P.q[k], P.q[k1], t0, t1)) continue;
        if (!owns_edge(M, k)) continue;
        for (int jj = 0; jj < ng; ++jj) {
          const R eta = t0 + (t1 - t0) * (R)gl[2 * jj];
          const R g = (R(1) - eta) * P.h[k] + eta * P.h[k1];
          if (g > R(0) && g < eps) fm |= 1u << (4 * k + jj);
          else if (g > -eps && g <= R(0)) pen_ = true;
        }
      }
      for (int k = 0; k < 3; ++k) {
        const R h = P.h[k], u = P.q[k][0], v = P.q[k][1];
        if (!(h > -eps && h < eps) || !(u > R(0) && v > R(0) && R(1) - u - v > R(0))) continue;
        if (!owns_vertex(M, k)) continue;
        if (h > R(0)) fm |= 1u << (12 + k);
        else pen_ = true;
      }
      return fm;
    };

    // The face samples of a chunk (up to 64 candidate pairs) are spread
    // over the lanes: each candidate lane clips its pair (polygon in buffer
    // 0, frame in fr) and owns (m - 2) nq items (sub-triangle s, rule point
    // q; item index (s - 1) nq + q within the pair, the bit of its mask);
    // the items of all pairs, in candidate order, are taken 64 at a time,
    // the candidate of an item found by binary search in istart.  Returns
    // the chunk's item count.  Every lane calls.
    auto chunk_items = [&](const MortarPair<R> &P, bool clip) -> int {
      int m = 0;
      if (clip) {
        m = mortar_clip(P, buf, lane);
        fr[0][lane] = P.q[0][0];
        fr[1][lane] = P.q[0][1];
        fr[2][lane] = P.qi[0][0];
        fr[3][lane] = P.qi[0][1];
        fr[4][lane] = P.qi[1][0];
        fr[5][lane] = P.qi[1][1];
        fr[6][lane] = P.h[0];
        fr[7][lane] = P.h[1];
        fr[8][lane] = P.h[2];
      }
      const int ni = m >= 3 ? (m - 2) * nq : 0;
      int incl = ni;
      for (int d = 1; d < kWave; d <<= 1) {
        const int v = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += v;
      }
      istart[lane] = incl - ni;
      if (lane == kWave - 1) istart[kWave] = incl;
      wave_sync();
      return __shfl(incl, kWave - 1, kWave);
    };
    auto item_of = [&](int f, int &cl, int &s, int &qq) -> int {  // f < the chunk's item count
      int lo = 0, hi = kWave - 1;  // the last lane whose items start at or before f
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (istart[mid] <= f) lo = mid;
        else hi = mid - 1;
      }
      cl = lo;
      const int local = f - istart[lo];
      s = local / nq + 1;
      qq = local - (s - 1) * nq;
      return local;
    };
    // sub-triangle s of candidate lane cl's polygon at rule point qq: slave
    // point (u, v), master barycentrics b1, b2, gap, twice the sub-triangle's
    // (u, v) area; false if the sub-triangle is degenerate
    auto face = [&](int cl, int s, int qq, R &u, R &v, R &b1, R &b2, R &g, R &a2) -> bool {
      const int s1i = s < 5 ? s : 4, s2i = s + 1 < 6 ? s + 1 : 5;  // in-range LDS reads
      const R Au = buf[0][0][0][cl], Av = buf[0][0][1][cl];
      const R Bu = buf[0][s1i][0][cl] - Au, Bv = buf[0][s1i][1][cl] - Av;
      const R Cu = buf[0][s2i][0][cl] - Au, Cv = buf[0][s2i][1][cl] - Av;
      const R cr = Bu * Cv - Bv * Cu;
      if (cr == R(0)) return false;
      const R xi = (R)rule[3 * qq], eta = (R)rule[3 * qq + 1];
      u = Au + xi * Bu + eta * Cu;
      v = Av + xi * Bv + eta * Cv;
      const R yu = u - fr[0][cl], yv = v - fr[1][cl];
      b1 = fr[2][cl] * yu + fr[3][cl] * yv;
      b2 = fr[4][cl] * yu + fr[5][cl] * yv;
      g = (R(1) - b1 - b2) * fr[6][cl] + b1 * fr[7][cl] + b2 * fr[8][cl];
      a2 = fabs(cr);
      return true;
    };

    // ---- counting pass: accepted samples per candidate pair (bit masks)
    int nrec = 0, npair = 0;
    bool pen = false;
    for (int ch = 0; ch < nchunk && ch < kMortarChunks; ++ch) {
      const int ci = ch * kWave + lane;
      MortarPair<R> P;
      P.ok = false;
      P.opposing = false;
      int M = -1;
      uint32_t fmask = 0;
      if (ci < cn) {
        M = a.cand[cb + ci];
        P = pair_of(M);
        if (features && P.opposing) fmask = feature_mask(P, M, pen);
      }
      const int tot = chunk_items(P, P.ok);
      for (int f0 = 0; f0 < tot; f0 += kWave) {
        const int f = f0 + lane;
        bool acc = false;
        if (f < tot) {
          int cl, s, qq;
          item_of(f, cl, s, qq);
          R u, v, b1, b2, g, a2;
          if (face(cl, s, qq, u, v, b1, b2, g, a2)) {
            if (g > R(0) && g < eps) acc = true;
            else if (g > -eps && g <= R(0)) pen = true;
          }
        }
        const uint64_t am = __ballot(acc);
        if (lane == 0) accw[f0 / kWave] = am;
      }
      wave_sync();
      uint64_t mask = 0;  // this lane's pair: bits [istart, istart + ni) of the chunk's words
      {
        const int i0 = istart[lane], ni = istart[lane + 1] - i0;
        if (ni > 0) {
          const int w0 = i0 >> 6, sh = i0 & 63;
          mask = accw[w0] >> sh;
          if (sh > 0 && sh + ni > 64) mask |= accw[w0 + 1] << (64 - sh);
          if (ni < 64) mask &= (1ull << ni) - 1;
        }
      }
      maskbuf[ch][lane] = mask;
      fmaskbuf[ch][lane] = fmask;
      const int cntl = __popcll(mask) + __popc(fmask);
      const uint64_t pm = __ballot(cntl > 0);
      npair += __popcll(pm);
      int tot_r = cntl;
      for (int o = 32; o > 0; o >>= 1) tot_r += __shfl_xor(tot_r, o, kWave);
      nrec += tot_r;
      wave_sync();  // the chunk's polygons, frames and words are reused by the next
    }
    if (__any(pen) && lane == 0) set_error(a.st, GMCP_E_PENETRATION, (unsigned long long)T);
    if (nchunk > kMortarChunks && lane == 0) atomicCAS(&a.st->code, 0, GMCP_E_CAPACITY);
    unsigned long long rbase = 0, pbase = 0;
    if (lane == 0 && (nrec || npair)) {  // records and pairs in one atomic (k_mortar_counts unpacks the totals)
      const unsigned long long old =
          atomicAdd(&a.st->mortar_alloc, ((unsigned long long)npair << 32) | (unsigned long long)nrec);
      rbase = old & 0xffffffffull;
      pbase = old >> 32;
    }
    rbase = __shfl(rbase, 0, kWave);
    pbase = __shfl(pbase, 0, kWave);
    const bool rec_ok = rbase + nrec <= (unsigned long long)a.cap_active;
    const bool pair_ok = pbase + npair <= (unsigned long long)a.cap_pairs;
    if (lane == 0 && ((nrec && !rec_ok) || (npair && !pair_ok))) atomicCAS(&a.st->code, 0, GMCP_E_CAPACITY);
    // every allocated pair slot is written whenever the pairs fit (the
    // bucket kernels read all n_pairs slots); records only when they fit too
    const bool write_rec = rec_ok && pair_ok;
    if (lane == 0) {
      a.tri_npair[T] = pair_ok ? npair : 0;
      a.tri_poff[T] = (int32_t)pbase;
      a.tri_rcnt[T] = write_rec ? nrec : 0;
      a.tri_roff[T] = (int32_t)rbase;
    }
    if (nrec == 0 || !pair_ok) continue;

    // ---- writing pass: exactly the samples of the masks, so the records
    // written always fill the allocated range.  A pair's records are its
    // face samples in item order, then its edge / point samples.
    R ts_[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // c2 bs_a bs_b (00 01 02 11 12 22), c1 bs_a
    // one active sample: the record at r, the triangle sums and energy, and
    // the pair sums' terms pt (mm 6, sm 9, gm 3)
    auto term = [&](unsigned long long r, int M, R u, R v, const R bm[3], R graw, R kw, R kap, R gam, R pt[18]) {
      // the counting pass accepted 0 < g < eps; a recomputation that rounds
      // differently is clamped into the band
      const R g = fmin(fmax(graw, eps * R(1e-6)), eps);
      const R dd = g - eps;
      const R L = log1p_r<R>(dd / eps);
      const R B = -dd * dd * L;
      const R B1 = -R(2) * dd * L - dd * dd / g;
      const R B2 = -R(2) * L - R(4) * dd / g + dd * dd / (g * g);
      const R c1 = kw * B1, c2 = fmax(kw * B2, R(0));
      E += (double)(kw * B);
      const R bs[3] = {R(1) - u - v, u, v};
      ts_[0] += c2 * bs[0] * bs[0];
      ts_[1] += c2 * bs[0] * bs[1];
      ts_[2] += c2 * bs[0] * bs[2];
      ts_[3] += c2 * bs[1] * bs[1];
      ts_[4] += c2 * bs[1] * bs[2];
      ts_[5] += c2 * bs[2] * bs[2];
      for (int z = 0; z < 3; ++z) ts_[6 + z] += c1 * bs[z];
      pt[0] = c2 * bm[0] * bm[0];
      pt[1] = c2 * bm[0] * bm[1];
      pt[2] = c2 * bm[0] * bm[2];
      pt[3] = c2 * bm[1] * bm[1];
      pt[4] = c2 * bm[1] * bm[2];
      pt[5] = c2 * bm[2] * bm[2];
      for (int s2 = 0; s2 < 3; ++s2)
        for (int m2 = 0; m2 < 3; ++m2) pt[6 + 3 * s2 + m2] = -(c2 * bs[s2] * bm[m2]);
      for (int m2 = 0; m2 < 3; ++m2) pt[15 + m2] = c1 * bm[m2];
      if (write_rec) {
        Rec<R> rc;
        rc.k = -1;
        rc.M = M;
        rc.T = T;
        rc.q = -1;
        rc.g = g;
        rc.b0 = bm[0];
        rc.b1 = bm[1];
        rc.b2 = bm[2];
        rc.c1 = c1;
        rc.c2 = c2;
        rc.p = -kap * gam * B1;
        rc.eps = eps;
        rc.s1 = u;
        rc.s2 = v;
        rc.kwg = kw;
        rc.pad = 0;
        a.rec[r] = rc;
      }
    };
    unsigned long long roff = rbase, poff = pbase;
    for (int ch = 0; ch < nchunk && ch < kMortarChunks; ++ch) {
      const int ci = ch * kWave + lane;
      const uint64_t mask = maskbuf[ch][lane];
      const uint32_t fmask = fmaskbuf[ch][lane];
      const int cntl = __popcll(mask) + __popc(fmask);
      int incl = cntl;
      for (int d = 1; d < kWave; d <<= 1) {
        const int v = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += v;
      }
      const uint64_t pm = __ballot(cntl > 0);
      const unsigned long long r0 = roff + (unsigned long long)(incl - cntl);  // this pair's first record
      const unsigned long long pslot = poff + __popcll(pm & below);
      roff += __shfl(incl, kWave - 1, kWave);
      poff += __popcll(pm);
      int M = -1;
      MortarPair<R> P;
      P.ok = false;
      P.opposing = false;
      if (cntl > 0) {
        M = a.cand[cb + ci];
        if (mask) P = pair_of(M);
      }
      candM[lane] = M;
      rstart[lane] = (int32_t)(r0 - rbase);
      const int tot = chunk_items(P, mask != 0);  // pairs with face samples only
      // face samples over the lanes; each pair's sums are segmented scans
      // over the lanes of its items (items of a pair are contiguous), taken
      // by the pair's own lane from the last of them: fixed order
      for (int z = 0; z < 18; ++z) pacc[z][lane] = R(0);
      for (int f0 = 0; f0 < tot; f0 += kWave) {
        const int f = f0 + lane;
        int seg = kWave + lane;  // idle lanes: segments of their own
        R pt[18];
        for (int z = 0; z < 18; ++z) pt[z] = R(0);
        if (f < tot) {
          int cl, s, qq;
          const int local = item_of(f, cl, s, qq);
          seg = cl;
          const uint64_t cm = maskbuf[ch][cl];
          if ((cm >> local) & 1ull) {
            R u = 0, v = 0, b1 = 0, b2 = 0, g = 0, a2 = 0;  // a degenerate item (never accepted) weighs 0
            face(cl, s, qq, u, v, b1, b2, g, a2);
            const R bm[3] = {R(1) - b1 - b2, b1, b2};
            const R gam = deltaT > R(0) ? hermite(fmin(bm[0], fmin(bm[1], bm[2])), deltaT) : R(1);
            const R wq = (R)rule[3 * qq + 2];
            const unsigned long long r = rbase + (unsigned long long)rstart[cl] + __popcll(cm & ((1ull << local) - 1));
            term(r, candM[cl], u, v, bm, bm[0] * fr[6][cl] + bm[1] * fr[7][cl] + bm[2] * fr[8][cl],
                 kappa * R(2) * (a2 * area) * wq * gam, kappa, gam, pt);
          }
        }
        for (int d = 1; d < kWave; d <<= 1) {
          const int su = __shfl_up(seg, d, kWave);
          const bool take = lane >= d && su == seg;
          for (int z = 0; z < 18; ++z) {
            const R t = __shfl_up(pt[z], d, kWave);
            if (take) pt[z] += t;
          }
        }
        const int i0 = istart[lane], i1 = istart[lane + 1];
        const bool mine = i1 > i0 && i1 > f0 && i0 < f0 + kWave;
        const int src = mine ? min(i1, f0 + kWave) - 1 - f0 : lane;
        for (int z = 0; z < 18; ++z) {
          const R t = __shfl(pt[z], src, kWave);
          if (mine) pacc[z][lane] += t;
        }
      }
      if (cntl > 0) {
        Pair<R> pr;
        pr.T = T;
        pr.M = M;
        for (int m = 0; m < 3; ++m) pr.mv[m] = a.tm[3 * (int64_t)M + m];
        for (int z = 0; z < 6; ++z) pr.mm[z] = pacc[z][lane];
        for (int z = 0; z < 9; ++z) pr.sm[z] = pacc[6 + z][lane];
        for (int z = 0; z < 3; ++z) pr.gm[z] = pacc[15 + z][lane];
        if (fmask) {
          const MortarPair<R> Q = pair_of(M);
          unsigned long long r = r0 + __popcll(mask);
          for (uint32_t bits = fmask; bits; bits &= bits - 1) {
            const int idx = __ffs(bits) - 1;
            R bm[3] = {0, 0, 0}, pt[18];
            if (idx < 12) {  // edge k, Gauss point jj
              const int k = idx >> 2, jj = idx & 3, k1 = k == 2 ? 0 : k + 1;
              R t0, t1;
              clip_seg(Q.q[k], Q.q[k1], t0, t1);
              const R eta = t0 + (t1 - t0) * (R)gl[2 * jj];
              bm[k] = R(1) - eta;
              bm[k1] = eta;
              const R u = Q.q[k][0] + eta * (Q.q[k1][0] - Q.q[k][0]), v = Q.q[k][1] + eta * (Q.q[k1][1] - Q.q[k][1]);
              const R gam = delta_e > R(0) ? hermite(eta, delta_e) * hermite(R(1) - eta, delta_e) : R(1);
              const R w = Q.len[k] * (t1 - t0) * (R)gl[2 * jj + 1];
              term(r++, M, u, v, bm, (R(1) - eta) * Q.h[k] + eta * Q.h[k1], kappa_e * w * gam, kappa_e, gam, pt);
            } else {  // vertex k: one point sample, weight 1
              const int k = idx - 12;
              bm[k] = R(1);
              term(r++, M, Q.q[k][0], Q.q[k][1], bm, Q.h[k], kappa_p, kappa_p, R(1), pt);
            }
            for (int z = 0; z < 6; ++z) pr.mm[z] += pt[z];
            for (int z = 0; z < 9; ++z) pr.sm[z] += pt[6 + z];
            for (int z = 0; z < 3; ++z) pr.gm[z] += pt[15 + z];
          }
        }
        a.pair[pslot] = pr;
        atomicAdd(&a.mp_cnt[M], 1);
      }
      wave_sync();  // the chunk's polygons, frames and tables are reused by the next
    }
    for (int z = 0; z < 9; ++z)
      for (int o = 32; o > 0; o >>= 1) ts_[z] += __shfl_xor(ts_[z], o, kWave);
    if (lane == 0) {
      for (int z = 0; z < 9; ++z) a.tri_sum[9 * (int64_t)T + z] = ts_[z];
      for (int d = 0; d < 3; ++d) a.tri_nrm[3 * (int64_t)T + d] = n[d];
    }
  }
  for (int o = 32; o > 0; o >>= 1) E += __shfl_xor(E, o, kWave);
  if (lane == 0) a.tile_E[tile_id] = E;
}

__global__ __launch_bounds__(kWave) void k_mortar_f32(NarrowArgs<float> a) { mortar_body<float>(a); }
__global__ __launch_bounds__(kWave) void k_mortar_f64(NarrowArgs<double> a) { mortar_body<double>(a); }

// ---------------------------------------------------- pairs by master tri
// pass 0: count pairs per master triangle; pass 1: place (slave triangle,
// pair) keys into the buckets in arrival order (counters return to zero)
// the totals of the clipped-sample allocation into the status counters
__global__ void k_mortar_counts(DevStatus *st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const unsigned long long v = st->mortar_alloc;
    st->n_active = v & 0xffffffffull;
    st->n_pairs = v >> 32;
  }
}

// pairs into their master triangle's bucket (counts from the narrow phase,
// offsets from their scan); the counters return to zero.  When the pairs
// overflowed, the written ones were counted but are not placed: the
// counters are cleared instead.
template <typename R>
__global__ void k_pair_bucket(const Pair<R> *__restrict__ pair, const DevStatus *st, int64_t cap_pairs,
                              int32_t *__restrict__ mp_cnt, const int32_t *__restrict__ mp_off,
                              long long *__restrict__ mp_key, int64_t Tm) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t np = (int64_t)st->n_pairs;
  if (np > cap_pairs) {
    for (int64_t i = p; i <= Tm; i += (int64_t)gridDim.x * blockDim.x) mp_cnt[i] = 0;
    return;
  }
  if (p >= np) return;
  int M = pair[p].M;
  int slot = mp_off[M] + atomicSub(&mp_cnt[M], 1) - 1;
  mp_key[slot] = ((long long)pair[p].T << 32) | (long long)p;
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
  const long long *mp_key;   // bucket slots: slave triangle << 32 | pair
  const R *mtri;             // per-master-triangle blocks and gradient (k_mtri)
  const DevStatus *st_r;
  DevStatus *st;
  int64_t cap_pairs;
  int32_t *row_cnt;
  const int32_t *row_ptr;
  int32_t *col;
  R *val;
  int64_t cap_nnzb;
  R *grad;   // nullable: written by the writing pass (pass 1) or alone (pass 2)
  int light_bound;  // column insertions of a light row (32, 64, 128 or 256)
};

constexpr int kRowWaves = 2;
// the list-walking row kernels use fixed grids, by default many times the
// blocks resident at once (kDefaultRowBlocks light, kDefaultHeavyBlocks
// heavy): a block's share of the list is short, so blocks that start late
// (the device is shared with the other stream's kernels) finish soon after
// the rest

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

// Four lanes per master triangle with contact pairs: the sum over its pairs
// (bucket order: sorted by slave triangle) of the master-master sums times
// n_T n_T^T - six vertex pairs (00 01 02 11 12 22) of six symmetric entries -
// and of the gradient sums gm_j n_T (three vertices).  Lane s of the group
// sums the pairs s, s + 4, ... in order (their loads issued four at a time),
// and the four partials are combined by a fixed butterfly, so the result is
// the same on every run.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_mtri(const Pair<R> *__restrict__ pair,
                                                    const int32_t *__restrict__ mp_off,
                                                    const int32_t *__restrict__ mp_list,
                                                    const R *__restrict__ tri_nrm, int64_t Tm, const DevStatus *st,
                                                    int64_t cap_pairs, R *__restrict__ mtri) {
  const int64_t gt = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t t = gt >> 2;
  const int sub = (int)(gt & 3);
  const bool live = t < Tm && (int64_t)st->n_pairs <= cap_pairs;
  const int b = live ? mp_off[t] : 0, e = live ? mp_off[t + 1] : 0;
  if (__all(b == e)) return;  // wave-uniform: the groups below shuffle
  R h[36], g[9];
  for (int z = 0; z < 36; ++z) h[z] = 0;
  for (int z = 0; z < 9; ++z) g[z] = 0;
  for (int i0 = b + sub; i0 < e; i0 += 16) {
    R mm[4][6], gm[4][3], nn[4][3];
    int T[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) T[k] = i0 + 4 * k < e ? pair[mp_list[i0 + 4 * k]].T : -1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (T[k] < 0) continue;
      const Pair<R> &P = pair[mp_list[i0 + 4 * k]];
      for (int v = 0; v < 6; ++v) mm[k][v] = P.mm[v];
      for (int m = 0; m < 3; ++m) gm[k][m] = P.gm[m];
      for (int d = 0; d < 3; ++d) nn[k][d] = tri_nrm[3 * (int64_t)T[k] + d];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (T[k] < 0) continue;
      const R n0 = nn[k][0], n1 = nn[k][1], n2 = nn[k][2];
      const R o[6] = {n0 * n0, n0 * n1, n0 * n2, n1 * n1, n1 * n2, n2 * n2};
      for (int v = 0; v < 6; ++v)
        for (int c = 0; c < 6; ++c) h[6 * v + c] += mm[k][v] * o[c];
      for (int m = 0; m < 3; ++m) {
        g[3 * m + 0] += gm[k][m] * n0;
        g[3 * m + 1] += gm[k][m] * n1;
        g[3 * m + 2] += gm[k][m] * n2;
      }
    }
  }
  for (int z = 0; z < 36; ++z) {
    h[z] += __shfl_xor(h[z], 1, kWave);
    h[z] += __shfl_xor(h[z], 2, kWave);
  }
  for (int z = 0; z < 9; ++z) {
    g[z] += __shfl_xor(g[z], 1, kWave);
    g[z] += __shfl_xor(g[z], 2, kWave);
  }
  if (b == e || sub != 0) return;
  R *out = mtri + 45 * t;
  for (int z = 0; z < 36; ++z) out[z] = h[z];
  for (int z = 0; z < 9; ++z) out[36 + z] = g[z];
}

// Thread per BSR row: counts the row's contributions (the entries the row
// kernel enumerates).  Rows without any get their count and gradient zeroed
// here; the others are listed for the wave kernels - light rows (at most
// a.light_bound entries, the common case) and heavy rows (master vertices under
// a much finer slave mesh) in separate lists, so that the light rows run
// with small LDS tables and full occupancy.  Nothing is listed when the
// pair records overflowed.  A light row has at most a.light_bound column
// insertions (a power of two); its column table has 2 a.light_bound slots
// and the hash tables inside it grow in powers of two up to that size.

template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_pre(RowArgs<R> a, int4 *__restrict__ rlist,
                                                       int32_t *__restrict__ rcount, int zero_cnt) {
  const int64_t row = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  int n_ent = 0, sb = 0, se = 0;
  if (row < a.V) {
    if ((int64_t)a.st_r->n_pairs <= a.cap_pairs) {
      const bool slave = row < a.Vs;
      const int64_t vid = slave ? row : row - a.Vs;
      sb = slave ? a.s_vt_off[vid] : a.m_vt_off[vid];
      se = slave ? a.s_vt_off[vid + 1] : a.m_vt_off[vid + 1];
      // four incident triangles at a time, their loads in flight together
      const int32_t *vt = slave ? a.s_vt : a.m_vt;
      for (int s0 = sb; s0 < se; s0 += 4) {
        int t[4], np[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] = s0 + k < se ? vt[s0 + k] >> 2 : -1;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          np[k] = t[k] < 0 ? 0 : (slave ? a.tri_npair[t[k]] : a.mp_off[t[k] + 1] - a.mp_off[t[k]]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (np[k] > 0) n_ent += 3 + ((slave && a.kinematic) ? 0 : 3 * np[k]);
      }
    }
    if (n_ent == 0) {
      if (zero_cnt) a.row_cnt[row] = 0;
      if (a.grad)
        for (int d = 0; d < 3; ++d) a.grad[3 * row + d] = R(0);
    }
  }
  // list appends: wave ballots, block prefix in LDS, one atomic per block and list
  __shared__ int wl[kThreads / kWave], wh[kThreads / kWave], bl, bh;
  const int w = threadIdx.x / kWave;
  const int lb = a.light_bound;
  const uint64_t ml = __ballot(n_ent > 0 && n_ent <= lb), mh = __ballot(n_ent > lb);
  if (lane == 0) {
    wl[w] = __popcll(ml);
    wh[w] = __popcll(mh);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int sl = 0, sh = 0;
    for (int k = 0; k < kThreads / kWave; ++k) {
      const int a0 = wl[k], b0 = wh[k];
      wl[k] = sl;
      wh[k] = sh;
      sl += a0;
      sh += b0;
    }
    bl = sl ? atomicAdd(&rcount[0], sl) : 0;
    bh = sh ? atomicAdd(&rcount[1], sh) : 0;
  }
  __syncthreads();
  const uint64_t below = (1ull << lane) - 1;
  const int4 rec = make_int4((int)row, sb, se, n_ent);
  if (n_ent > 0 && n_ent <= lb) rlist[bl + wl[w] + __popcll(ml & below)] = rec;
  if (n_ent > lb) rlist[a.V + bh + wh[w] + __popcll(mh & below)] = rec;
}

// One wave per listed BSR row (k_row_pre), a fixed grid walking the list.
//   PASS 0 counts the distinct columns, PASS 1 writes columns and values,
//   PASS 2 only computes the gradient row, PASS 3 fills the slave columns of
//   master rows.
// Slave row a: its contributions (column, coef, slave triangle T whose
// n_T n_T^T the coef multiplies) are enumerated in a canonical order - the
// incident triangles in adjacency order, each with its own three vertices
// and then its pairs' master vertices - and their columns inserted into an
// LDS hash set.  The (incident triangle, item) pairs - an item is the
// triangle's own three vertices or one of its pairs - are spread over the
// lanes (item offsets of the triangles in LDS, a binary search per item),
// and every contribution has a fixed slot in the canonical order.  In PASS 1
// the contributions and the incident triangles' normals are also kept in
// LDS (rows with more contributions than the stash, or more than kRowSrc
// incident triangles, re-walk their sources), each lane owns one distinct
// column and sums its contributions in the canonical order.
// Master row j: master columns take the per-master-triangle blocks of
// k_mtri, summed over the incident triangles in adjacency order; slave
// columns a are the slave vertices of the pairs of those triangles, and
// their blocks equal block (a, j) of slave row a (each contribution is a
// symmetric coef n n^T), so PASS 3 copies them after PASS 1 has written the
// slave rows.  Columns are ranked and written ascending.
constexpr int kRowEnt = 512;     // contribution stash of heavy rows (light rows: their bound)
// incident triangles of a row taken per chunk (kept in LDS): a vertex has
// far fewer than 32 in the common case, and the smaller table lets more
// waves share a CU (LDS bounds the row kernels' occupancy)
constexpr int kRowSrc = 32;

// LDS bytes of one wave of k_rows: hash set (slots, compacted in place),
// the incident-triangle table, the item marks of one round, and in PASS 1 the contribution stash - in
// groups of three (a triangle's own vertices, or one pair's master
// vertices: three distinct columns, the table index, three coefficients) -
// and the incident triangles' normals; a multiple of 16 bytes
template <typename R>
constexpr size_t row_lds_wave(int slots, int pass, bool heavy, int light_bound) {
  return ((size_t)slots * 4 + (size_t)8 * kRowSrc * 4 + (size_t)kWave * 4 +
          (pass == 1 ? (size_t)((heavy ? kRowEnt : light_bound) / 3 + 1) * (16 + 3 * sizeof(R)) +
                           (size_t)kRowSrc * 3 * sizeof(R)
                     : 0) +
          15) / 16 * 16;
}

template <typename R, int PASS, bool HEAVY>  // HEAVY: the heavy-row list (large LDS tables), same code
__global__ __launch_bounds__(kWave *kRowWaves) void k_rows(RowArgs<R> a, int slots, const int4 *__restrict__ rlist,
                                                           const int32_t *__restrict__ rcount) {
  constexpr int pass = PASS;
  extern __shared__ __align__(16) unsigned char smem[];
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int ecap = HEAVY ? kRowEnt : a.light_bound;
  const size_t per_wave = row_lds_wave<R>(slots, pass, HEAVY, a.light_bound);
  int32_t *key = reinterpret_cast<int32_t *>(smem + (size_t)w * per_wave);
  int32_t *dense = key;          // the set compacted in place
  int32_t *sip = key + slots;    // incident-triangle table: item prefix, contribution
  int32_t *seo = sip + kRowSrc;  // offset, triangle, corner, first pair
  int32_t *stt = seo + kRowSrc;
  int32_t *sco = stt + kRowSrc;
  int32_t *spb = sco + kRowSrc;
  int32_t *stv = spb + kRowSrc;  // master rows: the triangle's three vertex ids
  int32_t *smk = stv + 3 * kRowSrc;  // per round of 64 items: the table entry whose items start at a lane
  const int gcap = ecap / 3 + 1;
  int4 *egrp = reinterpret_cast<int4 *>(smk + kWave);  // PASS 1 stash: three columns + table index,
  R *ecoef = reinterpret_cast<R *>(egrp + gcap);          // three coefficients per group
  R *snrm = ecoef + 3 * gcap;                             // normals of the table's triangles
  if ((pass == 1 || pass == 3) && (int64_t)a.row_ptr[a.V] > a.cap_nnzb) return;

  // the table entry owning item f0 + lane (the last entry whose item prefix
  // is <= it): each entry with items marks the lane of its first item, a
  // ballot of the marks gives the highest mark at or below each lane, and a
  // lane before the round's first mark continues the previous round's last
  // entry (carry) - two round trips instead of a five-step binary search
  auto owner = [&](int f0, int first, int nit, int &carry) -> int {
    wave_sync();  // the previous round's mark reads are done
    smk[lane] = -1;
    if (lane < kRowSrc && nit > 0 && first >= f0 && first < f0 + kWave) smk[first - f0] = lane;
    wave_sync();
    const int mk = smk[lane];
    const uint64_t le = __ballot(mk >= 0) & ((2ull << lane) - 1);
    int lo = __shfl(mk, le ? 63 - __builtin_clzll(le) : 0, kWave);
    if (!le) lo = carry;
    carry = __builtin_amdgcn_readlane(lo, kWave - 1);
    return lo;
  };
  // the waves walk the list of rows with contributions (k_row_pre)
  const int64_t nlist = *rcount;
  const int nw = blockDim.x / kWave;
  // rows in dispatch order: an XCD-by-XCD mapping of the list measured
  // several times slower (the rows with work cluster in the list, so the
  // XCDs holding them finish last)
  const int lblk = blockIdx.x;
  // each list entry carries the row's adjacency range and contribution
  // count (k_row_pre), so a row starts with one load.  The loads are
  // pipelined over the wave's rows: the entry two rows ahead and the first
  // adjacency entries (one per lane) of the next row are in flight while the
  // wave works on the current one.
  const int64_t lstride = (int64_t)gridDim.x * nw;
  int64_t li = (int64_t)lblk * nw + w;
  auto first_ent = [&](const int4 r) -> int {  // adjacency entry sb + lane of row r
    if (pass == 3 || r.y + lane >= r.z) return 0;
    return r.x < a.Vs ? a.s_vt[r.y + lane] : a.m_vt[r.y + lane];
  };
  int4 rr_c = li < nlist ? rlist[li] : make_int4(0, 0, 0, 0);
  int4 rr_n = li + lstride < nlist ? rlist[li + lstride] : make_int4(0, 0, 0, 0);
  int ent_c = li < nlist ? first_ent(rr_c) : 0;
  for (; li < nlist; li += lstride) {
    const int ent_n = li + lstride < nlist ? first_ent(rr_n) : 0;
    const int4 rr_nn = li + 2 * lstride < nlist ? rlist[li + 2 * lstride] : make_int4(0, 0, 0, 0);
    [&](const int4 rr, const int ent0) {
  wave_sync();  // the previous row's LDS reads are done
  const int64_t row = rr.x;
  const bool slave = row < a.Vs;
  // adjacency entry src of this row (the first one per lane was prefetched)
  auto vt_at = [&](int src) -> int {
    return src - rr.y == lane ? ent0 : (slave ? a.s_vt[src] : a.m_vt[src]);
  };

  if (pass == 3) {
    if (slave) return;
    const int64_t e1 = a.row_ptr[row + 1];
    for (int64_t e = a.row_ptr[row] + lane; e < e1; e += kWave) {
      const int32_t c = a.col[e];
      if (c >= a.Vs) break;  // columns ascend: the slave columns come first
      // column `row` in slave row c: an 8-way search (seven probes loaded
      // together per round, then the last <= 8 entries at once), so a row of
      // up to 64 columns takes two rounds of loads
      int64_t lo = a.row_ptr[c], hi = a.row_ptr[c + 1];
      while (hi - lo > 8) {
        const int64_t step = (hi - lo + 7) >> 3;
        int32_t pv[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) pv[k] = lo + (k + 1) * step < hi ? a.col[lo + (k + 1) * step] : INT32_MAX;
        int64_t nlo = lo, nhi = hi;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
          const int64_t idx = lo + (k + 1) * step;
          if (idx >= hi) break;
          if (pv[k] <= (int32_t)row) nlo = idx;
          else if (idx < nhi) nhi = idx;
        }
        lo = nlo;
        hi = nhi;
      }
      int64_t at = -1;
      int32_t cv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) cv[k] = lo + k < hi ? a.col[lo + k] : -1;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (cv[k] == (int32_t)row) at = lo + k;
      if (at >= 0) {
        for (int z = 0; z < 9; ++z) a.val[9 * e + z] = a.val[9 * at + z];
      } else {
        set_error(a.st, GMCP_E_CAPACITY, (unsigned long long)row);  // unreachable: the patterns are symmetric
      }
    }
    return;
  }

  const int sb = rr.y, se = rr.z;
  const int n_ent = rr.w;

  if (!slave) {
    // ------------------------------------------------------ master row
    if (pass != 0 && a.grad) {
      // gradient row: lane partials over the incident triangles, fixed-order butterfly
      R gr[3] = {0, 0, 0};
      for (int src = sb + lane; src < se; src += kWave) {
        const int ent = vt_at(src), t = ent >> 2, corner = ent & 3;
        if (a.mp_off[t] == a.mp_off[t + 1]) continue;
        const R *G = a.mtri + 45 * (int64_t)t + 36 + 3 * corner;
        for (int d = 0; d < 3; ++d) gr[d] += G[d];
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
    bool full = false;
    // (incident triangle, item) pairs over the lanes: item 0 = the triangle's
    // three master vertices, item 1 + i = the slave vertices of its pair i
    const bool one_chunk = se - sb <= kRowSrc;
    for (int s0 = sb; s0 < se; s0 += kRowSrc) {
      const int src = s0 + lane;
      int t = 0, corner = 0, np = 0, pb = 0, tv[3] = {0, 0, 0};
      if (lane < kRowSrc && src < se) {
        const int ent = vt_at(src);
        t = ent >> 2;
        corner = ent & 3;
        pb = a.mp_off[t];
        np = a.mp_off[t + 1] - pb;
        if (np > 0)
          for (int m = 0; m < 3; ++m) tv[m] = a.tm[3 * (int64_t)t + m];
      }
      const int nit = np > 0 ? 1 + np : 0;
      const int iin = wave_incl_add(nit);
      const int items = __shfl(iin, kWave - 1, kWave);
      wave_sync();  // the previous chunk's table reads are done
      if (lane < kRowSrc) {
        sip[lane] = iin - nit;
        stt[lane] = np > 0 ? t : -1;  // -1: no pairs (no contribution)
        sco[lane] = corner;
        spb[lane] = pb;
        for (int m = 0; m < 3; ++m) stv[3 * lane + m] = tv[m];
      }
      int carry = 0;
      for (int f0 = 0; f0 < items; f0 += kWave) {
        const int lo = owner(f0, iin - nit, nit, carry), f = f0 + lane;
        if (f >= items) continue;
        const int j = f - sip[lo];
        if (j == 0) {
          for (int m = 0; m < 3; ++m) row_slot(key, tsz, (int32_t)(a.Vs + stv[3 * lo + m]), &full);
        } else {
          const int64_t T = a.mp_key[spb[lo] + j - 1] >> 32;
          for (int q = 0; q < 3; ++q) row_slot(key, tsz, a.ts[3 * T + q], &full);
        }
      }
    }
    if (__any(full)) {
      if (lane == 0) {
        // a table of n_ent slots always fits (distinct columns <= insertions)
        atomicMax(&a.st->need_row, (unsigned long long)max(2 * slots, min(n_ent, 4096)));
        atomicCAS(&a.st->code, 0, GMCP_E_CAPACITY);
        if (pass == 0) a.row_cnt[row] = 0;
      }
      return;
    }
    wave_sync();
    int nuniq = 0;
    for (int i0 = 0; i0 < tsz; i0 += kWave) {
      const int i = i0 + lane;
      const int32_t kv = i < tsz ? key[i] : -1;  // read before any lane writes (in place)
      const bool used = kv >= 0;
      const uint64_t m = __ballot(used);
      if (used) dense[nuniq + __popcll(m & ((1ull << lane) - 1))] = kv;
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
      const int64_t dst = (int64_t)a.row_ptr[row] + r;
      a.col[dst] = c;
      if (c < a.Vs) continue;  // slave column: PASS 3
      R v[6] = {0, 0, 0, 0, 0, 0};
      if (one_chunk) {  // the incident triangles are in the table, in adjacency order
        for (int k = 0; k < se - sb; ++k) {
          const int t = stt[k];
          if (t < 0) continue;
          for (int m = 0; m < 3; ++m) {
            if ((int32_t)(a.Vs + stv[3 * k + m]) != c) continue;
            const R *B = a.mtri + 45 * (int64_t)t + 6 * sym3(sco[k], m);
            for (int z = 0; z < 6; ++z) v[z] += B[z];
          }
        }
      } else {
        for (int src = sb; src < se; ++src) {
          const int ent = a.m_vt[src], t = ent >> 2, corner = ent & 3;
          if (a.mp_off[t] == a.mp_off[t + 1]) continue;
          for (int m = 0; m < 3; ++m) {
            if ((int32_t)(a.Vs + a.tm[3 * (int64_t)t + m]) != c) continue;
            const R *B = a.mtri + 45 * (int64_t)t + 6 * sym3(corner, m);
            for (int z = 0; z < 6; ++z) v[z] += B[z];
          }
        }
      }
      R *ov = a.val + 9 * dst;
      ov[0] = v[0]; ov[1] = v[1]; ov[2] = v[2];
      ov[3] = v[1]; ov[4] = v[3]; ov[5] = v[4];
      ov[6] = v[2]; ov[7] = v[4]; ov[8] = v[5];
    }
    return;
  }

  // -------------------------------------------------------- slave row
  // contributions of one source (incident triangle), in canonical order
  auto visit_src = [&](int src, auto &&visit) {
    const int ent = a.s_vt[src];
    const int t = ent >> 2, corner = ent & 3;
    if (a.tri_npair[t] == 0) return;
    const R *S = a.tri_sum + 9 * (int64_t)t;
    for (int b = 0; b < 3; ++b) visit(a.ts[3 * (int64_t)t + b], S[sym3(corner, b)], t);
    if (!a.kinematic) {
      const int pb = a.tri_poff[t], np = a.tri_npair[t];
      for (int p = pb; p < pb + np; ++p) {
        const Pair<R> &P = a.pair[p];
        for (int m = 0; m < 3; ++m) visit((int32_t)(a.Vs + P.mv[m]), P.sm[3 * corner + m], t);
      }
    }
  };

  if (pass != 0 && a.grad) {
    // gradient row: sum over incident triangles of -gs[T][a] n_T (lane
    // partials, fixed-order butterfly)
    R gr[3] = {0, 0, 0};
    for (int src = sb + lane; src < se; src += kWave) {
      const int ent = vt_at(src), t = ent >> 2, corner = ent & 3;
      if (a.tri_npair[t] == 0) continue;
      const R cf = -a.tri_sum[9 * (int64_t)t + 6 + corner];
      const R *nn = a.tri_nrm + 3 * (int64_t)t;
      for (int d = 0; d < 3; ++d) gr[d] += cf * nn[d];
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
  const bool stash = pass == 1 && n_ent <= ecap && se - sb <= kRowSrc;
  bool full = false;
  // one group of three contributions starting at canonical offset e0 (a multiple of 3)
  auto put3 = [&](const int32_t col[3], const R cf[3], int e0, int k) {
    for (int b = 0; b < 3; ++b) row_slot(key, tsz, col[b], &full);
    if (stash) {
      const int gi = e0 / 3;
      egrp[gi] = make_int4(col[0], col[1], col[2], k);
      for (int b = 0; b < 3; ++b) ecoef[3 * gi + b] = cf[b];
    }
  };
  int run = 0;  // contributions of the earlier chunks of incident triangles
  for (int s0 = sb; s0 < se; s0 += kRowSrc) {
    const int src = s0 + lane;
    int t = 0, corner = 0, np = 0, pb = 0;
    if (lane < kRowSrc && src < se) {
      const int ent = vt_at(src);
      t = ent >> 2;
      corner = ent & 3;
      np = a.tri_npair[t];
      if (np > 0 && !a.kinematic) pb = a.tri_poff[t];
    }
    const int nit = np > 0 ? 1 + (a.kinematic ? 0 : np) : 0;
    const int nen = np > 0 ? 3 + (a.kinematic ? 0 : 3 * np) : 0;
    const int iin = wave_incl_add(nit), ein = wave_incl_add(nen);
    const int items = __shfl(iin, kWave - 1, kWave), ents = __shfl(ein, kWave - 1, kWave);
    wave_sync();  // the previous chunk's table reads are done
    if (lane < kRowSrc) {
      sip[lane] = iin - nit;
      seo[lane] = run + ein - nen;
      stt[lane] = t;
      sco[lane] = corner;
      spb[lane] = pb;
      if (stash && np > 0)
        for (int d = 0; d < 3; ++d) snrm[3 * lane + d] = a.tri_nrm[3 * (int64_t)t + d];
    }
    int carry = 0;
    for (int f0 = 0; f0 < items; f0 += kWave) {
      const int lo = owner(f0, iin - nit, nit, carry), f = f0 + lane;
      if (f >= items) continue;
      const int j = f - sip[lo], tt = stt[lo], c = sco[lo];
      int32_t col[3];
      R cf[3];
      if (j == 0) {  // the triangle's own vertices
        const R *S = a.tri_sum + 9 * (int64_t)tt;
        for (int b = 0; b < 3; ++b) {
          col[b] = a.ts[3 * (int64_t)tt + b];
          cf[b] = S[sym3(c, b)];
        }
        put3(col, cf, seo[lo], lo);
      } else {  // pair j - 1 of the triangle: its master vertices
        const Pair<R> &P = a.pair[spb[lo] + j - 1];
        for (int m = 0; m < 3; ++m) {
          col[m] = (int32_t)(a.Vs + P.mv[m]);
          cf[m] = P.sm[3 * c + m];
        }
        put3(col, cf, seo[lo] + 3 + 3 * (j - 1), lo);
      }
    }
    run += ents;
  }
  if (__any(full)) {
    if (lane == 0) {
      // a table of n_ent slots always fits (distinct columns <= insertions)
      atomicMax(&a.st->need_row, (unsigned long long)max(2 * slots, min(n_ent, 4096)));
      atomicCAS(&a.st->code, 0, GMCP_E_CAPACITY);
      if (pass == 0) a.row_cnt[row] = 0;
    }
    return;
  }
  wave_sync();
  int nuniq = 0;
  for (int i0 = 0; i0 < tsz; i0 += kWave) {
    const int i = i0 + lane;
    const int32_t kv = i < tsz ? key[i] : -1;  // read before any lane writes (in place)
    const bool used = kv >= 0;
    const uint64_t m = __ballot(used);
    if (used) dense[nuniq + __popcll(m & ((1ull << lane) - 1))] = kv;
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
    auto add_n = [&](R cf, const R *nn) {
      v[0] += cf * nn[0] * nn[0];
      v[1] += cf * nn[0] * nn[1];
      v[2] += cf * nn[0] * nn[2];
      v[3] += cf * nn[1] * nn[1];
      v[4] += cf * nn[1] * nn[2];
      v[5] += cf * nn[2] * nn[2];
    };
    if (stash) {  // the three columns of a group are distinct: at most one matches
      for (int gi = 0; gi < n_ent / 3; ++gi) {
        const int4 cg = egrp[gi];
        const int b = cg.x == c ? 0 : (cg.y == c ? 1 : (cg.z == c ? 2 : -1));
        if (b >= 0) add_n(ecoef[3 * gi + b], snrm + 3 * cg.w);
      }
    } else {
      for (int src = sb; src < se; ++src)
        visit_src(src, [&](int32_t col, R cf, int t) {
          if (col == c) add_n(cf, a.tri_nrm + 3 * (int64_t)t);
        });
    }
    const int64_t dst = (int64_t)a.row_ptr[row] + r;
    a.col[dst] = c;
    R *ov = a.val + 9 * dst;
    ov[0] = v[0]; ov[1] = v[1]; ov[2] = v[2];
    ov[3] = v[1]; ov[4] = v[3]; ov[5] = v[4];
    ov[6] = v[2]; ov[7] = v[4]; ov[8] = v[5];
  }
    }(rr_c, ent_c);
    rr_c = rr_n;
    ent_c = ent_n;
    rr_n = rr_nn;
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
// per-environment sum of the tile energies: a fixed split over 1024
// threads, wave butterflies, then the 16 wave sums in order (deterministic)
__global__ __launch_bounds__(1024) void k_energy(const double *__restrict__ tile_E, const EnvInfo *__restrict__ env,
                                                 R *energy, const int32_t *__restrict__ row_ptr, int64_t V,
                                                 DevStatus *st, int64_t cap_nnzb) {
  __shared__ double part[1024 / kWave];
  const int e = blockIdx.x, lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (row_ptr && e == 0 && threadIdx.x == 0) {  // the BSR's block count (after the row kernels)
    const long long nnzb = row_ptr[V];
    st->nnzb = (unsigned long long)nnzb;
    if (nnzb > cap_nnzb) atomicCAS(&st->code, 0, GMCP_E_CAPACITY);
  }
  const int t0 = env[e].tile0, t1 = env[e].tile1;
  double s = 0.0;
  for (int t = t0 + threadIdx.x; t < t1; t += 1024) s += tile_E[t];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
  if (lane == 0) part[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int k = 0; k < 1024 / kWave; ++k) tot += part[k];
    energy[e] = (R)tot;
  }
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

// (slave triangle, master triangle) of every contact pair of the last
// assembly, in storage order (contiguous per slave triangle)
template <typename R>
__global__ void k_pair_export(const Pair<R> *__restrict__ pair, const DevStatus *st, int64_t cap_pairs, int64_t cap,
                              int32_t *T, int32_t *M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t np = (int64_t)st->n_pairs;
  if (np > cap_pairs || i >= np || i >= cap) return;
  T[i] = pair[i].T;
  M[i] = pair[i].M;
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
      R bs[3] = {R(1) - r.s1 - r.s2, r.s1, r.s2};
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
  ra.mp_key = b.mp_key;
  ra.mtri = (const R *)b.mtri;
  ra.st_r = b.status;
  ra.st = b.status;
  ra.cap_pairs = c->caps.pairs;
  ra.row_cnt = b.row_cnt;
  ra.row_ptr = H ? H->row_ptr : nullptr;
  ra.col = H ? H->col : nullptr;
  ra.val = H ? (R *)H->val : nullptr;
  ra.cap_nnzb = H ? H->cap_nnzb : 0;
  ra.grad = nullptr;
  ra.light_bound = light_row_bound(c);
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
  StageInit si;
  si.which = 2;
  si.zero[0] = b.rcount;  // row-list lengths
  si.nzero[0] = 2;
  si.zero[1] = b.row_cnt + c->V;  // the scan's tail
  si.nzero[1] = 1;
  si.zero[2] = b.atile_cnt;  // active-tile list length
  si.nzero[2] = 1;
  hipError_t e = stage_init(c, si);
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
  na.cand_cnt = b.cand_cnt;
  na.cand_pos = b.cand_tmp_off;
  na.cand = b.cand_tmp;
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
  na.mp_cnt = b.mp_cnt;
  na.atile = c->mortar ? nullptr : b.atile;  // clipped samples: the step bound walks every tile
  na.atile_cnt = b.atile_cnt;
  na.tile_act = c->mortar ? nullptr : b.tile_act;
  na.epoch = b.epoch;
  na.tile_E = b.tile_E;
  na.st = b.status;
  na.features = c->features;
  na.m_opp = b.m_opp;
  na.m_vt_off = b.m_vt_off;
  na.m_vt = b.m_vt;
  prof_mark(c, ST_NARROW, 0);
  if (c->n_tiles) {
    if (c->mortar) {
      if constexpr (sizeof(R) == 4)
        hipLaunchKernelGGL(k_mortar_f32, dim3((unsigned)c->n_tiles), dim3(kWave), 0, s, na);
      else
        hipLaunchKernelGGL(k_mortar_f64, dim3((unsigned)c->n_tiles), dim3(kWave), 0, s, na);
      hipLaunchKernelGGL(k_mortar_counts, dim3(1), dim3(64), 0, s, b.status);
    } else
      if constexpr (sizeof(R) == 4)
        hipLaunchKernelGGL(k_narrow_f32, dim3(nblk(c->n_tiles, narrow_waves<R>())), dim3(kWave * narrow_waves<R>()),
                           0, s, na);
      else
        hipLaunchKernelGGL(k_narrow_f64, dim3(nblk(c->n_tiles, narrow_waves<R>())), dim3(kWave * narrow_waves<R>()),
                           0, s, na);
  }
  prof_mark(c, ST_NARROW, 1);
  // bucket pairs by master triangle (needed for master rows and the HVP)
  const Pair<R> *pr = (const Pair<R> *)b.pair;
  unsigned pb = nblk(c->caps.pairs);
  prof_mark(c, ST_BUCKET, 0);
  e = scan_exclusive(c, b.mp_cnt, b.mp_off, c->Tm + 1);  // counts written by the narrow phase
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pair_bucket<R>, dim3(pb), dim3(kThreads), 0, s, pr, b.status, c->caps.pairs, b.mp_cnt,
                     b.mp_off, b.mp_key, c->Tm);
  hipLaunchKernelGGL(k_bucket_rank<R>, dim3(pb), dim3(kThreads), 0, s, pr, b.mp_off, b.mp_key, b.mp_list, b.status,
                     c->caps.pairs);
  prof_mark(c, ST_BUCKET, 1);
  RowArgs<R> ra = row_args<R>(c, H);
  ra.grad = grad;
  const int nw = kRowWaves;
  // light and heavy rows (and the master-triangle sums) are independent:
  // the heavy ones run on the library's second stream, forked after the row
  // lists and joined before what reads both (not while profiling)
  const bool par = c->side != nullptr && !c->prof.on;
  const hipStream_t hs = par ? c->side : s;
  auto fork = [&]() {
    if (!par) return hipSuccess;
    hipError_t r = hipEventRecord(c->ev_fork, s);
    return r != hipSuccess ? r : hipStreamWaitEvent(c->side, c->ev_fork, 0);
  };
  auto join = [&]() {
    if (!par) return hipSuccess;
    hipError_t r = hipEventRecord(c->ev_join, c->side);
    return r != hipSuccess ? r : hipStreamWaitEvent(s, c->ev_join, 0);
  };
  const bool sums = !c->kinematic && (grad || H) && c->Tm;
  auto mtri = [&](hipStream_t st) {
    prof_mark(c, ST_MTRI, 0);
    hipLaunchKernelGGL(k_mtri<R>, dim3(nblk(4 * c->Tm, kThreads)), dim3(kThreads), 0, st, pr, b.mp_off,
                       b.mp_list, (const R *)b.tri_nrm, c->Tm, b.status, c->caps.pairs, (R *)b.mtri);
    prof_mark(c, ST_MTRI, 1);
  };
  if (sums && !H) mtri(s);  // the gradient rows read the sums
  if (grad || H) {
    prof_mark(c, ST_ROWS_PRE, 0);
    if (c->V)
      hipLaunchKernelGGL(k_row_pre<R>, dim3(nblk(c->V)), dim3(kThreads), 0, s, ra, b.rlist, b.rcount, H ? 1 : 0);
    prof_mark(c, ST_ROWS_PRE, 1);
  }
  // the row kernels walk the two row lists with fixed grids: light rows with
  // small LDS tables, heavy rows with tables of up to 4096 slots
  const int64_t rneed = (c->V + nw - 1) / nw;
  const int64_t rmax = light_row_blocks(c);
  const dim3 rgrid((unsigned)(rneed < rmax ? (rneed > 0 ? rneed : 1) : rmax));
  const dim3 hgrid((unsigned)heavy_row_blocks(c));
  const int4 *light = b.rlist, *heavy = b.rlist + c->V;
  const int32_t *nlight = b.rcount, *nheavy = b.rcount + 1;
  if (grad && !H) {  // gradient alone: the row kernel's gradient-only pass
    prof_mark(c, ST_GRAD, 0);
    if ((e = fork()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_rows<R, 2, true>), hgrid, dim3(kWave * nw), 0, hs, ra, 64, heavy, nheavy);
    hipLaunchKernelGGL((k_rows<R, 2, false>), rgrid, dim3(kWave * nw), 0, s, ra, 64, light, nlight);
    if ((e = join()) != hipSuccess) return e;
    prof_mark(c, ST_GRAD, 1);
  }
  if (H) {
    // per wave: distinct-column set and list (8 B per slot) plus, in the
    // writing pass, the row's contributions (<= kRowEnt).  Heavy tables start
    // at 512 slots (a row's distinct columns never exceed its insertions, so
    // rows below 512 insertions always fit) and grow with the capacity
    // reported by a row that did not fit
    const int lslots = 2 * ra.light_bound;
    int hslots = 512;
    while (hslots < c->caps.row_entries && hslots < 4096) hslots <<= 1;
    auto lds = [&](int sl, int pass, bool heavy) {
      return (size_t)nw * row_lds_wave<R>(sl, pass, heavy, ra.light_bound);
    };
    if ((e = fork()) != hipSuccess) return e;
    if (sums) mtri(hs);  // read by the writing pass
    prof_mark(c, ST_ROWS_COUNT_H, 0);
    hipLaunchKernelGGL((k_rows<R, 0, true>), hgrid, dim3(kWave * nw), lds(hslots, 0, true), hs, ra, hslots, heavy,
                       nheavy);
    prof_mark(c, ST_ROWS_COUNT_H, 1);
    prof_mark(c, ST_ROWS_COUNT, 0);
    hipLaunchKernelGGL((k_rows<R, 0, false>), rgrid, dim3(kWave * nw), lds(lslots, 0, false), s, ra, lslots, light,
                       nlight);
    prof_mark(c, ST_ROWS_COUNT, 1);
    if ((e = join()) != hipSuccess) return e;
    e = scan_exclusive(c, b.row_cnt, H->row_ptr, c->V + 1);
    if (e != hipSuccess) return e;
    if ((e = fork()) != hipSuccess) return e;
    prof_mark(c, ST_ROWS_FILL_H, 0);
    hipLaunchKernelGGL((k_rows<R, 1, true>), hgrid, dim3(kWave * nw), lds(hslots, 1, true), hs, ra, hslots, heavy,
                       nheavy);
    prof_mark(c, ST_ROWS_FILL_H, 1);
    prof_mark(c, ST_ROWS_FILL, 0);
    hipLaunchKernelGGL((k_rows<R, 1, false>), rgrid, dim3(kWave * nw), lds(lslots, 1, false), s, ra, lslots, light,
                       nlight);
    prof_mark(c, ST_ROWS_FILL, 1);
    if ((e = join()) != hipSuccess) return e;
    if (c->V > c->Vs) {
      prof_mark(c, ST_ROWS_COPY, 0);
      if ((e = fork()) != hipSuccess) return e;
      hipLaunchKernelGGL((k_rows<R, 3, true>), hgrid, dim3(kWave * nw), 0, hs, ra, hslots, heavy, nheavy);
      hipLaunchKernelGGL((k_rows<R, 3, false>), rgrid, dim3(kWave * nw), 0, s, ra, lslots, light, nlight);
      if ((e = join()) != hipSuccess) return e;
      prof_mark(c, ST_ROWS_COPY, 1);
    }
  }
  // per-environment energy (and the BSR's block count when written)
  hipLaunchKernelGGL(k_energy<R>, dim3(c->n_env), dim3(1024), 0, s, b.tile_E, b.env, energy,
                     H ? (const int32_t *)H->row_ptr : nullptr, c->V, b.status, H ? H->cap_nnzb : (int64_t)0);
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

template <typename R>
hipError_t launch_pair_export(gmcp_ctx *c, int32_t *T, int32_t *M, int64_t cap) {
  const int64_t n = std::min<int64_t>(cap, c->caps.pairs);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_export<R>, dim3(nblk(n)), dim3(kThreads), 0, c->stream, (const Pair<R> *)c->b.pair,
                     c->b.status, c->caps.pairs, cap, T, M);
  return hipGetLastError();
}

// Energy of the last assembly's samples at new positions, every sample
// frozen: slave triangle normal n_T, rule point, master triangle and its
// barycentric coordinates, weight, face weight and support radius.  The gap
// is then affine in x, g = n_T . (sum_j bm_j x_mj - sum_a bs_a x_sa), and the
// gradient of this energy at the assembly positions is the assembled
// gradient (Sec. 4.2's gradient and Hessian approximation).  One wave per
// work tile, lane = triangle of the tile looping over its records (in lane
// order), a fixed butterfly per tile: deterministic.  A gap <= 0 gives +inf.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_energy_frozen(const R *__restrict__ xs, const R *__restrict__ xm,
                                                             const int32_t *__restrict__ ts,
                                                             const int32_t *__restrict__ tm,
                                                             const Tile *__restrict__ tiles, int n_tiles,
                                                             const int32_t *__restrict__ s_order,
                                                             const EnvInfo *__restrict__ env,
                                                             const double *__restrict__ rule, const R *__restrict__ area,
                                                             const Rec<R> *__restrict__ rec,
                                                             const int32_t *__restrict__ tri_roff,
                                                             const int32_t *__restrict__ tri_rcnt,
                                                             const R *__restrict__ tri_nrm, const DevStatus *st,
                                                             int64_t cap_active, double *__restrict__ tile_E) {
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int tile_id = blockIdx.x * kTilePerBlock + w;
  if (tile_id >= n_tiles) return;
  if ((int64_t)st->n_active > cap_active) {
    if (lane == 0) tile_E[tile_id] = NAN;
    return;
  }
  const Tile tl = tiles[tile_id];
  double E = 0.0;
  if (lane < tl.count) {
    const int T = s_order[tl.first + lane];
    const int r0 = tri_roff[T], r1 = r0 + tri_rcnt[T];
    if (r1 > r0) {
      R s0[3], e1[3], e2[3];
      const int64_t v0 = ts[3 * (int64_t)T], v1 = ts[3 * (int64_t)T + 1], v2 = ts[3 * (int64_t)T + 2];
      for (int d = 0; d < 3; ++d) {
        s0[d] = xs[3 * v0 + d];
        e1[d] = xs[3 * v1 + d] - s0[d];
        e2[d] = xs[3 * v2 + d] - s0[d];
      }
      const R n0 = tri_nrm[3 * (int64_t)T], n1 = tri_nrm[3 * (int64_t)T + 1], n2 = tri_nrm[3 * (int64_t)T + 2];
      for (int r = r0; r < r1; ++r) {
        const Rec<R> rc = rec[r];
        const R xi = rc.s1, eta = rc.s2;
        const int64_t m0 = tm[3 * (int64_t)rc.M], m1 = tm[3 * (int64_t)rc.M + 1], m2 = tm[3 * (int64_t)rc.M + 2];
        R dv[3];
        for (int d = 0; d < 3; ++d)
          dv[d] = rc.b0 * (xm[3 * m0 + d] - s0[d]) + rc.b1 * (xm[3 * m1 + d] - s0[d]) +
                  rc.b2 * (xm[3 * m2 + d] - s0[d]) - (xi * e1[d] + eta * e2[d]);
        const R g = n0 * dv[0] + n1 * dv[1] + n2 * dv[2];
        const R eps = rc.eps;
        if (!(g > R(0))) {
          E = INFINITY;
        } else if (g < eps) {
          const R dd = g - eps;
          const R B = -dd * dd * log1p_r<R>(dd / eps);
          E += (double)(rc.kwg * B);
        }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) E += __shfl_xor(E, o, kWave);
  if (lane == 0) tile_E[tile_id] = E;
}

template <typename R>
hipError_t launch_energy_frozen(gmcp_ctx *c, const R *xs, const R *xm, R *energy) {
  Buffers &b = c->b;
  if (c->n_tiles)
    hipLaunchKernelGGL(k_energy_frozen<R>, dim3(nblk(c->n_tiles, kTilePerBlock)), dim3(kThreads), 0, c->stream, xs, xm,
                       c->ts, c->tm, b.tiles, (int)c->n_tiles, b.s_order, b.env, b.rule, (const R *)b.area,
                       (const Rec<R> *)b.rec, b.tri_roff, b.tri_rcnt, (const R *)b.tri_nrm, b.status, c->caps.active,
                       b.tile_E);
  hipLaunchKernelGGL(k_energy<R>, dim3(c->n_env), dim3(1024), 0, c->stream, b.tile_E, b.env, energy, nullptr,
                     (int64_t)0, b.status, (int64_t)0);
  return hipGetLastError();
}

#define GMCP_INST(R)                                                                                            \
  template hipError_t launch_rest_area<R>(gmcp_ctx *, const R *, R *);                                          \
  template hipError_t launch_assemble<R>(gmcp_ctx *, const R *, const R *, const R *, const R *, R *, R *,      \
                                         const gmcp_bsr *);                                                     \
  template hipError_t launch_hvp<R>(gmcp_ctx *, const R *, const R *, R *, R *);                                \
  template hipError_t launch_sample_results<R>(gmcp_ctx *, int32_t *, R *, R *, R *, R *, R *);                \
  template hipError_t launch_energy_frozen<R>(gmcp_ctx *, const R *, const R *, R *);                         \
  template hipError_t launch_pair_export<R>(gmcp_ctx *, int32_t *, int32_t *, int64_t);
GMCP_INST(float)
GMCP_INST(double)

}  // namespace gmcp
