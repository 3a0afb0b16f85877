// Host side of the GMCP library: C ABI, workspace plan, static tables.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <map>
#include <vector>

#include "common.h"

using namespace gmcp;

namespace {

// ------------------------------------------------------------ quadrature
// Gauss rules from the three-term recurrence of the monic orthogonal
// polynomials of a weight on [-1,1]:  p_{k+1} = (x - a_k) p_k - b_k p_{k-1}.
// Nodes: roots of p_n (bracketed on a fine grid, refined by bisection);
// weights by the Christoffel formula  w_i = 1 / sum_k p_k(x_i)^2 / h_k,
// h_0 = mu_0, h_k = b_k h_{k-1}.
struct Recurrence {
  double a[8], b[8], mu0;
};

double eval_monic(const Recurrence &r, int n, double x, double *vals) {
  double pm1 = 0.0, p = 1.0;
  if (vals) vals[0] = 1.0;
  for (int k = 0; k < n; ++k) {
    double pn = (x - r.a[k]) * p - (k > 0 ? r.b[k] * pm1 : 0.0);
    pm1 = p;
    p = pn;
    if (vals && k + 1 < n) vals[k + 1] = p;
  }
  return p;
}

void gauss_from_recurrence(const Recurrence &r, int n, double *x, double *w) {
  const int kGrid = 20000;
  int found = 0;
  double prev_x = -1.0, prev_f = eval_monic(r, n, -1.0, nullptr);
  for (int i = 1; i <= kGrid && found < n; ++i) {
    double xx = -1.0 + 2.0 * i / kGrid;
    double f = eval_monic(r, n, xx, nullptr);
    if (f == 0.0) {  // a root on the grid itself: take it, bracket nothing
      x[found++] = xx;
      prev_x = xx;
      prev_f = 0.0;
      continue;
    }
    if (prev_f != 0.0 && (prev_f < 0) != (f < 0)) {
      double lo = prev_x, hi = xx, flo = prev_f;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        double fm = eval_monic(r, n, mid, nullptr);
        if ((fm < 0) == (flo < 0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      x[found++] = 0.5 * (lo + hi);
    }
    prev_x = xx;
    prev_f = f;
  }
  for (int i = 0; i < n; ++i) {
    double vals[8];
    eval_monic(r, n, x[i], vals);
    double h = r.mu0, s = 0.0;
    for (int k = 0; k < n; ++k) {
      if (k > 0) h *= r.b[k];
      s += vals[k] * vals[k] / h;
    }
    w[i] = 1.0 / s;
  }
}

// rule[n-1][q][3] = (xi, eta, w) of the n x n Stroud conical product rule
// and, from kGaussOff, gl[n-1][j][2] = (node, weight) of the n-point
// Gauss-Legendre rule on [0, 1] (edge samples)
void build_rules(double *rule) {
  memset(rule, 0, sizeof(double) * kRuleDoubles);
  for (int n = 1; n <= kMaxRule; ++n) {
    // Jacobi (alpha=1, beta=0): weight (1-x), mu0 = 2,
    // a_k = -1/((2k+1)(2k+3)), b_k = k(k+1)/(2k+1)^2
    Recurrence jac{}, leg{};
    jac.mu0 = 2.0;
    leg.mu0 = 2.0;
    for (int k = 0; k < 8; ++k) {
      jac.a[k] = -1.0 / ((2.0 * k + 1.0) * (2.0 * k + 3.0));
      jac.b[k] = k > 0 ? k * (k + 1.0) / ((2.0 * k + 1.0) * (2.0 * k + 1.0)) : 0.0;
      // Legendre: a_k = 0, b_k = k^2 / (4k^2 - 1)
      leg.a[k] = 0.0;
      leg.b[k] = k > 0 ? (double)k * k / (4.0 * k * k - 1.0) : 0.0;
    }
    double xj[8], wj[8], xl[8], wl[8];
    gauss_from_recurrence(jac, n, xj, wj);
    gauss_from_recurrence(leg, n, xl, wl);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double u = 0.5 * (1.0 + xj[i]), Wu = 0.25 * wj[i];
        double v = 0.5 * (1.0 + xl[j]), Wv = 0.5 * wl[j];
        double *r = rule + ((n - 1) * 16 + i * n + j) * 3;
        r[0] = u;
        r[1] = v * (1.0 - u);
        r[2] = Wu * Wv;
      }
    for (int j = 0; j < n; ++j) {
      double *g = rule + kGaussOff + ((n - 1) * 4 + j) * 2;
      g[0] = 0.5 * (1.0 + xl[j]);
      g[1] = 0.5 * wl[j];
    }
  }
}

// ------------------------------------------------------- workspace plan
struct Plan {
  size_t off = 0;
  char *base = nullptr;
  template <typename T>
  T *take(int64_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += sizeof(T) * (size_t)(count > 0 ? count : 1);
    return p;
  }
};

struct Sizes {
  int n_env;
  int64_t Vs, Vm, Ts, Tm, Ns, V, n_tiles, cells;
  bool f64, kin, feat;
};

bool layout_sizes(const gmcp_layout *L, Sizes *s) {
  if (!L || L->n_env <= 0 || !L->slave_v_off || !L->slave_t_off || !L->master_v_off ||
      !L->master_t_off || !L->rule_n || !L->kappa || !L->dhat || !L->delta_T)
    return false;
  s->n_env = L->n_env;
  s->f64 = (L->flags & GMCP_F64) != 0;
  s->kin = (L->flags & GMCP_KINEMATIC_MASTER) != 0;
  s->feat = (L->flags & GMCP_FEATURES) != 0;
  if (s->feat && !(L->flags & GMCP_MORTAR)) return false;  // edge / point samples join clipped face samples
  if (L->slave_v_off[0] != 0 || L->slave_t_off[0] != 0 || L->master_v_off[0] != 0 ||
      L->master_t_off[0] != 0)
    return false;
  s->Ns = 0;
  s->n_tiles = 0;
  for (int e = 0; e < L->n_env; ++e) {
    if (L->slave_v_off[e + 1] < L->slave_v_off[e] || L->slave_t_off[e + 1] < L->slave_t_off[e] ||
        L->master_v_off[e + 1] < L->master_v_off[e] || L->master_t_off[e + 1] < L->master_t_off[e])
      return false;
    int n = L->rule_n[e];
    if (n < 1 || n > kMaxRule) return false;
    if (!(L->dhat[e] > 0.0) || !(L->kappa[e] >= 0.0) || !(L->delta_T[e] >= 0.0)) return false;
    int64_t te = L->slave_t_off[e + 1] - L->slave_t_off[e];
    int per = kWave / (n * n);
    s->Ns += te * n * n;
    s->n_tiles += (te + per - 1) / per;
  }
  s->Vs = L->slave_v_off[L->n_env];
  s->Ts = L->slave_t_off[L->n_env];
  s->Vm = L->master_v_off[L->n_env];
  s->Tm = L->master_t_off[L->n_env];
  s->V = s->kin ? s->Vs : s->Vs + s->Vm;
  return s->Ns < (int64_t(1) << 31) && s->V < (int64_t(1) << 30);
}

// lays out every buffer; with base == nullptr only computes the size
size_t plan_workspace(const Sizes &s, const gmcp_caps &cp, char *base, Buffers *b, size_t *scan_elems) {
  Plan p;
  p.base = base;
  Buffers t{};
  int rsz = s.f64 ? 8 : 4;
  t.status = p.take<DevStatus>(1);
  t.env = p.take<EnvInfo>(s.n_env);
  t.tiles = p.take<Tile>(s.n_tiles);
  t.s_order = p.take<int32_t>(s.Ts);
  t.samp_off = p.take<int32_t>(s.Ts + 1);
  t.s_env = p.take<int32_t>(s.Ts);
  t.s_venv = p.take<int32_t>(s.Vs);
  t.m_env = p.take<int32_t>(s.Tm);
  t.s_vt_off = p.take<int32_t>(s.Vs + 1);
  t.s_vt = p.take<int32_t>(3 * s.Ts);
  t.m_vt_off = p.take<int32_t>(s.Vm + 1);
  t.m_vt = p.take<int32_t>(3 * s.Tm);
  t.rule = p.take<double>(kRuleDoubles);
  t.m_opp = p.take<int32_t>(s.feat ? 3 * s.Tm : 0);
  t.area = p.take<char>(rsz * s.Ts);
  t.grid = p.take<GridEnv>(s.n_env);
  t.box = p.take<uint32_t>(6 * s.n_env);
  t.cell_cnt = p.take<int32_t>(cp.grid_cells + 1);
  t.cell_start = p.take<int32_t>(cp.grid_cells + 1);
  t.items = p.take<int32_t>(cp.grid_items);
  t.mbox = p.take<float4>(3 * s.Tm);
  t.cand_cnt = p.take<int32_t>(s.Ts + 1);
  t.cand_off = p.take<int32_t>(s.Ts + 1);
  t.cand = p.take<int32_t>(cp.candidates);
  t.cand_tmp = p.take<int32_t>(cp.candidates);
  t.cand_tmp_off = p.take<int32_t>(s.Ts);
  t.cand_blk = p.take<int32_t>(kQueryBlocks);
  t.qlist = p.take<int32_t>(s.Ts);
  t.qcount = p.take<int32_t>(1);
  t.qrec = p.take<float4>(3 * s.Ts);
  t.slist = p.take<int32_t>(s.n_tiles);
  t.scount = p.take<int32_t>(1);
  t.tflag = p.take<int32_t>(s.n_tiles);
  t.atile = p.take<int32_t>(s.n_tiles);
  t.atile_cnt = p.take<int32_t>(1);
  t.epoch = p.take<uint32_t>(1);
  t.tile_act = p.take<uint32_t>(s.n_tiles);
  t.rec = p.take<char>((s.f64 ? sizeof(Rec<double>) : sizeof(Rec<float>)) * cp.active);
  t.tri_nrm = p.take<char>(rsz * 3 * s.Ts);
  t.tri_sum = p.take<char>(rsz * 9 * s.Ts);
  t.tri_npair = p.take<int32_t>(s.Ts);
  t.tri_poff = p.take<int32_t>(s.Ts);
  t.tri_roff = p.take<int32_t>(s.Ts);
  t.tri_rcnt = p.take<int32_t>(s.Ts);
  t.pair = p.take<char>((s.f64 ? sizeof(Pair<double>) : sizeof(Pair<float>)) * cp.pairs);
  t.tile_E = p.take<double>(s.n_tiles);
  t.mp_cnt = p.take<int32_t>(s.Tm + 1);
  t.mp_off = p.take<int32_t>(s.Tm + 1);
  t.mp_list = p.take<int32_t>(cp.pairs);
  t.mp_key = p.take<long long>(cp.pairs);
  t.mtri = p.take<char>(s.kin ? 0 : rsz * 45 * s.Tm);
  t.row_cnt = p.take<int32_t>(s.V + 1);
  t.rlist = p.take<int4>(2 * s.V);
  t.rcount = p.take<int32_t>(2);
  t.sgrid = p.take<GridEnv>(s.n_env);
  t.sbox = p.take<uint32_t>(6 * s.n_env);
  t.scell_cnt = p.take<int32_t>(cp.grid_cells + 1);
  t.scell_start = p.take<int32_t>(cp.grid_cells + 1);
  t.sitems = p.take<int32_t>(cp.grid_items);
  t.smbox = p.take<float4>(3 * s.Tm);
  t.alpha_bits = p.take<uint32_t>(s.n_env);
  t.hv_tri = p.take<char>(rsz * 3 * s.Ts);
  t.hv_pair = p.take<char>(rsz * 3 * cp.pairs);
  int64_t nmax = std::max<int64_t>({s.Ts + 1, s.Tm + 1, s.V + 1, cp.grid_cells + 1, 1});
  size_t se = (size_t)(2 * (nmax / 1024 + 2) + 2 * 1024 + 64);
  t.scan_tmp = p.take<int32_t>((int64_t)se);
  t.scan_tmp2 = p.take<int32_t>((int64_t)se);
  if (scan_elems) *scan_elems = se;
  if (b) *b = t;
  return p.off + 256;
}

bool caps_ok(const gmcp_caps *c) {
  return c && c->grid_cells > 0 && c->grid_items > 0 && c->candidates > 0 && c->active > 0 &&
         c->pairs > 0 && c->grid_cells < (int64_t(1) << 31) && c->grid_items < (int64_t(1) << 31) &&
         c->candidates < (int64_t(1) << 31) && c->active < (int64_t(1) << 31) &&
         c->pairs < (int64_t(1) << 31);
}

uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

int fail(gmcp_ctx *c, hipError_t e) {
  (void)c;
  return e == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

}  // namespace

namespace gmcp {

void prof_mark(gmcp_ctx *c, int stage, int end) {
  Prof &p = c->prof;
  if (!p.on) return;
  if (!end) {
    // each timed stage takes two consecutive events: start, end
    while (p.pool.size() < p.used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        p.on = false;
        return;
      }
      p.pool.push_back(e);
    }
    p.stage.push_back(stage);
    p.first.push_back(p.used);
    (void)hipEventRecord(p.pool[p.used], c->stream);
    p.used += 2;
  } else if (!p.first.empty()) {
    (void)hipEventRecord(p.pool[p.first.back() + 1], c->stream);
  }
}

}  // namespace gmcp

extern "C" {

size_t gmcp_workspace_size(const gmcp_layout *layout, const gmcp_caps *caps) {
  Sizes s;
  if (!layout_sizes(layout, &s) || !caps_ok(caps)) return 0;
  return plan_workspace(s, *caps, nullptr, nullptr, nullptr);
}

int gmcp_create(gmcp_ctx **out, const gmcp_layout *L, const gmcp_caps *caps, const int32_t *slave_tri,
                const int32_t *master_tri, void *workspace, size_t bytes, void *stream) {
  if (!out) return GMCP_E_ARG;
  *out = nullptr;
  Sizes s;
  if (!layout_sizes(L, &s) || !caps_ok(caps) || !workspace) return GMCP_E_ARG;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return GMCP_E_ARG;
  if ((s.Ts > 0 && !slave_tri) || (s.Tm > 0 && !master_tri)) return GMCP_E_ARG;
  size_t need = plan_workspace(s, *caps, nullptr, nullptr, nullptr);
  if (bytes < need) return GMCP_E_ARG;

  gmcp_ctx *c = new (std::nothrow) gmcp_ctx();
  if (!c) return GMCP_E_ARG;
  c->stream = (hipStream_t)stream;
  c->f64 = s.f64;
  c->kinematic = s.kin;
  c->mortar = (L->flags & GMCP_MORTAR) != 0;
  c->features = s.feat;
  c->n_env = s.n_env;
  c->Vs = s.Vs;
  c->Vm = s.Vm;
  c->Ts = s.Ts;
  c->Tm = s.Tm;
  c->Ns = s.Ns;
  c->V = s.V;
  c->n_tiles = s.n_tiles;
  c->caps = *caps;
  c->ts = slave_tri;
  c->tm = master_tri;
  c->samples_built = false;
  c->broadphase_done = false;
  c->assembled = false;
  c->swept_ready = false;
  c->query_blocks = 0;
  c->query_grid_max = 0;
  c->tune = gmcp_tuning{0, 0, 0, 0};
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      c->n_cu = ncu;
    else
      c->n_cu = 1;
  }
  plan_workspace(s, *caps, (char *)workspace, &c->b, &c->scan_tmp_elems);

  // ---- topology back to the host
  std::vector<int32_t> ts(3 * s.Ts), tm(3 * s.Tm);
  hipError_t e = hipSuccess;
  if (s.Ts) e = hipMemcpy(ts.data(), slave_tri, sizeof(int32_t) * 3 * s.Ts, hipMemcpyDeviceToHost);
  if (e == hipSuccess && s.Tm)
    e = hipMemcpy(tm.data(), master_tri, sizeof(int32_t) * 3 * s.Tm, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    delete c;
    return GMCP_E_HIP;
  }
  // per-environment table and id checks
  c->henv.resize(s.n_env);
  std::vector<int32_t> s_env(s.Ts), m_env(s.Tm), samp_off(s.Ts + 1);
  int64_t weight_tot = 0;
  for (int en = 0; en < s.n_env; ++en)
    weight_tot += (L->slave_t_off[en + 1] - L->slave_t_off[en]) + (L->master_t_off[en + 1] - L->master_t_off[en]);
  int64_t cell0 = 0, samp0 = 0;
  int32_t tile0 = 0;
  for (int en = 0; en < s.n_env; ++en) {
    EnvInfo &v = c->henv[en];
    v.kappa = L->kappa[en];
    v.dhat = L->dhat[en];
    v.delta_T = L->delta_T[en];
    v.cell = L->cell ? L->cell[en] : 0.0;
    v.kappa_e = L->kappa_edge ? L->kappa_edge[en] : 0.0;
    v.kappa_p = L->kappa_point ? L->kappa_point[en] : 0.0;
    v.delta_e = L->delta_e ? L->delta_e[en] : 0.0;
    v.rule_n = L->rule_n[en];
    v.nq = v.rule_n * v.rule_n;
    v.sv0 = L->slave_v_off[en];
    v.sv1 = L->slave_v_off[en + 1];
    v.st0 = L->slave_t_off[en];
    v.st1 = L->slave_t_off[en + 1];
    v.mv0 = L->master_v_off[en];
    v.mv1 = L->master_v_off[en + 1];
    v.mt0 = L->master_t_off[en];
    v.mt1 = L->master_t_off[en + 1];
    int64_t wgt = (v.st1 - v.st0) + (v.mt1 - v.mt0);
    int64_t budget = weight_tot > 0 ? (caps->grid_cells * wgt) / weight_tot : 0;
    if (budget < 1) budget = 1;
    if (cell0 + budget > caps->grid_cells) budget = caps->grid_cells - cell0;
    v.cell0 = cell0;
    v.cell_budget = budget;
    cell0 += budget;
    v.samp0 = samp0;
    int per = kWave / v.nq;
    v.tile0 = tile0;
    tile0 += (v.st1 - v.st0 + per - 1) / per;
    v.tile1 = tile0;
    for (int t = v.st0; t < v.st1; ++t) {
      s_env[t] = en;
      samp_off[t] = (int32_t)samp0;
      samp0 += v.nq;
      for (int j = 0; j < 3; ++j) {
        int32_t id = ts[3 * t + j];
        if (id < v.sv0 || id >= v.sv1) {
          delete c;
          return GMCP_E_ARG;
        }
      }
    }
    for (int t = v.mt0; t < v.mt1; ++t) {
      m_env[t] = en;
      for (int j = 0; j < 3; ++j) {
        int32_t id = tm[3 * t + j];
        if (id < v.mv0 || id >= v.mv1) {
          delete c;
          return GMCP_E_ARG;
        }
      }
    }
  }
  samp_off[s.Ts] = (int32_t)samp0;
  c->total_cells = cell0;
  // environment of every slave vertex that a slave triangle uses (-1: none),
  // so the slave surface's boxes come from a coalesced pass over vertices
  std::vector<int32_t> s_venv(s.Vs, -1);
  for (int64_t t = 0; t < s.Ts; ++t)
    for (int j = 0; j < 3; ++j) s_venv[ts[3 * t + j]] = s_env[t];
  // vertex -> (triangle, corner) adjacency, triangles ascending per vertex
  auto adjacency = [](int64_t V, int64_t T, const std::vector<int32_t> &tri, std::vector<int32_t> &off,
                      std::vector<int32_t> &lst) {
    off.assign(V + 1, 0);
    for (int64_t i = 0; i < 3 * T; ++i) off[tri[i] + 1]++;
    for (int64_t v = 0; v < V; ++v) off[v + 1] += off[v];
    lst.resize(3 * T);
    std::vector<int32_t> cur(off.begin(), off.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int j = 0; j < 3; ++j) lst[cur[tri[3 * t + j]]++] = (int32_t)(t * 4 + j);
  };
  std::vector<int32_t> svo, svt, mvo, mvt;
  adjacency(s.Vs, s.Ts, ts, svo, svt);
  adjacency(s.Vm, s.Tm, tm, mvo, mvt);
  std::vector<double> rule(kRuleDoubles);
  build_rules(rule.data());

  auto up = [&](void *dst, const void *src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpy(dst, src, n, hipMemcpyHostToDevice);
  };
  up(c->b.env, c->henv.data(), sizeof(EnvInfo) * s.n_env);
  up(c->b.samp_off, samp_off.data(), sizeof(int32_t) * (s.Ts + 1));
  up(c->b.s_env, s_env.data(), sizeof(int32_t) * s.Ts);
  up(c->b.s_venv, s_venv.data(), sizeof(int32_t) * s.Vs);
  up(c->b.m_env, m_env.data(), sizeof(int32_t) * s.Tm);
  up(c->b.s_vt_off, svo.data(), sizeof(int32_t) * (s.Vs + 1));
  up(c->b.s_vt, svt.data(), sizeof(int32_t) * 3 * s.Ts);
  up(c->b.m_vt_off, mvo.data(), sizeof(int32_t) * (s.Vm + 1));
  up(c->b.m_vt, mvt.data(), sizeof(int32_t) * 3 * s.Tm);
  up(c->b.rule, rule.data(), sizeof(double) * rule.size());
  if (s.feat && s.Tm) {
    // triangle across each master edge (manifold edges; -1 on the boundary)
    std::vector<int32_t> opp(3 * s.Tm, -1);
    std::map<std::pair<int32_t, int32_t>, int64_t> edge;
    for (int64_t t = 0; t < s.Tm; ++t)
      for (int k = 0; k < 3; ++k) {
        int32_t a = tm[3 * t + k], b = tm[3 * t + (k + 1) % 3];
        auto key = std::make_pair(std::min(a, b), std::max(a, b));
        auto it = edge.find(key);
        if (it == edge.end()) {
          edge.emplace(key, 3 * t + k);
        } else {
          opp[3 * t + k] = (int32_t)(it->second / 3);
          opp[it->second] = (int32_t)t;
        }
      }
    up(c->b.m_opp, opp.data(), sizeof(int32_t) * opp.size());
  }
  DevStatus st{};
  st.index = ~0ull;
  up(c->b.status, &st, sizeof(st));
  if (e != hipSuccess) {
    delete c;
    return GMCP_E_HIP;
  }
  // zeroed counters the broad phase and bucketing rely on
  if (fill_i32(c, c->b.cell_cnt, 0, caps->grid_cells + 1) != hipSuccess ||
      fill_i32(c, c->b.scell_cnt, 0, caps->grid_cells + 1) != hipSuccess ||
      fill_i32(c, c->b.mp_cnt, 0, s.Tm + 1) != hipSuccess ||
      fill_i32(c, c->b.scan_tmp, 0, (int64_t)c->scan_tmp_elems) != hipSuccess ||
      fill_i32(c, c->b.tflag, 0, s.n_tiles) != hipSuccess ||
      fill_i32(c, reinterpret_cast<int32_t *>(c->b.epoch), 0, 1) != hipSuccess ||
      fill_i32(c, reinterpret_cast<int32_t *>(c->b.tile_act), 0, s.n_tiles) != hipSuccess ||
      fill_i32(c, c->b.scan_tmp2, 0, (int64_t)c->scan_tmp_elems) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    delete c;
    return GMCP_E_HIP;
  }
  {  // the static slave boxes start empty (each broad phase empties them for the next)
    gmcp::StageInit si;
    si.box = c->b.box;
    if (gmcp::stage_init(c, si) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
      delete c;
      return GMCP_E_HIP;
    }
  }
  c->side = nullptr;
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess) {
    if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(c->side);
      c->side = nullptr;
    } else if (hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
      (void)hipEventDestroy(c->ev_fork);
      (void)hipStreamDestroy(c->side);
      c->side = nullptr;
    }
  } else {
    c->side = nullptr;
  }
  *out = c;
  return GMCP_OK;
}

void gmcp_destroy(gmcp_ctx *c) {
  if (!c) return;
  for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipEventDestroy(c->ev_fork);
    (void)hipEventDestroy(c->ev_join);
    (void)hipStreamDestroy(c->side);
  }
  delete c;
}

int gmcp_set_stream(gmcp_ctx *c, void *stream) {
  if (!c) return GMCP_E_ARG;
  c->stream = (hipStream_t)stream;
  return GMCP_OK;
}

int gmcp_set_tuning(gmcp_ctx *c, const gmcp_tuning *t) {
  if (!c || !t) return GMCP_E_ARG;
  const int lb = t->light_row_bound;
  if (t->query_blocks < 0 || t->query_blocks > gmcp::kQueryBlocks) return GMCP_E_ARG;
  if (lb != 0 && lb != 32 && lb != 64 && lb != 128 && lb != 256) return GMCP_E_ARG;
  if (t->light_row_blocks < 0 || t->light_row_blocks > (1 << 20)) return GMCP_E_ARG;
  if (t->heavy_row_blocks < 0 || t->heavy_row_blocks > 65536) return GMCP_E_ARG;
  c->tune = *t;
  return GMCP_OK;
}

int gmcp_get_tuning(const gmcp_ctx *c, gmcp_tuning *t) {
  if (!c || !t) return GMCP_E_ARG;
  t->query_blocks = c->tune.query_blocks ? c->tune.query_blocks : (int32_t)c->query_grid_max;
  t->light_row_bound = gmcp::light_row_bound(c);
  t->light_row_blocks = gmcp::light_row_blocks(c);
  t->heavy_row_blocks = gmcp::heavy_row_blocks(c);
  return GMCP_OK;
}

int64_t gmcp_num_samples(const gmcp_ctx *c) { return c ? c->Ns : -1; }

int gmcp_rule(int n, double *out) {
  if (n < 1 || n > kMaxRule || !out) return GMCP_E_ARG;
  std::vector<double> rule(kRuleDoubles);
  build_rules(rule.data());
  memcpy(out, rule.data() + (n - 1) * 16 * 3, sizeof(double) * 3 * n * n);
  return GMCP_OK;
}

int gmcp_build_samples(gmcp_ctx *c, const void *x_rest, void *weights) {
  if (!c || !x_rest) return GMCP_E_ARG;
  hipError_t e = c->f64 ? launch_rest_area<double>(c, (const double *)x_rest, (double *)weights)
                        : launch_rest_area<float>(c, (const float *)x_rest, (float *)weights);
  if (e != hipSuccess) return GMCP_E_HIP;
  // Morton-ordered work tiles from the rest centroids
  size_t rsz = c->f64 ? 8 : 4;
  std::vector<char> xb(rsz * 3 * c->Vs);
  std::vector<int32_t> ts(3 * c->Ts);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return GMCP_E_HIP;
  if (c->Vs && hipMemcpy(xb.data(), x_rest, rsz * 3 * c->Vs, hipMemcpyDeviceToHost) != hipSuccess)
    return GMCP_E_HIP;
  if (c->Ts && hipMemcpy(ts.data(), c->ts, sizeof(int32_t) * 3 * c->Ts, hipMemcpyDeviceToHost) != hipSuccess)
    return GMCP_E_HIP;
  auto X = [&](int64_t v, int d) -> double {
    return c->f64 ? ((const double *)xb.data())[3 * v + d] : (double)((const float *)xb.data())[3 * v + d];
  };
  std::vector<int32_t> order(c->Ts);
  std::vector<Tile> tiles(c->n_tiles);
  for (int en = 0; en < c->n_env; ++en) {
    const EnvInfo &v = c->henv[en];
    int64_t n = v.st1 - v.st0;
    if (n <= 0) continue;
    std::vector<double> cen(3 * n);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d) {
        int64_t t = v.st0 + i;
        double m = (X(ts[3 * t], d) + X(ts[3 * t + 1], d) + X(ts[3 * t + 2], d)) / 3.0;
        cen[3 * i + d] = m;
        lo[d] = std::min(lo[d], m);
        hi[d] = std::max(hi[d], m);
      }
    double span = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-30});
    std::vector<std::pair<uint32_t, int32_t>> key(n);
    for (int64_t i = 0; i < n; ++i) {
      uint32_t code = 0;
      for (int d = 0; d < 3; ++d) {
        double f = (cen[3 * i + d] - lo[d]) / span;
        uint32_t q = (uint32_t)std::min(1023.0, std::max(0.0, floor(f * 1024.0)));
        code |= spread3(q) << d;
      }
      key[i] = {code, (int32_t)(v.st0 + i)};
    }
    std::sort(key.begin(), key.end());
    for (int64_t i = 0; i < n; ++i) order[v.st0 + i] = key[i].second;
    int per = kWave / v.nq;
    for (int32_t tl = v.tile0; tl < v.tile1; ++tl) {
      int64_t first = v.st0 + (int64_t)(tl - v.tile0) * per;
      tiles[tl].first = (int32_t)first;
      tiles[tl].count = (int32_t)std::min<int64_t>(per, v.st1 - first);
      tiles[tl].env = en;
      tiles[tl].nq = v.nq;
    }
  }
  if (c->Ts && hipMemcpy(c->b.s_order, order.data(), sizeof(int32_t) * c->Ts, hipMemcpyHostToDevice) != hipSuccess)
    return GMCP_E_HIP;
  if (c->n_tiles && hipMemcpy(c->b.tiles, tiles.data(), sizeof(Tile) * c->n_tiles, hipMemcpyHostToDevice) != hipSuccess)
    return GMCP_E_HIP;
  c->samples_built = true;
  return GMCP_OK;
}

int gmcp_broadphase(gmcp_ctx *c, const void *xs, const void *xm) {
  if (!c || !xs || (c->Tm > 0 && !xm) || !c->samples_built) return GMCP_E_ARG;
  hipError_t e = c->f64 ? launch_broadphase<double>(c, (const double *)xs, (const double *)xm)
                        : launch_broadphase<float>(c, (const float *)xs, (const float *)xm);
  if (e == hipSuccess) c->broadphase_done = true;
  return fail(c, e);
}

int gmcp_assemble(gmcp_ctx *c, const void *xs, const void *xm, const void *g_ref, const void *dgap,
                  void *energy, void *grad, const gmcp_bsr *H) {
  if (!c || !xs || (c->Tm > 0 && !xm) || !energy || !c->samples_built || !c->broadphase_done)
    return GMCP_E_ARG;
  if (c->mortar && dgap) return GMCP_E_ARG;  // clipped samples have no fixed ids (g_ref: one per slave triangle)
  if (H && (!H->row_ptr || (H->cap_nnzb > 0 && (!H->col || !H->val)) || H->cap_nnzb < 0 ||
            H->cap_nnzb >= (int64_t(1) << 31)))
    return GMCP_E_ARG;
  hipError_t e = c->f64 ? launch_assemble<double>(c, (const double *)xs, (const double *)xm,
                                                  (const double *)g_ref, (const double *)dgap,
                                                  (double *)energy, (double *)grad, H)
                        : launch_assemble<float>(c, (const float *)xs, (const float *)xm, (const float *)g_ref,
                                                 (const float *)dgap, (float *)energy, (float *)grad, H);
  if (e == hipSuccess) c->assembled = true;
  return fail(c, e);
}

int gmcp_ccd_step(gmcp_ctx *c, const void *xs, const void *xm, const void *dxs, const void *dxm,
                  void *alpha) {
  if (!c || !xs || (c->Tm > 0 && !xm) || !dxs || !alpha || !c->assembled) return GMCP_E_ARG;
  hipError_t e = c->f64 ? launch_ccd<double>(c, (const double *)xs, (const double *)xm, (const double *)dxs,
                                             (const double *)dxm, (double *)alpha)
                        : launch_ccd<float>(c, (const float *)xs, (const float *)xm, (const float *)dxs,
                                            (const float *)dxm, (float *)alpha);
  return fail(c, e);
}

int gmcp_ccd_swept(gmcp_ctx *c, const void *xs, const void *xm, const void *dxs, const void *dxm) {
  if (!c || !xs || (c->Tm > 0 && !xm) || !dxs || !c->samples_built) return GMCP_E_ARG;
  hipError_t e = c->f64 ? launch_ccd_swept<double>(c, (const double *)xs, (const double *)xm, (const double *)dxs,
                                                   (const double *)dxm)
                        : launch_ccd_swept<float>(c, (const float *)xs, (const float *)xm, (const float *)dxs,
                                                  (const float *)dxm);
  c->swept_ready = e == hipSuccess;
  return fail(c, e);
}

int gmcp_ccd_finish(gmcp_ctx *c, const void *dxs, const void *dxm, void *alpha) {
  if (!c || !dxs || !alpha || !c->assembled || !c->swept_ready) return GMCP_E_ARG;
  c->swept_ready = false;
  hipError_t e = c->f64 ? launch_ccd_finish<double>(c, (const double *)dxs, (const double *)dxm, (double *)alpha)
                        : launch_ccd_finish<float>(c, (const float *)dxs, (const float *)dxm, (float *)alpha);
  return fail(c, e);
}

int gmcp_hvp(gmcp_ctx *c, const void *vx, const void *vd, void *ox, void *od) {
  if (!c || !vx || !ox || !c->assembled) return GMCP_E_ARG;
  if (c->mortar && (vd || od)) return GMCP_E_ARG;
  hipError_t e = c->f64 ? launch_hvp<double>(c, (const double *)vx, (const double *)vd, (double *)ox, (double *)od)
                        : launch_hvp<float>(c, (const float *)vx, (const float *)vd, (float *)ox, (float *)od);
  return fail(c, e);
}

int gmcp_energy_frozen(gmcp_ctx *c, const void *xs, const void *xm, void *energy) {
  if (!c || !xs || !xm || !energy || !c->assembled) return GMCP_E_ARG;
  hipError_t e = c->f64 ? launch_energy_frozen<double>(c, (const double *)xs, (const double *)xm, (double *)energy)
                        : launch_energy_frozen<float>(c, (const float *)xs, (const float *)xm, (float *)energy);
  return fail(c, e);
}

int gmcp_sample_results(gmcp_ctx *c, int32_t *M, void *g, void *bm, void *c1, void *c2, void *p) {
  if (!c || !c->assembled || c->mortar) return GMCP_E_ARG;
  hipError_t e = c->f64 ? launch_sample_results<double>(c, M, (double *)g, (double *)bm, (double *)c1,
                                                        (double *)c2, (double *)p)
                        : launch_sample_results<float>(c, M, (float *)g, (float *)bm, (float *)c1, (float *)c2,
                                                       (float *)p);
  return fail(c, e);
}

int gmcp_pairs(gmcp_ctx *c, int32_t *T, int32_t *M, int64_t cap) {
  if (!c || !T || !M || cap < 0 || !c->assembled) return GMCP_E_ARG;
  hipError_t e = c->f64 ? launch_pair_export<double>(c, T, M, cap) : launch_pair_export<float>(c, T, M, cap);
  return fail(c, e);
}

int gmcp_candidates(gmcp_ctx *c, int32_t *cand_off, int32_t *cand, int64_t cap) {
  if (!c || !cand_off || !c->broadphase_done) return GMCP_E_ARG;
  hipError_t e = build_candidate_csr(c);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cand_off, c->b.cand_off, sizeof(int32_t) * (c->Ts + 1), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && cand && cap > 0) {
    int64_t n = std::min<int64_t>(cap, c->caps.candidates);
    e = hipMemcpyAsync(cand, c->b.cand, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c->stream);
  }
  return fail(c, e);
}

int gmcp_status(gmcp_ctx *c, gmcp_status_info *info) {
  if (!c || !info) return GMCP_E_ARG;
  DevStatus st;
  if (hipMemcpyAsync(&st, c->b.status, sizeof(st), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return GMCP_E_HIP;
  memset(info, 0, sizeof(*info));
  info->code = st.code;
  info->index = st.index == ~0ull ? -1 : (int64_t)st.index;
  info->n_active = (int64_t)st.n_active;
  info->n_pairs = (int64_t)st.n_pairs;
  info->nnzb = (int64_t)st.nnzb;
  // candidates: the query blocks' totals (no single-address atomics in the query)
  int64_t ncand = 0;
  if (c->query_blocks > 0) {
    std::vector<int32_t> blk(c->query_blocks);
    if (hipMemcpyAsync(blk.data(), c->b.cand_blk, sizeof(int32_t) * blk.size(), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return GMCP_E_HIP;
    for (int32_t v : blk) ncand += v;
  }
  info->n_candidates = ncand;
  info->n_swept = (int64_t)st.n_swept;
  info->need.grid_cells = c->caps.grid_cells;
  // the counters are complete totals even when a buffer overflowed
  info->need.grid_items = std::max<int64_t>((int64_t)st.need_items, 0);
  info->need.candidates = std::max<int64_t>((int64_t)st.need_cand, ncand);
  info->need.active = (int64_t)st.n_active;
  info->need.pairs = (int64_t)st.n_pairs;
  info->need.row_entries = (int64_t)st.need_row;
  // clear the sticky error
  DevStatus clr = st;
  clr.code = 0;
  clr.index = ~0ull;
  clr.need_items = clr.need_cand = clr.need_active = clr.need_pairs = clr.need_row = 0;
  if (hipMemcpy(c->b.status, &clr, sizeof(clr), hipMemcpyHostToDevice) != hipSuccess) return GMCP_E_HIP;
  return GMCP_OK;
}

static const char *kStageNames[gmcp::ST_COUNT] = {
    "grid_build", "query", "cand_move", "narrow",     "pair_bucket", "grad_rows",
    "rows_count", "rows_fill",   "ccd_linear", "ccd_grid",   "ccd_accd",  "master_tri_sums", "rows_copy", "query_pre", "rows_pre", "rows_count_heavy", "rows_fill_heavy"};

int gmcp_profile(gmcp_ctx *c, int enable) {
  if (!c) return GMCP_E_ARG;
  c->prof.on = enable != 0;
  if (enable) {
    c->prof.used = 0;
    c->prof.stage.clear();
    c->prof.first.clear();
  }
  return GMCP_OK;
}

int gmcp_profile_stages(void) { return gmcp::ST_COUNT; }

const char *gmcp_profile_stage_name(int s) { return (s >= 0 && s < gmcp::ST_COUNT) ? kStageNames[s] : ""; }

int gmcp_profile_read(gmcp_ctx *c, double *ms, int64_t *count) {
  if (!c || !ms || !count) return GMCP_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return GMCP_E_HIP;
  for (int s = 0; s < gmcp::ST_COUNT; ++s) {
    ms[s] = 0.0;
    count[s] = 0;
  }
  for (size_t i = 0; i < c->prof.stage.size(); ++i) {
    float t = 0.0f;
    size_t f = c->prof.first[i];
    if (hipEventElapsedTime(&t, c->prof.pool[f], c->prof.pool[f + 1]) != hipSuccess) continue;
    ms[c->prof.stage[i]] += t;
    count[c->prof.stage[i]] += 1;
  }
  return GMCP_OK;
}

int gmcp_row_classes(gmcp_ctx *c, int64_t *out, const int32_t *row_ptr) {
  if (!c || !out || !row_ptr || !c->assembled) return GMCP_E_ARG;
  int32_t h[2];
  if (hipMemcpyAsync(h, c->b.rcount, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return GMCP_E_HIP;
  std::vector<int4> rl((size_t)h[0] + h[1]);
  std::vector<int32_t> rp(c->V + 1);
  if ((h[0] && hipMemcpy(rl.data(), c->b.rlist, sizeof(int4) * h[0], hipMemcpyDeviceToHost) != hipSuccess) ||
      (h[1] && hipMemcpy(rl.data() + h[0], c->b.rlist + c->V, sizeof(int4) * h[1], hipMemcpyDeviceToHost) !=
                   hipSuccess) ||
      hipMemcpy(rp.data(), row_ptr, sizeof(int32_t) * (c->V + 1), hipMemcpyDeviceToHost) != hipSuccess)
    return GMCP_E_HIP;
  int64_t nb[2] = {0, 0};
  for (int64_t i = 0; i < (int64_t)rl.size(); ++i) {
    const int32_t r = rl[i].x;
    if (r < 0 || r >= c->V) return GMCP_E_HIP;
    nb[i < h[0] ? 0 : 1] += rp[r + 1] - rp[r];
  }
  out[0] = h[0];
  out[1] = h[1];
  out[2] = nb[0];
  out[3] = nb[1];
  return GMCP_OK;
}

const char *gmcp_strerror(int code) {
  switch (code) {
    case GMCP_OK: return "ok";
    case GMCP_E_ARG: return "invalid argument";
    case GMCP_E_CAPACITY: return "workspace capacity exceeded";
    case GMCP_E_PENETRATION: return "penetration: an inside opposing hit with non-positive gap";
    case GMCP_E_DEGENERATE: return "degenerate slave triangle";
    case GMCP_E_NONFINITE: return "non-finite input";
    case GMCP_E_HIP: return "HIP runtime error";
    case GMCP_E_TIMEOUT: return "a device-side wait passed its bound (internal error)";
    default: return "unknown status";
  }
}

}  // extern "C"
