// Internal declarations of the GMCP HIP library (gfx950 only).
//
// Device-side data layout (all carved from the caller's workspace):
//   static   - rules, per-environment parameters, Morton-ordered work tiles,
//              vertex->triangle adjacency of both meshes, rest areas;
//   per call - broad-phase grid and candidate lists, active-sample records,
//              per-slave-triangle sums, contact pairs, pairs bucketed by
//              master triangle, BSR row counts, step-bound scratch, status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/gmcp.h"

namespace gmcp {

constexpr int kWave = 64;
constexpr int kMaxRule = 4;            // n <= 4  => <= 16 samples per triangle
constexpr int kRuleDoubles = kMaxRule * 16 * 3 + kMaxRule * 4 * 2;  // 2D rules, then 1D Gauss-Legendre
constexpr int kGaussOff = kMaxRule * 16 * 3;
constexpr int kQueryBlocks = 2048;  // largest grid of the list-walking query (its per-block candidate slots)
constexpr int kTilePerBlock = 4;       // narrow phase: 4 waves, one tile each

// ---------------------------------------------------------------- status
struct DevStatus {
  int32_t code;
  int32_t pad;
  unsigned long long index;  // min offending id (atomicMin), ~0ull if none
  unsigned long long n_active, n_pairs, nnzb, n_cand, n_swept;
  unsigned long long need_items, need_cand, need_active, need_pairs, need_row;
  unsigned long long mortar_alloc;  // clipped samples: pairs << 32 | records, one atomic per triangle
};

// --------------------------------------------------------- per environment
struct EnvInfo {
  double kappa, dhat, delta_T, cell;
  double kappa_e, kappa_p, delta_e;  // edge / point samples (GMCP_FEATURES)
  int32_t rule_n, nq;
  int32_t sv0, sv1, st0, st1;   // slave vertex / triangle ranges
  int32_t mv0, mv1, mt0, mt1;   // master ranges
  int64_t cell0, cell_budget;   // grid cell slice [cell0, cell0 + budget)
  int64_t samp0;                // first sample id
  int32_t tile0, tile1;         // work tiles of this environment
};

struct GridEnv {           // one environment's uniform grid for this call
  float lo[3];
  float h, inv_h;
  int32_t nx, ny, nz;
  int32_t valid;
};

struct Tile {              // narrow-phase work item: tris [first, first+count) of s_order
  int32_t first, count, env, nq;
};

template <typename R>
struct Rec {               // active sample record
  int32_t k, M, T, q;      // sample id (-1 for clipped mortar samples), master / slave triangle, rule point
  R g, b0, b1, b2;         // gap, master barycentrics
  R c1, c2, p, eps;        // kappa w gamma B', clamped kappa w gamma B'', pressure, support radius
  R s1, s2, kwg, pad;      // slave barycentrics beta^s_1, beta^s_2; kappa w gamma
};

template <typename R>
struct Pair {              // one (slave triangle, master triangle) contact
  int32_t T, M;
  int32_t mv[3];           // M's vertex ids (saves the row kernels a dependent gather)
  R mm[6];   // sum c2 bm_i bm_j           (sym, order 00 01 02 11 12 22)
  R sm[9];   // sum -c2 bs_a bm_j          (a-major)
  R gm[3];   // sum c1 bm_j
};

// ----------------------------------------------------------------- context
struct Buffers {
  // static
  EnvInfo *env;
  Tile *tiles;
  int32_t *s_order, *samp_off, *s_env, *m_env;
  int32_t *s_venv;                              // [Vs]: environment of a slave vertex on a slave triangle, else -1
  int32_t *s_vt_off, *s_vt, *m_vt_off, *m_vt;   // vt entries: tri*4 + corner
  double *rule;                                 // [4][16][3] xi, eta, w; then [4][4][2] 1D Gauss-Legendre
  int32_t *m_opp;                               // [Tm][3] triangle across edge k of a master triangle, -1
  void *area;                                   // [Ts] R
  // broad phase
  GridEnv *grid;
  uint32_t *box;                                // [n_env][6] ordered-float bits
  int32_t *cell_cnt, *cell_start, *items;
  float4 *mbox;                                 // [Tm][3]: lo, hi, unit normal
  int32_t *cand_cnt, *cand_off, *cand;
  int32_t *cand_tmp, *cand_tmp_off;             // one-pass query: scratch lists and their offsets
  int32_t *cand_blk;                            // [kQueryBlocks] candidates found by each query block
  int32_t *qlist, *qcount;                      // [Ts], [1]: slave triangles whose prism meets occupied cells
  float4 *qrec;                                 // [Ts][3]: their frames (box lo | T, box hi | env, normal)
  int32_t *slist, *scount;                      // [n_tiles], [1]: work tiles whose swept boxes meet occupied cells
  int32_t *tflag;                               // [n_tiles]: tile listed (zero between calls)
  int32_t *atile, *atile_cnt;                   // [n_tiles], [1]: tiles with selected samples (last assembly)
  uint32_t *epoch;                              // [1]: broad phases so far (marks the active tiles)
  uint32_t *tile_act;                           // [n_tiles]: the epoch of the last broad phase that listed a triangle of the tile
  // narrow / assembly
  void *rec;                                    // Rec<R>[cap.active]
  void *tri_nrm;                                // [Ts][3] R
  void *tri_sum;                                // [Ts][9] R: ss[6], gs[3]
  int32_t *tri_npair, *tri_poff, *tri_roff, *tri_rcnt;
  void *pair;                                   // Pair<R>[cap.pairs]
  double *tile_E;
  int32_t *mp_cnt, *mp_off, *mp_list;
  long long *mp_key;                            // [pairs] (slave triangle << 32 | pair)
  void *mtri;                                   // [Tm][45] R: per master triangle, sum over its
                                                // pairs of mm n n^T (6 vertex pairs x 6) and gm n (3 x 3)
  int32_t *row_cnt;                             // [V+1]
  int4 *rlist;                                  // [2V]: BSR rows with contributions (light | heavy):
                                                //   row, adjacency range [first, end), contributions
  int32_t *rcount;                              // [2]: list lengths
  // step bound
  GridEnv *sgrid;
  uint32_t *sbox;
  int32_t *scell_cnt, *scell_start, *sitems;
  float4 *smbox;                                // [Tm][3]: swept lo, hi, (unused)
  uint32_t *alpha_bits;                         // [n_env]
  // hvp
  void *hv_tri;                                 // [Ts][3] R
  void *hv_pair;                                // [pairs][3] R
  // scan scratch
  int32_t *scan_tmp;
  int32_t *scan_tmp2;                           // the swept grid's scans (second stream)
  DevStatus *status;
};

// kernel stages timed by the optional event profiler (gmcp_profile)
// (stages marked "kernel" bracket exactly one kernel launch)
enum Stage {
  ST_GRID = 0,     // grid build (boxes, counts, scan, placement)
  ST_QUERY_COUNT,  // kernel k_query (one pass: sets, sorted scratch lists)
  ST_QUERY_FILL,   // kernel k_cand_move (scratch lists to the CSR)
  ST_NARROW,       // kernel k_narrow: narrow phase + barrier + sums
  ST_BUCKET,       // pairs bucketed by master triangle (count, scan, place, sort)
  ST_GRAD,         // kernel k_grad: gradient rows
  ST_ROWS_COUNT,   // kernel k_rows, counting pass (light rows)
  ST_ROWS_FILL,    // kernel k_rows, writing pass (light rows)
  ST_CCD_LINEAR,   // kernel k_ccd_linear
  ST_CCD_GRID,     // swept grid build
  ST_CCD_ACCD,     // kernel k_ccd_accd
  ST_MTRI,         // kernel k_mtri: per-master-triangle Hessian blocks and gradient
  ST_ROWS_COPY,    // kernel k_rows, master rows' slave columns copied from the slave rows
  ST_QUERY_PRE,    // kernel k_query_pre: frame checks, prism boxes, query list
  ST_ROWS_PRE,     // kernel k_row_pre: list of rows with contributions
  ST_ROWS_COUNT_H, // kernel k_rows, counting pass, heavy rows
  ST_ROWS_FILL_H,  // kernel k_rows, writing pass, heavy rows
  ST_COUNT
};

struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<int> stage;          // per recorded pair
  std::vector<size_t> first;       // index of the start event in pool
};

}  // namespace gmcp

struct gmcp_ctx {
  gmcp::Prof prof;
  hipStream_t stream;
  // the library's second stream (default priority) and its fork / join
  // events: independent launches of one call overlap (forked from and
  // joined back into `stream`, so the caller sees one stream, also under
  // graph capture); null if creation failed (then everything runs in order)
  hipStream_t side;
  hipEvent_t ev_fork, ev_join;
  bool f64, kinematic, mortar, features;
  int n_env;
  int64_t Vs, Vm, Ts, Tm, Ns, V, n_tiles, total_cells;
  gmcp_caps caps;
  const int32_t *ts, *tm;
  std::vector<gmcp::EnvInfo> henv;
  bool samples_built, broadphase_done, assembled;
  bool swept_ready;  // gmcp_ccd_swept enqueued, gmcp_ccd_finish not yet
  int query_blocks;  // grid of the last query (its entries of b.cand_blk are valid)
  int n_cu;          // compute units of the context's device
  int64_t query_grid_max;  // resident query blocks (0 until the first broad phase)
  gmcp_tuning tune;        // launch shapes (gmcp_set_tuning; zeros = defaults)
  gmcp::Buffers b;
  size_t scan_tmp_elems;
};

namespace gmcp {

// Blocks of `kernel` (threads per block, dynamic LDS bytes) resident on the
// device at once, at least one per compute unit.  A kernel that walks a
// work list with a fixed grid sizes it by this when it has the device to
// itself: blocks beyond it would start only as the first ones finish and
// walk their share of the list alone.
template <typename K>
inline int64_t resident_blocks(const gmcp_ctx *c, K kernel, int threads, size_t lds) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  return (int64_t)per_cu * (c->n_cu > 0 ? c->n_cu : 1);
}

// launch shapes in effect (gmcp_tuning, defaults for zeros)
constexpr int kDefaultLightBound = 128;   // column insertions of a light BSR row
constexpr int kDefaultRowBlocks = 65536;  // light-row grid
constexpr int kDefaultHeavyBlocks = 2048; // heavy-row grid
inline int light_row_bound(const gmcp_ctx *c) {
  return c->tune.light_row_bound ? c->tune.light_row_bound : kDefaultLightBound;
}
inline int light_row_blocks(const gmcp_ctx *c) {
  return c->tune.light_row_blocks ? c->tune.light_row_blocks : kDefaultRowBlocks;
}
inline int heavy_row_blocks(const gmcp_ctx *c) {
  return c->tune.heavy_row_blocks ? c->tune.heavy_row_blocks : kDefaultHeavyBlocks;
}

// ------------------------------------------------------------ launchers
// each returns hipSuccess or the launch error
// side = true uses the second scratch (the swept grid's scans may run on
// another stream, concurrently with the broad phase and assembly)
// grid: the environments' grids of a cell-count scan (only their used cells
// and the total get valid starts), nullptr for a plain scan
hipError_t scan_exclusive(gmcp_ctx *c, const int32_t *in, int32_t *out, int64_t n, bool side = false,
                          const GridEnv *grid = nullptr);
hipError_t fill_i32(gmcp_ctx *c, int32_t *p, int32_t v, int64_t n);
// one launch for a stage's scalar set-up: the status fields of the stage
// (which: 1 broad phase, 2 assembly, 4 step bound), empty boxes and +inf
// step-bound bits per environment, and a few words set to zero
struct StageInit {
  int which = 0;
  uint32_t *box = nullptr;
  uint32_t *alpha = nullptr;
  int32_t *zero[3] = {nullptr, nullptr, nullptr};
  int nzero[3] = {0, 0, 0};  // <= 64 words each
};
hipError_t stage_init(gmcp_ctx *c, const StageInit &a);
// event profiler: prof_mark(c, s, 0) before a stage's launches, (c, s, 1) after
void prof_mark(gmcp_ctx *c, int stage, int end);

template <typename R> hipError_t launch_rest_area(gmcp_ctx *c, const R *x_rest, R *weights);
template <typename R> hipError_t launch_broadphase(gmcp_ctx *c, const R *xs, const R *xm);
// the candidate lists of the last broad phase as a CSR (cand_off, cand), for export
hipError_t build_candidate_csr(gmcp_ctx *c);
// grid over master triangles per environment; swept != 0 uses the boxes of
// the motion x -> x + dx (domain: slave swept box) instead of the prism region
template <typename R>
hipError_t build_grid(gmcp_ctx *c, const R *xs, const R *xm, const R *dxs, const R *dxm, bool swept);
template <typename R>
hipError_t launch_assemble(gmcp_ctx *c, const R *xs, const R *xm, const R *g_ref, const R *dgap,
                           R *energy, R *grad, const gmcp_bsr *H);
template <typename R>
hipError_t launch_ccd(gmcp_ctx *c, const R *xs, const R *xm, const R *dxs, const R *dxm, R *alpha);
// the step bound in two parts: swept grid + additive CCD (needs only the
// samples), then Eq. (ccd) over the assembled samples + the final bound
template <typename R>
hipError_t launch_ccd_swept(gmcp_ctx *c, const R *xs, const R *xm, const R *dxs, const R *dxm);
template <typename R>
hipError_t launch_ccd_finish(gmcp_ctx *c, const R *dxs, const R *dxm, R *alpha);
template <typename R>
hipError_t launch_hvp(gmcp_ctx *c, const R *vx, const R *vd, R *ox, R *od);
template <typename R>
hipError_t launch_energy_frozen(gmcp_ctx *c, const R *xs, const R *xm, R *energy);
template <typename R>
hipError_t launch_sample_results(gmcp_ctx *c, int32_t *M, R *g, R *bm, R *c1, R *c2, R *p);
template <typename R>
hipError_t launch_pair_export(gmcp_ctx *c, int32_t *T, int32_t *M, int64_t cap);

// ---------------------------------------------------------- device utils
__device__ inline uint32_t float_to_ordered(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ordered_to_float(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ inline void set_error(DevStatus *st, int code, unsigned long long index) {
  atomicCAS(&st->code, 0, code);
  atomicMin(&st->index, index);
}

// xcd-aware block index: hardware dispatches consecutive blocks round-robin
// over the 8 XCDs; this makes consecutive logical blocks land on one XCD so
// neighbouring (Morton-adjacent) work shares that XCD's L2.
__device__ inline int xcd_block(int bid, int nblocks) {
  constexpr int kXcd = 8;
  int per = (nblocks + kXcd - 1) / kXcd;
  int x = bid % kXcd, i = bid / kXcd;
  int full = nblocks % kXcd;  // XCDs 0..full-1 get `per` blocks, others per-1
  if (full == 0) return x * per + i;
  if (x < full) return x * per + i;
  return full * per + (x - full) * (per - 1) + i;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP lane moves
// (VALU operations, no LDS round trips): shifts by 1, 2, 4 and 8 lanes
// within each row of 16 scan the rows; then the last lane of row 0 is added
// to row 1 and that of row 2 to row 3 (row broadcast 15, rows 1 and 3
// enabled), then the last lane of row 1 to rows 2 and 3 (row broadcast 31,
// rows 2 and 3 enabled).  A lane whose source is outside its row, or whose
// row is not enabled, adds 0.  Every lane of the wave must be active.
__device__ inline int wave_incl_add(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

}  // namespace gmcp
