/*
 * gmcp.h - C ABI of the GMCP hot path for AMD Instinct MI355X (gfx950).
 *
 * The Geometric Mortar Contact Potential (IsaacIPC paper, Sec. 4) puts a
 * barrier potential on contact samples of a tactile (slave) surface:
 *
 *   Psi = sum_k kappa w_k gamma_k B(g_k, eps_k)            Eq. (gmcp_potential)
 *
 * with w_k the sample's share of slave area, g_k the signed gap along the
 * slave normal to the opposing (master) triangle (Eq. (gap)), gamma_k the
 * master-face weight (Eq. (gamma), face branch), eps_k the support radius
 * (Eq. (adaptive_eps)) and B the IPC log barrier.  This library evaluates,
 * for every sample: the closest opposing master triangle within eps_k, the
 * energy, gradient and PSD Hessian (Sec. 4.2), scattered into a 3x3 block
 * sparse (BSR) Newton system, and the step bound that caps the line search
 * (Eqs. (ccd), (global_ccd), plus additive CCD over swept sample/triangle
 * pairs).
 *
 * Samples.  Every slave triangle carries n*n face samples (n = rule_n, 1..4)
 * from the Stroud conical-product rule: (xi, eta) = (u_i, v_j (1 - u_i))
 * with u_i Gauss-Jacobi(1,0) and v_j Gauss-Legendre nodes on [0,1], weight
 * W_i W_j; slave barycentrics (1 - xi - eta, xi, eta); sample id
 * k = sample_offset(T) + i*n + j; weight w_k = 2 A_rest(T) W_i W_j.
 *
 * Clipped mortar samples (GMCP_MORTAR, Sec. 4.1 face samples as the paper
 * defines them).  For every slave triangle T and opposing candidate master
 * triangle M, M is projected along n_T onto T's plane and clipped by T
 * (Sutherland-Hodgman); the polygon is fan-triangulated from its first
 * vertex and each sub-triangle carries the n x n rule above.  A sample has
 * slave barycentrics from its position in T, master barycentrics from its
 * position in the projected M, gap g = n_T . (x_m - x_s) and weight
 * w = 2 A_sub W_q, A_sub the sub-triangle's share of T's rest area; it is
 * active for 0 < g < dhat (-dhat < g <= 0 is a penetration, reported with
 * the slave triangle's index).  Every opposing pair contributes (no
 * closest-triangle selection).  Clipped samples have no fixed ids: in this
 * mode gmcp_assemble takes no delta_gap, gmcp_hvp no v_d / out_d, and
 * gmcp_sample_results is unavailable (GMCP_E_ARG); g_ref holds one
 * reference gap per slave triangle ([Ts]: every clipped sample of T has
 * eps = min(0.9 g_ref[T], eps_max), Eq. (adaptive_eps)); the active
 * capacity counts clipped samples.
 *
 * Edge and point samples (GMCP_FEATURES with GMCP_MORTAR, Sec. 4.1).  The
 * edges and vertices of the opposing candidate master triangles of a slave
 * triangle T (each feature once) are projected along n_T into T: an edge is
 * clipped by T to a parameter interval [t0, t1] and carries rule_n
 * Gauss-Legendre points eta (master point (1 - eta) x_a + eta x_b, weight
 * |x_b - x_a| (t1 - t0) W_j, a length, gamma = H(eta, delta_e) H(1 - eta,
 * delta_e), stiffness kappa_edge); a vertex whose projection lies strictly
 * inside T is one point sample (weight 1, gamma 1, stiffness kappa_point).
 * Gaps, activity, gradient and Hessian as for face samples; each feature
 * sample joins the (T, M) pair of the master triangle that owns the feature
 * (the smallest-index opposing candidate containing it; manifold edges).
 *
 * Environments.  n_env independent problems are concatenated: slave
 * vertices/triangles of environment e are [v_off[e], v_off[e+1]) and
 * [t_off[e], t_off[e+1]) (same for the master).  Triangle vertex ids are
 * global (already offset).  Environments never interact.
 *
 * Global vertex numbering of gradient and BSR: slave vertices 0..Vs-1, then
 * master vertices Vs..Vs+Vm-1.  With GMCP_KINEMATIC_MASTER the master rows
 * and columns are dropped (V = Vs).
 *
 * Memory.  Every array argument is DEVICE memory unless marked "host".
 * Positions are [V][3] row-major, float or double (GMCP_F64).  The caller
 * owns every buffer, including the workspace sized by gmcp_workspace_size;
 * the library never allocates device memory and keeps no pointer past a
 * call except the context's workspace, triangle arrays and stream.
 *
 * Execution.  Every call except gmcp_create, gmcp_status and gmcp_destroy
 * only enqueues work on the context's HIP stream and returns immediately;
 * none synchronises.  Argument errors are returned synchronously
 * (GMCP_E_ARG, GMCP_E_HIP).  Data-dependent errors (capacity, penetration,
 * degenerate triangle, non-finite input) are recorded in a device status
 * word that gmcp_status reads back; after such an error the outputs of the
 * failing call are unspecified.  Calls that overlap on one context race.
 */
#ifndef GMCP_H
#define GMCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GMCP_OK = 0,
  GMCP_E_ARG = 1,         /* bad argument (returned synchronously)            */
  GMCP_E_CAPACITY = 2,    /* a workspace capacity was too small; see needs     */
  GMCP_E_PENETRATION = 3, /* an inside opposing hit with -eps < g <= 0         */
  GMCP_E_DEGENERATE = 4,  /* zero-area slave triangle at the current positions */
  GMCP_E_NONFINITE = 5,   /* NaN / Inf input position                          */
  GMCP_E_HIP = 6,         /* a HIP runtime call failed                         */
  GMCP_E_TIMEOUT = 7      /* a device-side wait passed its bound (internal
                             error; the call's results are invalid)           */
} gmcp_status_code;

enum {
  GMCP_F64 = 1,              /* positions and outputs in double              */
  GMCP_KINEMATIC_MASTER = 2, /* master is prescribed: drop its rows/columns  */
  GMCP_MORTAR = 4,           /* clipped mortar face samples (see below)      */
  GMCP_FEATURES = 8          /* plus edge and point samples (needs MORTAR)   */
};

/* Problem layout (all host memory, copied by gmcp_create). */
typedef struct {
  int32_t n_env;
  const int32_t *slave_v_off;  /* [n_env+1] host */
  const int32_t *slave_t_off;  /* [n_env+1] host */
  const int32_t *master_v_off; /* [n_env+1] host */
  const int32_t *master_t_off; /* [n_env+1] host */
  const int32_t *rule_n;       /* [n_env] host, samples per triangle = n*n, 1 <= n <= 4 */
  const double *kappa;         /* [n_env] host, barrier stiffness kappa (face samples)  */
  const double *dhat;          /* [n_env] host, support-radius bound eps_max            */
  const double *delta_T;       /* [n_env] host, face transition width; 0 => gamma = 1   */
  const double *cell;          /* [n_env] host or NULL, broad-phase cell size (m); 0 = auto */
  uint32_t flags;              /* GMCP_F64 | GMCP_KINEMATIC_MASTER | GMCP_MORTAR | GMCP_FEATURES */
  const double *kappa_edge;    /* [n_env] host or NULL (0): kappa of edge samples (GMCP_FEATURES)  */
  const double *kappa_point;   /* [n_env] host or NULL (0): kappa of point samples (GMCP_FEATURES) */
  const double *delta_e;       /* [n_env] host or NULL (0): edge transition width, Eq. (gamma)     */
} gmcp_layout;

/* Capacities of the data-dependent buffers carved from the workspace.
 * Overflow sets GMCP_E_CAPACITY and reports the needed sizes. */
typedef struct {
  int64_t grid_cells;  /* total broad-phase cells over all environments        */
  int64_t grid_items;  /* (master triangle, cell) incidences                   */
  int64_t candidates;  /* (slave triangle, master triangle) candidate pairs    */
  int64_t active;      /* active samples (0 < g < eps after selection)         */
  int64_t pairs;       /* distinct (slave triangle, master triangle) contacts  */
  int64_t row_entries; /* distinct columns of the longest BSR row (<= 4096)      */
} gmcp_caps;

/* Read back by gmcp_status. */
typedef struct {
  int32_t code;         /* gmcp_status_code of the first error, 0 if none        */
  int32_t reserved;
  int64_t index;        /* offending sample / triangle id, -1 if none            */
  int64_t n_active;     /* active samples of the last assembly                   */
  int64_t n_pairs;      /* contact pairs of the last assembly                    */
  int64_t nnzb;         /* BSR blocks written by the last assembly               */
  int64_t n_candidates; /* candidate pairs of the last broad phase               */
  int64_t n_swept;      /* swept (sample, master triangle) pairs of the last CCD */
  gmcp_caps need;       /* sizes that would have fitted (valid after CAPACITY)   */
} gmcp_status_info;

/* 3x3 block CSR output, both triangles stored, columns ascending in a row.
 * row_ptr[V+1] and col[cap_nnzb] int32, val[cap_nnzb][9] row-major blocks
 * (float or double). */
typedef struct {
  int32_t *row_ptr;
  int32_t *col;
  void *val;
  int64_t cap_nnzb;
} gmcp_bsr;

/* Launch shapes of the list-walking kernels, for an autotuner: later calls
 * on the context use them (a captured graph keeps the shapes it was
 * captured with).  Zero selects the default.  Results do not depend on
 * them, except that a BSR row's class (light or heavy table) follows
 * light_row_bound.
 *   query_blocks      grid of the broad-phase query, 1..2048
 *                     (default: the blocks resident at once, at most 2048)
 *   light_row_bound   column insertions of a BSR row processed with the
 *                     small tables (2 x bound slots): 32, 64, 128 or 256
 *                     (default 128); longer rows use the large tables
 *   light_row_blocks  grid of the light-row kernels, 1..2^20 (default 65536)
 *   heavy_row_blocks  grid of the heavy-row kernels, 1..65536 (default 2048) */
typedef struct {
  int32_t query_blocks;
  int32_t light_row_bound;
  int32_t light_row_blocks;
  int32_t heavy_row_blocks;
} gmcp_tuning;

typedef struct gmcp_ctx gmcp_ctx;

/* Bytes of workspace needed for this layout and these capacities. */
size_t gmcp_workspace_size(const gmcp_layout *layout, const gmcp_caps *caps);

/*
 * Creates a context.  slave_tri [Ts][3] and master_tri [Tm][3] are device
 * int32 arrays with global vertex ids; they must stay valid and unchanged
 * while the context lives.  workspace (device, >= gmcp_workspace_size bytes,
 * 256-byte aligned) is owned by the caller.  stream is a hipStream_t (NULL =
 * default stream).  Reads the triangle arrays back to build the static
 * tables (vertex-to-triangle adjacency, Morton-ordered work tiles, the
 * quadrature rules), so this call synchronises.  Returns GMCP_E_ARG on a bad
 * layout (rule_n out of range, offsets not monotone, vertex id out of range).
 */
int gmcp_create(gmcp_ctx **out, const gmcp_layout *layout, const gmcp_caps *caps,
                const int32_t *slave_tri, const int32_t *master_tri, void *workspace,
                size_t workspace_bytes, void *stream);

/* Frees the host side of the context (never the caller's buffers). */
void gmcp_destroy(gmcp_ctx *ctx);

/* Changes the stream later calls are enqueued on. */
int gmcp_set_stream(gmcp_ctx *ctx, void *stream);

/* Sets (GMCP_E_ARG if a field is out of range, nothing changed) or reads
 * the launch shapes; gmcp_get_tuning reports the values in effect, with
 * the defaults filled in (query_blocks 0 until the first broad phase). */
int gmcp_set_tuning(gmcp_ctx *ctx, const gmcp_tuning *tuning);
int gmcp_get_tuning(const gmcp_ctx *ctx, gmcp_tuning *tuning);

/*
 * Sample table (Sec. 4.1, face samples; Eq. (gmcp_potential) weights).
 * From the slave rest positions x_rest [Vs][3] computes and keeps the rest
 * triangle areas; if weights != NULL writes w_k [Ns] = 2 A_rest(T) W_q.
 * Run once per slave mesh, before the first assembly.
 */
int gmcp_build_samples(gmcp_ctx *ctx, const void *x_rest, void *weights);

/* Number of samples Ns over all environments (host query). */
int64_t gmcp_num_samples(const gmcp_ctx *ctx);

/* The n x n face-sample rule the library uses (host only, no GPU):
 * out [n*n][3] host = (xi, eta, W) for q = i*n + j.  GMCP_E_ARG unless 1 <= n <= 4. */
int gmcp_rule(int n, double *out);

/*
 * Broad phase.  For every slave triangle T, lists the master triangles M of
 * its environment that face it (n_T . N_M < 0) and whose bounding box meets
 * the box of T's support prism {p + t n_T : p in T, |t| <= eps_max}: every
 * triangle the narrow phase could accept or flag as penetrating.  Uses a
 * uniform grid per environment over the prism region.  x_slave [Vs][3],
 * x_master [Vm][3].  The lists stay in the workspace for gmcp_assemble.
 * This culls the projection of master features onto slave triangles
 * (Sec. 4.1) to those that can land inside the barrier's support
 * (Sec. 4.2, 0 < g < eps); the paper fixes no acceleration structure.
 */
int gmcp_broadphase(gmcp_ctx *ctx, const void *x_slave, const void *x_master);

/*
 * Assembly.  For every sample: the closest opposing master triangle among
 * the candidates along the slave normal with an inside hit (min master
 * barycentric >= 0) and 0 < g < eps_k (ties: smaller master index); then
 * E_k, c1 = kappa w gamma B'(g), c2 = max(kappa w gamma B''(g), 0) (the
 * rank-one block c2 grad g grad g^T is PSD-projected by clamping c2), the
 * gradient sum_k c1 grad g_k with grad g_k = -beta^s_a n_T (slave vertex a),
 * +beta^m_j n_T (master vertex j), and the Hessian sum_k c2 grad g grad g^T.
 * Sec. 4.2 and Eqs. (gap), (gram), (smoothstep), (gamma), (adaptive_eps).
 *   g_ref     [Ns] nullable: reference gaps, eps_k = min(0.9 g_ref, eps_max)
 *             (mortar mode: [Ts], one per slave triangle)
 *   delta_gap [Ns] nullable: gap offsets added after selection (g += delta)
 *   energy    [n_env] output (sum per environment)
 *   grad      [V][3] nullable output
 *   H         nullable: BSR output (pattern = blocks touched by active samples)
 * Requires gmcp_broadphase on the same positions.  Deterministic: two calls
 * on the same input give bitwise-identical outputs.
 */
int gmcp_assemble(gmcp_ctx *ctx, const void *x_slave, const void *x_master, const void *g_ref,
                  const void *delta_gap, void *energy, void *grad, const gmcp_bsr *H);

/*
 * Step bound for the search direction (dx_slave [Vs][3], dx_master [Vm][3],
 * dx_master NULL = static master):
 *   alpha[e] = min(1, min_k 0.9 g_k / (-grad g_k . dx)   over the active
 *                  samples of the last assembly with grad g_k . dx < 0,
 *                  min over swept pairs of additive CCD (separation 0.1))
 * times (1 - 2^-13) for the part below 1, so the float result never exceeds
 * the exact one.  A swept pair is a sample point and a master triangle whose
 * axis-aligned boxes over the linear motion overlap.  Eqs. (ccd),
 * (global_ccd).  alpha [n_env] float or double.  Needs a prior assembly on x.
 */
int gmcp_ccd_step(gmcp_ctx *ctx, const void *x_slave, const void *x_master, const void *dx_slave,
                  const void *dx_master, void *alpha);

/*
 * The same step bound in two calls, so that its part that does not depend
 * on the assembly can run on another stream while the broad phase and the
 * assembly run (Eqs. (ccd), (global_ccd)):
 *   gmcp_ccd_swept   swept grid and additive CCD over every swept pair
 *                    (needs only gmcp_build_samples); starts a new bound;
 *   gmcp_ccd_finish  Eq. (ccd) over the active samples of the last assembly,
 *                    then alpha [n_env] exactly as gmcp_ccd_step writes it.
 * Same arguments as gmcp_ccd_step (dx_master NULL = static master).  The
 * caller orders the two on the device: gmcp_ccd_finish's stream must wait
 * for the work gmcp_ccd_swept enqueued (an event, or the same stream), and
 * for the assembly.  gmcp_ccd_swept uses its own scan scratch and grid, so
 * it may overlap gmcp_broadphase and gmcp_assemble of the same context on a
 * second stream; it must not overlap another step-bound call.
 * gmcp_ccd_finish returns GMCP_E_ARG unless gmcp_ccd_swept was called since
 * the last bound (host order) and an assembly exists.
 */
int gmcp_ccd_swept(gmcp_ctx *ctx, const void *x_slave, const void *x_master, const void *dx_slave,
                   const void *dx_master);
int gmcp_ccd_finish(gmcp_ctx *ctx, const void *dx_slave, const void *dx_master, void *alpha);

/*
 * Joint Hessian-vector product of E(x, delta) with the samples of the last
 * assembly frozen:  [out_x; out_d] = sum_k c2_k (grad g_k . v_x + v_d[k]) [grad g_k; e_k].
 * v_x, out_x [V][3]; v_d, out_d [Ns] nullable.  Deterministic.
 */
int gmcp_hvp(gmcp_ctx *ctx, const void *v_x, const void *v_d, void *out_x, void *out_d);

/*
 * Energy of the last assembly's samples at new positions x_slave [Vs][3],
 * x_master [Vm][3], every sample frozen (the reading of Sec. 4.2's gradient
 * and Hessian approximation): slave normal n_T, rule point, master triangle
 * and barycentric coordinates, weight w_k, face weight gamma_k and support
 * radius eps_k stay as assembled, so g_k = n_T . (sum_j bm_j x_mj -
 * sum_a bs_a x_sa) is affine in x and this energy's gradient at the
 * assembly positions is the assembled gradient (gap offsets are not
 * applied).  energy [n_env]; +inf for an environment where a frozen gap is
 * <= 0.  The line search of an implicit step uses it so that the energy it
 * tests and the gradient it descends belong to the same function.
 * Deterministic.  GMCP_E_ARG before any assembly.
 */
int gmcp_energy_frozen(gmcp_ctx *ctx, const void *x_slave, const void *x_master, void *energy);

/*
 * Per-sample export of the last assembly (for checks and pressure maps):
 *   master [Ns] int32 (-1 inactive), gap [Ns], bary_m [Ns][3], c1 [Ns],
 *   c2 [Ns], pressure [Ns] = -kappa gamma B'(g) (0 inactive).  Any may be NULL.
 */
int gmcp_sample_results(gmcp_ctx *ctx, int32_t *master, void *gap, void *bary_m, void *c1,
                        void *c2, void *pressure);

/* Contact pairs of the last assembly: T [n], M [n] (device int32) receive
 * the slave and master triangle of each distinct (slave triangle, master
 * triangle) contact, for n = min(cap, n_pairs of gmcp_status) entries in
 * storage order (contiguous per slave triangle).  For checks of which
 * pairs the selection (whole-triangle samples) or the clipping (mortar
 * samples, Sec. 4.1) produced.  GMCP_E_ARG before any assembly. */
int gmcp_pairs(gmcp_ctx *ctx, int32_t *T, int32_t *M, int64_t cap);

/* Candidate lists of the last broad phase: cand_off [Ts+1], cand [cap]
 * (master triangle ids, ascending within a slave triangle). */
int gmcp_candidates(gmcp_ctx *ctx, int32_t *cand_off, int32_t *cand, int64_t cap);

/* Copies the device status to info (host) and clears the error code.
 * Synchronises the stream. */
int gmcp_status(gmcp_ctx *ctx, gmcp_status_info *info);

/*
 * Optional per-stage timing with HIP events recorded on the context's
 * stream around each stage's kernels.  enable != 0 starts a new
 * measurement (and clears the previous one); enable == 0 stops recording.
 */
int gmcp_profile(gmcp_ctx *ctx, int enable);

/* Number of profiled stages (GMCP_STAGE_COUNT) and the name of stage i. */
int gmcp_profile_stages(void);
const char *gmcp_profile_stage_name(int stage);

/*
 * Synchronises, then writes per stage the summed elapsed milliseconds
 * (ms [n]) and the number of timed occurrences (count [n]) since the last
 * gmcp_profile(ctx, 1).  Host arrays of at least gmcp_profile_stages().
 */
int gmcp_profile_read(gmcp_ctx *ctx, double *ms, int64_t *count);

/*
 * Synchronises and writes host out[4] for the last assembly with a Hessian:
 * BSR rows processed as light rows (at most 128 contributions, small LDS
 * tables), heavy rows, and the blocks written by each class (counted on the
 * host from row_ptr, the [V+1] device array of that assembly's BSR).  For
 * per-kernel byte accounting of the profiled stages.
 */
int gmcp_row_classes(gmcp_ctx *ctx, int64_t *out, const int32_t *row_ptr);

/* Human-readable name of a status code. */
const char *gmcp_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* GMCP_H */
