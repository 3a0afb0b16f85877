/*
 * gmcp_fem.h - C ABI of the implicit-step system around the GMCP contact
 * potential: linear-elastic tetrahedra, lumped mass and a block-Jacobi
 * preconditioned conjugate-gradient solve of the Newton system
 *
 *   (M / dt^2 + K + H) d = rhs,
 *
 * where H is the contact Hessian in the BSR layout gmcp_assemble writes
 * (kinematic master: rows and columns are the slave vertices, which are the
 * vertices of the tetrahedral body).  This is the incremental-potential
 * Newton system of IPC, which the paper's contact model plugs into (Sec. 1,
 * Sec. 3.1: libuipc runs linear FEM bodies with IPC contact).
 *
 * Energy of one implicit Euler step with target x_tilde = x_t + dt v_t:
 *   E(x) = 1/2 |x - x_tilde|^2_M / dt^2 + 1/2 (x - X)^T K (x - X) + Psi(x),
 * K the linear-elastic stiffness (Lame mu, lambda from Young's modulus and
 * Poisson's ratio), M the lumped mass (density * volume / 4 per tet vertex).
 * Dirichlet vertices are held fixed (zero gradient, zero update); single
 * components can be held too (gmcp_fem_constrain).
 *
 * All arrays are device memory, double precision, unless marked host.  The
 * caller owns the workspace.  Calls enqueue on the stream; gmcp_fem_create
 * and gmcp_fem_solve synchronise (the solve checks its residual every 8
 * iterations).
 */
#ifndef GMCP_FEM_H
#define GMCP_FEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmcp_fem gmcp_fem;

/* Workspace bytes for tets [n_tet][4] (host, vertex ids < n_vert); 0 on bad input. */
size_t gmcp_fem_workspace_size(const int32_t *tets, int64_t n_tet, int64_t n_vert);

/* Builds the static stiffness (BSR, deterministic per-block sums), the
 * lumped mass and the Dirichlet mask.  tets, X_rest [n_vert][3] and fixed
 * [n_fixed] are HOST arrays.  GMCP_E_ARG on bad sizes or material. */
int gmcp_fem_create(gmcp_fem **out, const int32_t *tets, int64_t n_tet, int64_t n_vert, const double *X_rest,
                    double young, double poisson, double density, double dt, const int32_t *fixed,
                    int64_t n_fixed, void *workspace, size_t bytes, void *stream);
void gmcp_fem_destroy(gmcp_fem *fem);
/* Holds further displacement components (roller conditions, e.g. the patch
 * test's u_x = u_y = 0 on a whole block, Sec. 5): verts [n] HOST vertex ids,
 * mask bit d (1 = x, 2 = y, 4 = z) = component d held, added to what the
 * vertex already holds.  Held components take no part in the solve (zero
 * gradient, zero update, rows and columns removed), exactly like whole
 * Dirichlet vertices.  Synchronises the stream; GMCP_E_ARG on a bad id or
 * mask.  */
int gmcp_fem_constrain(gmcp_fem *fem, const int32_t *verts, int64_t n, int mask);
int gmcp_fem_set_stream(gmcp_fem *fem, void *stream);

/* Number of 3x3 blocks of K; copy of K's BSR (row_ptr [V+1], col, val [nnzb][9]). */
int64_t gmcp_fem_nnzb(const gmcp_fem *fem);
int gmcp_fem_stiffness(gmcp_fem *fem, int32_t *row_ptr, int32_t *col, double *val);

/* energy (one device double) = inertial + elastic terms of E at x; grad
 * [V][3] nullable = their gradient, 0 in held components. */
int gmcp_fem_energy(gmcp_fem *fem, const double *x, const double *x_tilde, double *energy, double *grad);

/* y = (M/dt^2 + K + H) x with held rows and columns removed (y = 0 there);
 * H nullable (all three pointers or none). */
int gmcp_fem_apply(gmcp_fem *fem, const int32_t *h_row_ptr, const int32_t *h_col, const double *h_val,
                   const double *x, double *y);

/* Preconditioned CG from x = 0 until |r| <= rtol |rhs| or max_iter; Dirichlet
 * entries of x are 0.  iters, rel_res: host outputs (nullable). */
int gmcp_fem_solve(gmcp_fem *fem, const int32_t *h_row_ptr, const int32_t *h_col, const double *h_val,
                   const double *rhs, double *x, double rtol, int max_iter, int *iters, double *rel_res);

#ifdef __cplusplus
}
#endif

#endif /* GMCP_FEM_H */
