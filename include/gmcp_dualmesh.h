/*
 * gmcp_dualmesh.h - C ABI of the dual-mesh mapper (Sec. 3, "Dual-Mesh
 * Mapper"): a visual mesh rides on the surface of the simulation mesh.
 *
 * Precomputation (Eqs. (bary_proj), (decomp), (gram)): each visual vertex p
 * is attached to its nearest simulation surface triangle T = (v0, v1, v2)
 * by Euclidean point-triangle distance (ties go to the smaller triangle
 * index; triangles of zero area are never chosen).  With e1 = v1 - v0,
 * e2 = v2 - v0, n = e1 x e2 / |e1 x e2| and d = p - v0, the stored offset is
 * delta = d . n and (v, w) solve the 2x2 Gram system
 *   [e1.e1 e1.e2; e1.e2 e2.e2] (v, w)^T = (d.e1, d.e2)^T,  u = 1 - v - w,
 * so that d = v e1 + w e2 + delta n holds exactly (u, v, w describe the
 * projection onto the plane of T and may leave [0, 1] when the nearest
 * point of T is on its boundary).
 *
 * Per-frame update (Eq. (bary_interp)): p' = u v0' + v v1' + w v2' + delta n'
 * with n' the unit normal of the deformed triangle.
 *
 * All pointers are device pointers owned by the caller; nothing is
 * allocated.  Calls enqueue on `stream` (a hipStream_t) and return
 * GMCP_OK (0), GMCP_E_ARG (1: a null pointer with a non-zero size, a
 * negative size, no triangles for a non-empty visual mesh) or GMCP_E_HIP
 * (6: the launch failed).  Triangle vertex ids must index V / Vd; the
 * library does not check them.
 */
#ifndef GMCP_DUALMESH_H
#define GMCP_DUALMESH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* P [N][3], V [nV][3] double; F [nT][3] int32.  Writes tri [N] (int32),
 * bary [N][3] = (u, v, w) and delta [N] (double), and, if dist2 is not
 * NULL, the squared distance to the chosen triangle [N] (double). */
int gmcp_dualmesh_embed(const double *P, int64_t N, const double *V, const int32_t *F, int64_t nT, int32_t *tri,
                        double *bary, double *delta, double *dist2, void *stream);

/* out [N][3] = Eq. (bary_interp) on the deformed simulation positions
 * Vd [nV][3].  flags & GMCP_F64 (1): Vd, bary, delta and out are double;
 * otherwise float. */
int gmcp_dualmesh_update(const void *Vd, const int32_t *F, const int32_t *tri, const void *bary, const void *delta,
                         int64_t N, void *out, uint32_t flags, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GMCP_DUALMESH_H */
