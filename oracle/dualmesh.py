"""Oracle: the dual-mesh mapper (Sec. 3, "Dual-Mesh Mapper") - TEST
INFRASTRUCTURE ONLY (FP64, numpy).

Precomputation (Eqs. (bary_proj), (decomp), (gram)): every visual vertex p
is attached to its nearest simulation triangle T (Euclidean point-triangle
distance, ties to the smaller triangle index, zero-area triangles never
chosen); with e1 = v1 - v0,
e2 = v2 - v0, n = e1 x e2 / |e1 x e2| and d = p - v0, the offset is
delta = d . n and (v, w) solve the 2x2 Gram system
[e1.e1 e1.e2; e1.e2 e2.e2] (v, w) = (d.e1, d.e2), u = 1 - v - w.

Per-frame update (Eq. (bary_interp)): p' = u v0' + v v1' + w v2' + delta n'
with n' the unit normal of the deformed triangle.

Pins (tests/test_oracle_dualmesh.py): reconstruction at rest, rigid
invariance, the O(h^2) error under a smooth deformation, the nearest
triangle against dense sampling of every triangle.
"""
from __future__ import annotations

import numpy as np


def closest_points(p, A, B, C):
    """Closest point of each triangle (A[t], B[t], C[t]) to the point p
    ([T][3] arrays): the plane projection when it falls inside the triangle,
    else the nearest of the three edges' clamped projections."""
    e1, e2 = B - A, C - A
    d = p - A
    g11, g12, g22 = (e1 * e1).sum(1), (e1 * e2).sum(1), (e2 * e2).sum(1)
    r1, r2 = (d * e1).sum(1), (d * e2).sum(1)
    det = g11 * g22 - g12 * g12
    v = (g22 * r1 - g12 * r2) / det
    w = (g11 * r2 - g12 * r1) / det
    inside = (v >= 0.0) & (w >= 0.0) & (v + w <= 1.0)
    best = A + v[:, None] * e1 + w[:, None] * e2
    bd = np.full(A.shape[0], np.inf)
    edge_best = np.zeros_like(A)
    for s0, s1 in ((A, B), (B, C), (C, A)):
        e = s1 - s0
        t = np.clip(((p - s0) * e).sum(1) / (e * e).sum(1), 0.0, 1.0)
        q = s0 + t[:, None] * e
        dq = ((p - q) ** 2).sum(1)
        take = dq < bd
        edge_best[take] = q[take]
        bd = np.where(take, dq, bd)
    return np.where(inside[:, None], best, edge_best)


def nearest_triangle(p, V, F):
    """(index, squared distance) of the nearest triangle; ties to the smaller index."""
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    with np.errstate(divide="ignore", invalid="ignore"):
        q = closest_points(p, A, B, C)
    d2 = ((p - q) ** 2).sum(1)
    d2[(np.cross(B - A, C - A) ** 2).sum(1) == 0.0] = np.inf    # zero-area triangles are never chosen
    t = int(np.argmin(d2))          # first minimum: the smaller index on ties
    return t, float(d2[t])


def frame(V, F, t):
    """(v0, e1, e2, unit normal) of triangle t."""
    v0, v1, v2 = V[F[t, 0]], V[F[t, 1]], V[F[t, 2]]
    e1, e2 = v1 - v0, v2 - v0
    n = np.cross(e1, e2)
    return v0, e1, e2, n / np.linalg.norm(n)


def embed_on(p, V, F, t):
    """(u, v, w, delta) of p on triangle t (Eqs. (decomp), (gram))."""
    v0, e1, e2, n = frame(V, F, t)
    d = p - v0
    G = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
    v, w = np.linalg.solve(G, np.array([d @ e1, d @ e2]))
    return 1.0 - v - w, v, w, float(d @ n)


def embed(P, V, F):
    """Mapping of every visual vertex: T [N] int, bary [N][3], delta [N], dist2 [N]."""
    N = P.shape[0]
    T = np.zeros(N, dtype=np.int64)
    B = np.zeros((N, 3))
    D = np.zeros(N)
    d2 = np.zeros(N)
    for i in range(N):
        T[i], d2[i] = nearest_triangle(P[i], V, F)
        u, v, w, D[i] = embed_on(P[i], V, F, T[i])
        B[i] = (u, v, w)
    return T, B, D, d2


def update(Vd, F, T, B, D):
    """Visual positions on the deformed simulation mesh Vd (Eq. (bary_interp))."""
    out = np.zeros((T.shape[0], 3))
    for i in range(T.shape[0]):
        n = frame(Vd, F, T[i])[3]
        a, b, c = Vd[F[T[i]]]
        out[i] = B[i, 0] * a + B[i, 1] * b + B[i, 2] * c + D[i] * n
    return out
