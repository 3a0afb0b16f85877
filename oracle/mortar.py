"""Oracle: clipped mortar face samples (Sec. 4.1, face samples) - TEST
INFRASTRUCTURE ONLY (FP64, numpy, pure-Python loops for small cases).

For a slave triangle T_s (current positions s0, s1, s2, edges e1 = s1 - s0,
e2 = s2 - s0, unit normal n = e1 x e2 / |e1 x e2|) and an opposing master
triangle T_m (n . N_m < 0), both are projected along n onto the plane of T_s
and the projected master triangle is clipped by T_s (Sutherland-Hodgman,
Sec. 4.1).  Coordinates in the plane are the slave barycentric pair (u, v)
(x = s0 + u e1 + v e2), so T_s is the reference triangle u, v >= 0,
u + v <= 1.  The clipped polygon is fan-triangulated from its first vertex
and every sub-triangle carries the n x n Stroud rule.  A quadrature point y
has slave barycentrics beta^s = (1 - u - v, u, v), master barycentrics
beta^m = the barycentric coordinates of y in the projected master triangle
(projection along n is affine, so they are the master triangle's own), and
the signed gap (Eq. (gap)) g = n . (sum_j beta^m_j m_j - x_s).

Readings (the paper does not fix them):
* weight w = 2 A_sub W_q with A_sub the sub-triangle's share of the slave
  triangle's REST area (2 |area in (u, v)| A_rest(T_s)), so the weights of a
  fully covered slave triangle sum to its rest area;
* pairs: every opposing master triangle; samples with 0 < g < eps are
  active (eps = dhat), -eps < g <= 0 is a penetration error;
* gamma = H(min beta^m, delta_T) (1 when delta_T = 0), kappa for faces.

Energy, gradient and Hessian of the samples follow Sec. 4.2 with the
samples frozen, as for the whole-triangle samples.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle


def clip_by_reference(poly):
    """Sutherland-Hodgman clip of a polygon (list of (u, v) arrays) by the
    half-planes u >= 0, v >= 0, 1 - u - v >= 0."""
    planes = (lambda p: p[0], lambda p: p[1], lambda p: 1.0 - p[0] - p[1])
    out = [np.asarray(p, float) for p in poly]
    for f in planes:
        if not out:
            break
        inp, out = out, []
        for i in range(len(inp)):
            P, Q = inp[i], inp[(i + 1) % len(inp)]
            fp, fq = f(P), f(Q)
            if fp >= 0.0:
                out.append(P)
                if fq < 0.0:
                    out.append(P + (Q - P) * (fp / (fp - fq)))
            elif fq >= 0.0:
                out.append(P + (Q - P) * (fp / (fp - fq)))
    return out


@dataclass
class Sample:
    T: int
    M: int
    bs: np.ndarray      # slave barycentrics (3)
    bm: np.ndarray      # master barycentrics (3)
    w: float
    g: float
    n: np.ndarray       # slave unit normal


def pair_samples(P: "oracle.Problem", T: int, M: int, area_rest: float, rule):
    """Quadrature points of the clipped overlap of slave triangle T and
    master triangle M ([] if not opposing or no overlap)."""
    s = P.xs[P.ts[T]]
    m = P.xm[P.tm[M]]
    e1, e2 = s[1] - s[0], s[2] - s[0]
    c = np.cross(e1, e2)
    n = c / np.linalg.norm(c)
    if n @ np.cross(m[1] - m[0], m[2] - m[0]) >= 0.0:
        return []
    G = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
    q = [np.linalg.solve(G, np.array([(mj - s[0]) @ e1, (mj - s[0]) @ e2])) for mj in m]
    Q = np.array([q[1] - q[0], q[2] - q[0]]).T        # columns: projected master edges
    if abs(np.linalg.det(Q)) <= 1e-14:
        return []                                     # master triangle edge-on to the slave plane
    poly = clip_by_reference(q)
    out = []
    for i in range(1, len(poly) - 1):
        A, B, C = poly[0], poly[i], poly[i + 1]
        a2 = abs((B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0]))   # 2 |area| in (u, v)
        if a2 == 0.0:
            continue
        for xi, eta, wq in rule:
            y = A + xi * (B - A) + eta * (C - A)
            bs = np.array([1.0 - y[0] - y[1], y[0], y[1]])
            b12 = np.linalg.solve(Q, y - q[0])
            bm = np.array([1.0 - b12[0] - b12[1], b12[0], b12[1]])
            xs_k = s[0] + y[0] * e1 + y[1] * e2
            g = float(n @ (bm @ m - xs_k))
            out.append(Sample(T, M, bs, bm, 2.0 * (a2 * area_rest) * wq, g, n))
    return out


def samples(P: "oracle.Problem", tris=None):
    """All clipped face samples of the slave triangles `tris` (default all)
    against every master triangle.  Raises OracleError(PENETRATION) for a
    sample with -eps < g <= 0 (index = slave triangle)."""
    area = oracle.rest_area(P.xs_rest, P.ts)
    rule = P.rule
    eps = P.dhat
    tris = range(P.ts.shape[0]) if tris is None else tris
    hm = None
    out = []
    for T in tris:
        s = P.xs[P.ts[T]]
        c = np.cross(s[1] - s[0], s[2] - s[0])
        n = c / np.linalg.norm(c)
        # heights of the master vertices above the slave plane: the gap is
        # their barycentric combination, so a master triangle entirely
        # beyond +eps or below -eps has no sample in range
        hm = (P.xm - s[0]) @ n
        h = hm[P.tm]
        near = np.nonzero((h.min(1) < eps) & (h.max(1) > -eps))[0]
        for M in near:
            for smp in pair_samples(P, T, int(M), area[T], rule):
                if -eps < smp.g <= 0.0:
                    raise oracle.OracleError(oracle.E_PENETRATION, T)
                out.append(smp)
    return out


@dataclass
class MortarAssembly:
    energy: float
    grad: np.ndarray          # [Vs + Vm, 3]
    blocks: dict              # (row, col) -> 3x3, rows/cols: slave 0..Vs-1, master Vs..
    active: list              # active samples
    c1: np.ndarray
    c2: np.ndarray


def assemble(P: "oracle.Problem", smps, kinematic: bool = False, with_hessian: bool = True):
    """Energy, gradient and PSD Hessian of the active samples (Sec. 4.2,
    samples frozen): grad g = -bs_a n at slave vertex a, +bm_j n at master
    vertex j; E_k = kappa w gamma B, c1 = kappa w gamma B', c2 = max(kappa
    w gamma B'', 0)."""
    Vs = P.Vs
    V = Vs + P.Vm
    grad = np.zeros((V, 3))
    blocks = {}
    E = 0.0
    act, c1s, c2s = [], [], []
    for smp in smps:
        if not (0.0 < smp.g < P.dhat):
            continue
        gam = oracle.hermite(min(smp.bm), P.delta_T) if P.delta_T > 0 else 1.0
        kw = P.kappa * smp.w * gam
        E += kw * oracle.barrier(smp.g, P.dhat)
        c1 = kw * oracle.barrier_d1(smp.g, P.dhat)
        c2 = max(kw * oracle.barrier_d2(smp.g, P.dhat), 0.0)
        act.append(smp)
        c1s.append(c1)
        c2s.append(c2)
        ids = [int(v) for v in P.ts[smp.T]] + ([] if kinematic else [Vs + int(v) for v in P.tm[smp.M]])
        coef = list(-smp.bs) + ([] if kinematic else list(smp.bm))
        nn = np.outer(smp.n, smp.n)
        for i, ci in zip(ids, coef):
            grad[i] += c1 * ci * smp.n
            if with_hessian:
                for j, cj in zip(ids, coef):
                    blocks[(i, j)] = blocks.get((i, j), 0.0) + c2 * ci * cj * nn
    return MortarAssembly(E, grad, blocks, act, np.array(c1s), np.array(c2s))


def linear_step(P: "oracle.Problem", active, dxs, dxm=None) -> float:
    """Eq. (ccd) over clipped samples: min over active samples with
    grad g . dx < 0 of 0.9 g / (-grad g . dx) (inf if none), samples frozen."""
    a = np.inf
    for s in active:
        gd = -s.n @ (s.bs @ dxs[P.ts[s.T]])
        if dxm is not None:
            gd += s.n @ (s.bm @ dxm[P.tm[s.M]])
        if gd < 0.0:
            a = min(a, 0.9 * s.g / (-gd))
    return a
