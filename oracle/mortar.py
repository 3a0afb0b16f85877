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

Edge and point samples (Sec. 4.1) are generated from the edges and
vertices of the opposing master triangles (feature_samples).

Readings (the paper does not fix them):
* weight w = 2 A_sub W_q with A_sub the sub-triangle's share of the slave
  triangle's REST area (2 |area in (u, v)| A_rest(T_s)), so the weights of a
  fully covered slave triangle sum to its rest area;
* pairs: every opposing master triangle; samples with 0 < g < eps are
  active, -eps < g <= 0 is a penetration error; eps = dhat, or with
  reference gaps (Eq. (adaptive_eps)) one per slave triangle,
  eps_T = min(0.9 g_ref[T], dhat) for every sample of T (clipped samples
  have no fixed identity, the slave triangle is what they keep);
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
    M: int              # master triangle (face samples), -1 for edge / point samples
    bs: np.ndarray      # slave barycentrics (3)
    bm: np.ndarray      # coefficients of the master vertices mv
    w: float
    g: float
    n: np.ndarray       # slave unit normal
    mv: np.ndarray = None   # master vertex ids (3 face, 2 edge, 1 point)
    kind: int = 2           # 2 face, 1 edge, 0 point (Eq. (gmcp_potential))
    eta: float = 0.0        # edge parameter (edge samples)
    eps: float = None       # support radius (None: the problem's dhat)


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
            out.append(Sample(T, M, bs, bm, 2.0 * (a2 * area_rest) * wq, g, n, np.asarray(P.tm[M])))
    return out


def clip_segment(qa, qb):
    """Parameter interval (t0, t1) of the segment qa + t (qb - qa), t in
    [0, 1], inside the reference triangle, or None (Liang-Barsky)."""
    t0, t1 = 0.0, 1.0
    for f in (lambda p: p[0], lambda p: p[1], lambda p: 1.0 - p[0] - p[1]):
        fa, fb = f(qa), f(qb)
        d = fb - fa
        if d == 0.0:
            if fa < 0.0:
                return None
            continue
        t = -fa / d
        if d > 0.0:
            t0 = max(t0, t)
        else:
            t1 = min(t1, t)
    return (t0, t1) if t1 > t0 else None


def _frame(P, T):
    s = P.xs[P.ts[T]]
    e1, e2 = s[1] - s[0], s[2] - s[0]
    c = np.cross(e1, e2)
    n = c / np.linalg.norm(c)
    G = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
    return s[0], e1, e2, n, G


def feature_samples(P: "oracle.Problem", T: int, opposing):
    """Edge and point samples (Sec. 4.1) of slave triangle T against the
    edges and vertices of the opposing master triangles `opposing` (each
    feature once).  Edge (a, b): projected along n_T, clipped by T to the
    parameter interval [t0, t1], Gauss-Legendre with rule_n points: eta,
    x_m = (1 - eta) x_a + eta x_b, weight |x_b - x_a| (t1 - t0) W_j (a
    length), gap (1 - eta) h_a + eta h_b.  Vertex p: its projection strictly
    inside T (a point on a slave edge belongs to no triangle), weight 1,
    gap h_p."""
    s0, e1, e2, n, G = _frame(P, T)
    proj = lambda x: np.linalg.solve(G, np.array([(x - s0) @ e1, (x - s0) @ e2]))
    xg, wg = np.polynomial.legendre.leggauss(P.rule_n)
    xg, wg = (xg + 1.0) / 2.0, wg / 2.0
    tri = P.tm[np.asarray(opposing, dtype=np.int64)]
    ed = np.sort(np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]), axis=1)
    ed = np.unique(ed, axis=0) if ed.size else ed.reshape(0, 2)
    hv = (P.xm - s0) @ n
    # an edge entirely beyond +eps or below -eps has no sample in range
    keep = (np.minimum(hv[ed[:, 0]], hv[ed[:, 1]]) < P.dhat) & (np.maximum(hv[ed[:, 0]], hv[ed[:, 1]]) > -P.dhat)
    verts = np.unique(tri)
    out = []
    for a, b in ed[keep]:
        a, b = int(a), int(b)
        xa, xb = P.xm[a], P.xm[b]
        ha, hb = (xa - s0) @ n, (xb - s0) @ n
        qa, qb = proj(xa), proj(xb)
        seg = clip_segment(qa, qb)
        if seg is None:
            continue
        t0, t1 = seg
        L = float(np.linalg.norm(xb - xa))
        for xj, wj in zip(xg, wg):
            eta = t0 + (t1 - t0) * xj
            y = qa + eta * (qb - qa)
            bs = np.array([1.0 - y[0] - y[1], y[0], y[1]])
            out.append(Sample(T, -1, bs, np.array([1.0 - eta, eta]), L * (t1 - t0) * wj,
                              float((1.0 - eta) * ha + eta * hb), n, np.array([a, b]), 1, float(eta)))
    for p in verts[np.abs(hv[verts]) < P.dhat]:
        p = int(p)
        h = float((P.xm[p] - s0) @ n)
        if not (-P.dhat < h < P.dhat):
            continue
        y = proj(P.xm[p])
        if y[0] > 0.0 and y[1] > 0.0 and 1.0 - y[0] - y[1] > 0.0:
            out.append(Sample(T, -1, np.array([1.0 - y[0] - y[1], y[0], y[1]]), np.array([1.0]), 1.0, h, n,
                              np.array([p]), 0))
    return out


def samples(P: "oracle.Problem", tris=None, features: bool = False, g_ref_tri=None):
    """All clipped face samples of the slave triangles `tris` (default all)
    against every opposing master triangle, and with `features` the edge
    and point samples of those triangles' edges and vertices.  g_ref_tri
    (optional, one per slave triangle) sets the triangle's support radius
    eps_T = min(0.9 g_ref_tri[T], dhat), Eq. (adaptive_eps).  Raises
    OracleError(PENETRATION) for a sample with -eps < g <= 0 (index = slave
    triangle)."""
    area = oracle.rest_area(P.xs_rest, P.ts)
    rule = P.rule
    tris = range(P.ts.shape[0]) if tris is None else tris
    out = []
    for T in tris:
        eps = P.dhat if g_ref_tri is None else min(0.9 * float(g_ref_tri[T]), P.dhat)
        s0, e1, e2, n, _ = _frame(P, T)
        # heights of the master vertices above the slave plane: the gap is
        # their barycentric combination, so a master triangle entirely
        # beyond +eps or below -eps has no sample in range
        h = ((P.xm - s0) @ n)[P.tm]
        near = np.nonzero((h.min(1) < eps) & (h.max(1) > -eps))[0]
        got = []
        for M in near:
            got += pair_samples(P, T, int(M), area[T], rule)
        if features:
            mm = P.xm[P.tm]
            N = np.cross(mm[:, 1] - mm[:, 0], mm[:, 2] - mm[:, 0])
            opposing = np.nonzero(N @ n < 0.0)[0]
            got += feature_samples(P, T, opposing)
        for smp in got:
            smp.eps = eps
            if -eps < smp.g <= 0.0:
                raise oracle.OracleError(oracle.E_PENETRATION, T)
        out += got
    return out


@dataclass
class MortarAssembly:
    energy: float
    grad: np.ndarray          # [Vs + Vm, 3]
    blocks: dict              # (row, col) -> 3x3, rows/cols: slave 0..Vs-1, master Vs..
    active: list              # active samples
    c1: np.ndarray
    c2: np.ndarray


def gamma(P: "oracle.Problem", smp, delta_e: float = 0.0) -> float:
    """Master-feature weight, Eq. (gamma): f_T = H(min beta^m, delta_T) for
    face samples, f_e = H(eta, delta_e) H(1 - eta, delta_e) for edge samples,
    1 for point samples (H = 1 for a zero width)."""
    if smp.kind == 2:
        return oracle.hermite(min(smp.bm), P.delta_T) if P.delta_T > 0 else 1.0
    if smp.kind == 1:
        return (oracle.hermite(smp.eta, delta_e) * oracle.hermite(1.0 - smp.eta, delta_e)) if delta_e > 0 else 1.0
    return 1.0


def assemble(P: "oracle.Problem", smps, kinematic: bool = False, with_hessian: bool = True,
             kappa_edge: float = 0.0, kappa_point: float = 0.0, delta_e: float = 0.0):
    """Energy, gradient and PSD Hessian of the active samples (Sec. 4.2,
    samples frozen): grad g = -bs_a n at slave vertex a, +bm_j n at master
    vertex mv_j; E_k = kappa_q w gamma B, c1 = kappa_q w gamma B', c2 =
    max(kappa_q w gamma B'', 0), kappa_q = P.kappa (faces), kappa_edge,
    kappa_point (Eq. (gmcp_potential))."""
    Vs = P.Vs
    V = Vs + P.Vm
    grad = np.zeros((V, 3))
    blocks = {}
    E = 0.0
    act, c1s, c2s = [], [], []
    kap = {2: P.kappa, 1: kappa_edge, 0: kappa_point}
    for smp in smps:
        eps = P.dhat if smp.eps is None else smp.eps
        if not (0.0 < smp.g < eps):
            continue
        kw = kap[smp.kind] * smp.w * gamma(P, smp, delta_e)
        E += kw * oracle.barrier(smp.g, eps)
        c1 = kw * oracle.barrier_d1(smp.g, eps)
        c2 = max(kw * oracle.barrier_d2(smp.g, eps), 0.0)
        act.append(smp)
        c1s.append(c1)
        c2s.append(c2)
        ids = [int(v) for v in P.ts[smp.T]] + ([] if kinematic else [Vs + int(v) for v in smp.mv])
        coef = list(-smp.bs) + ([] if kinematic else list(smp.bm))
        nn = np.outer(smp.n, smp.n)
        for i, ci in zip(ids, coef):
            grad[i] += c1 * ci * smp.n
            if with_hessian:
                for j, cj in zip(ids, coef):
                    blocks[(i, j)] = blocks.get((i, j), 0.0) + c2 * ci * cj * nn
    return MortarAssembly(E, grad, blocks, act, np.array(c1s), np.array(c2s))


def frozen_energy(P: "oracle.Problem", active, xs_new, xm_new, kappa_edge: float = 0.0,
                  kappa_point: float = 0.0, delta_e: float = 0.0) -> float:
    """Energy of the active samples with every sample frozen (Sec. 4.2):
    normal, slave barycentrics, master vertices and coefficients, weight
    and feature weight fixed, so g_k = n . (sum_j bm_j x_mj - sum_a bs_a x_sa)
    is affine in the positions; +inf if a gap is <= 0."""
    kap = {2: P.kappa, 1: kappa_edge, 0: kappa_point}
    E = 0.0
    for s in active:
        g = float(s.n @ (s.bm @ xm_new[s.mv] - s.bs @ xs_new[P.ts[s.T]]))
        if g <= 0.0:
            return float("inf")
        eps = P.dhat if s.eps is None else s.eps
        if g < eps:
            E += kap[s.kind] * s.w * gamma(P, s, delta_e) * oracle.barrier(g, eps)
    return E


def linear_step(P: "oracle.Problem", active, dxs, dxm=None) -> float:
    """Eq. (ccd) over clipped samples: min over active samples with
    grad g . dx < 0 of 0.9 g / (-grad g . dx) (inf if none), samples frozen."""
    a = np.inf
    for s in active:
        gd = -s.n @ (s.bs @ dxs[P.ts[s.T]])
        if dxm is not None:
            gd += s.n @ (s.bm @ dxm[s.mv])
        if gd < 0.0:
            a = min(a, 0.9 * s.g / (-gd))
    return a
