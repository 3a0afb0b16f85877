"""FP64 CPU oracle for the GMCP hot path — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never imports it and shares no code with it.

The numerical core is plain C (``gmcp_oracle.c``, double precision, built by
``oracle.build``); this module marshals numpy arrays to it.  Every function
follows a passage of the paper (Sec. 4, "Geometric Mortar Contact
Potential"); see the C source for the per-function citations.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, brute force or finite differences.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from .rule import stroud_rule

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, E_ARG, E_CAPACITY, E_PENETRATION, E_DEGENERATE, E_NONFINITE = 0, 1, 2, 3, 4, 5
FLAG_SUPPORT, FLAG_INSIDE, FLAG_TIE, FLAG_PARALLEL, FLAG_ZERO = 1, 2, 4, 8, 16


class OracleError(RuntimeError):
    def __init__(self, code, index):
        super().__init__(f"oracle status {code} at index {index}")
        self.code = code
        self.index = index


def use_library(path: str):
    """Load the oracle from another build of gmcp_oracle.c (for example the
    -march=native build that times the oracle); later calls use it."""
    global _LIB
    _LIB = None
    return lib(path)


def set_threads(n: int):
    """Threads of the oracle's OpenMP loops."""
    lib().ora_set_threads(int(n))


def max_threads() -> int:
    return int(lib().ora_max_threads())


def lib(path: str | None = None):
    global _LIB
    if _LIB is None:
        if path is None:
            path = os.path.join(HERE, "liboracle.so")
            src = os.path.join(HERE, "gmcp_oracle.c")
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
                from .build import build
                build()
        L = C.CDLL(path)
        d, i, i64 = C.c_double, C.c_int, C.c_int64
        P = C.c_void_p
        L.ora_barrier.restype = d
        L.ora_barrier.argtypes = [d, d]
        L.ora_barrier_d1.restype = d
        L.ora_barrier_d1.argtypes = [d, d]
        L.ora_barrier_d2.restype = d
        L.ora_barrier_d2.argtypes = [d, d]
        L.ora_hermite.restype = d
        L.ora_hermite.argtypes = [d, d]
        L.ora_rest_area.argtypes = [i, P, P, P]
        L.ora_narrow.restype = i
        L.ora_narrow.argtypes = [i, i, P, P, i, i, P, P, i, P, d, P, i, P, P, P, P, P]
        L.ora_sample_geom.restype = i
        L.ora_sample_geom.argtypes = [P, P, P, P, i, P, i64, i, P, P, P]
        L.ora_psd_project.restype = d
        L.ora_psd_project.argtypes = [i, P]
        L.ora_local_block12.restype = d
        L.ora_local_block12.argtypes = [d, P, P, P]
        L.ora_assemble.restype = i
        L.ora_assemble.argtypes = [i, i, P, P, i, i, P, P, i, P, P, d, d, d, P, P, P, i, i,
                                   P, P, P, P, P, P, i64, P, P, P, P, P, P]
        L.ora_pressure_loss.restype = d
        L.ora_pressure_loss.argtypes = [i, i, P, P, i, P, P, i, P, d, d, d, P, P, P, P, P, P]
        L.ora_hvp.argtypes = [i, i, P, P, i, P, P, i, P, P, P, P, P, P, P]
        L.ora_step_linear.restype = d
        L.ora_step_linear.argtypes = [i, P, P, P, P, i, P, P, P, P]
        L.ora_point_tri_dist2.restype = d
        L.ora_point_tri_dist2.argtypes = [P, P, P, P]
        L.ora_accd.restype = d
        L.ora_accd.argtypes = [P, P, P, P, P, P, P, P, d, d]
        L.ora_ccd_step.restype = d
        L.ora_ccd_step.argtypes = [i, i, P, P, i, i, P, P, i, P, P, P, P, d, i, P, P, P]
        L.ora_swept_count.restype = i64
        L.ora_swept_count.argtypes = [i, P, P, i, P, P, i, P, P, P, d, d, i]
        L.ora_set_threads.restype = None
        L.ora_set_threads.argtypes = [i]
        L.ora_max_threads.restype = i
        L.ora_max_threads.argtypes = []
        _LIB = L
    return _LIB


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------ scalars
def barrier(g, eps):
    return lib().ora_barrier(float(g), float(eps))


def barrier_d1(g, eps):
    return lib().ora_barrier_d1(float(g), float(eps))


def barrier_d2(g, eps):
    return lib().ora_barrier_d2(float(g), float(eps))


def hermite(x, delta):
    return lib().ora_hermite(float(x), float(delta))


def rest_area(x, tri):
    x, tri = _f64(x), _i32(tri)
    out = np.empty(tri.shape[0])
    lib().ora_rest_area(tri.shape[0], _p(x), _p(tri), _p(out))
    return out


def psd_project(H):
    H = _f64(H).copy()
    clamped = lib().ora_psd_project(H.shape[0], _p(H))
    return H, clamped


def local_block12(c2, bm, n):
    H = np.empty((12, 12))
    clamped = lib().ora_local_block12(float(c2), _p(_f64(bm)), _p(_f64(n)), _p(H))
    return H, clamped


def point_tri_dist2(p, a, b, c):
    return lib().ora_point_tri_dist2(_p(_f64(p)), _p(_f64(a)), _p(_f64(b)), _p(_f64(c)))


def accd(p, dp, a, da, b, db, c, dc, s=0.1, tmax=1.0):
    return lib().ora_accd(*[_p(_f64(v)) for v in (p, dp, a, da, b, db, c, dc)], float(s), float(tmax))


# --------------------------------------------------------------- problem
@dataclass
class Problem:
    """One contact problem: slave (tactile) and master surfaces + parameters."""
    xs: np.ndarray
    ts: np.ndarray
    xm: np.ndarray
    tm: np.ndarray
    rule_n: int = 2
    kappa: float = 1e5
    dhat: float = 1e-3
    delta_T: float = 0.0
    g_ref: np.ndarray | None = None
    xs_rest: np.ndarray | None = None
    rule: np.ndarray = field(init=False)

    def __post_init__(self):
        self.xs = _f64(self.xs)
        self.xm = _f64(self.xm)
        self.ts = _i32(self.ts)
        self.tm = _i32(self.tm)
        self.rule = stroud_rule(self.rule_n)
        if self.xs_rest is None:
            self.xs_rest = self.xs
        self.xs_rest = _f64(self.xs_rest)
        if self.g_ref is not None:
            self.g_ref = _f64(self.g_ref)

    @property
    def nq(self):
        return self.rule.shape[0]

    @property
    def Ns(self):
        return self.ts.shape[0] * self.nq

    @property
    def Vs(self):
        return self.xs.shape[0]

    @property
    def Vm(self):
        return self.xm.shape[0]

    def with_positions(self, xs=None, xm=None):
        p = Problem(self.xs if xs is None else xs, self.ts, self.xm if xm is None else xm, self.tm,
                    self.rule_n, self.kappa, self.dhat, self.delta_T, self.g_ref, self.xs_rest)
        return p


@dataclass
class NarrowResult:
    M: np.ndarray      # [Ns] int32, -1 inactive
    g: np.ndarray      # [Ns]
    bm: np.ndarray     # [Ns, 3]
    flags: np.ndarray  # [Ns] int32 ambiguity flags


def narrow(P: Problem, use_grid: bool = True) -> NarrowResult:
    Ns = P.Ns
    M = np.empty(Ns, np.int32)
    g = np.empty(Ns)
    bm = np.empty((Ns, 3))
    fl = np.empty(Ns, np.int32)
    bad = C.c_int64(-1)
    rc = lib().ora_narrow(P.Vs, P.ts.shape[0], _p(P.xs), _p(P.ts), P.Vm, P.tm.shape[0], _p(P.xm),
                          _p(P.tm), P.nq, _p(P.rule), P.dhat, _p(P.g_ref), int(use_grid),
                          _p(M), _p(g), _p(bm), _p(fl), C.byref(bad))
    if rc != OK:
        raise OracleError(rc, bad.value)
    return NarrowResult(M, g, bm, fl)


@dataclass
class Assembly:
    energy: float
    Ek: np.ndarray
    c1: np.ndarray
    c2: np.ndarray
    press: np.ndarray
    grad: np.ndarray          # [Vs+Vm, 3]
    row_ptr: np.ndarray | None
    col: np.ndarray | None
    val: np.ndarray | None    # [nnzb, 3, 3]
    max_clamped: float

    def dense_hessian(self):
        V = self.row_ptr.shape[0] - 1
        H = np.zeros((3 * V, 3 * V))
        for r in range(V):
            for j in range(self.row_ptr[r], self.row_ptr[r + 1]):
                c = self.col[j]
                H[3 * r:3 * r + 3, 3 * c:3 * c + 3] = self.val[j]
        return H


def assemble(P: Problem, M, delta_gap=None, kinematic=False, project=True, hessian=True) -> Assembly:
    Ns, Vt = P.Ns, P.Vs + P.Vm
    M = _i32(M)
    area = rest_area(P.xs_rest, P.ts)
    Ek, c1, c2, pr = (np.empty(Ns) for _ in range(4))
    grad = np.empty((Vt, 3))
    dg = None if delta_gap is None else _f64(delta_gap)
    nact = int((M >= 0).sum())
    cap = max(1, 36 * nact) if hessian else 0
    row_ptr = np.empty(Vt + 1, np.int64) if hessian else None
    col = np.empty(cap, np.int64) if hessian else None
    val = np.empty((cap, 3, 3)) if hessian else None
    E = C.c_double(0.0)
    nnzb = C.c_int64(0)
    clamped = C.c_double(0.0)
    bad = C.c_int64(-1)
    rc = lib().ora_assemble(P.Vs, P.ts.shape[0], _p(P.xs), _p(P.ts), P.Vm, P.tm.shape[0], _p(P.xm),
                            _p(P.tm), P.nq, _p(P.rule), _p(area), P.kappa, P.dhat, P.delta_T,
                            _p(P.g_ref), _p(dg), _p(M), int(kinematic), int(project), C.byref(E),
                            _p(Ek), _p(c1), _p(c2), _p(pr), _p(grad), cap, _p(row_ptr), _p(col),
                            _p(val), C.byref(nnzb), C.byref(clamped), C.byref(bad))
    if rc != OK:
        raise OracleError(rc, bad.value)
    nb = nnzb.value
    return Assembly(E.value, Ek, c1, c2, pr, grad, row_ptr,
                    None if col is None else col[:nb].copy(),
                    None if val is None else val[:nb].copy(), clamped.value)


def frozen_energy(P: Problem, M, bm, xs_new, xm_new) -> float:
    """Energy of the samples selected at P's positions (master triangle M[k],
    its barycentric coordinates bm[k]) evaluated at new positions with every
    sample frozen (Sec. 4.2's gradient and Hessian approximation): the slave
    normal n_T at P's positions, the rule point, M[k] and bm[k], the weight,
    face weight and support radius.  Then g_k = n_T . (sum_j bm_j x_mj -
    sum_a bs_a x_sa) is affine in the positions.  +inf if a gap is <= 0."""
    xs_new, xm_new = _f64(xs_new), _f64(xm_new)
    w = weights(P)
    E = 0.0
    for k in np.nonzero(np.asarray(M) >= 0)[0]:
        T, q = divmod(int(k), P.nq)
        a, b, c = P.ts[T]
        e1, e2 = P.xs[b] - P.xs[a], P.xs[c] - P.xs[a]
        n = np.cross(e1, e2)
        n /= np.linalg.norm(n)
        xi, eta = P.rule[q, 0], P.rule[q, 1]
        xs_k = (1 - xi - eta) * xs_new[a] + xi * xs_new[b] + eta * xs_new[c]
        xm_k = sum(bm[k][j] * xm_new[P.tm[M[k], j]] for j in range(3))
        g = float(n @ (xm_k - xs_k))
        eps = P.dhat if P.g_ref is None else min(0.9 * P.g_ref[k], P.dhat)
        if g <= 0.0:
            return float("inf")
        if g < eps:
            gam = hermite(min(bm[k]), P.delta_T) if P.delta_T > 0 else 1.0
            E += P.kappa * w[k] * gam * barrier(g, eps)
    return E


def sample_geom(P: Problem, k: int, M: int):
    g = C.c_double(0.0)
    bm = np.empty(3)
    n = np.empty(3)
    rc = lib().ora_sample_geom(_p(P.xs), _p(P.ts), _p(P.xm), _p(P.tm), P.nq, _p(P.rule), int(k), int(M),
                               C.byref(g), _p(bm), _p(n))
    if rc != OK:
        raise OracleError(rc, k)
    return g.value, bm, n


def pressure_loss(P: Problem, M, ptarget, delta_gap=None):
    Vt = P.Vs + P.Vm
    dLdx = np.empty((Vt, 3))
    dLdd = np.empty(P.Ns)
    dg = None if delta_gap is None else _f64(delta_gap)
    L = lib().ora_pressure_loss(P.Vs, P.ts.shape[0], _p(P.xs), _p(P.ts), P.Vm, _p(P.xm), _p(P.tm),
                                P.nq, _p(P.rule), P.kappa, P.dhat, P.delta_T, _p(P.g_ref), _p(dg),
                                _p(_i32(M)), _p(_f64(ptarget)), _p(dLdx), _p(dLdd))
    return L, dLdx, dLdd


def hvp(P: Problem, M, c2, vx, vd=None):
    Vt = P.Vs + P.Vm
    ox = np.empty((Vt, 3))
    od = np.empty(P.Ns)
    lib().ora_hvp(P.Vs, P.ts.shape[0], _p(P.xs), _p(P.ts), P.Vm, _p(P.xm), _p(P.tm), P.nq,
                  _p(P.rule), _p(_i32(M)), _p(_f64(c2)), _p(_f64(vx)),
                  _p(None if vd is None else _f64(vd)), _p(ox), _p(od))
    return ox, od


def step_linear(P: Problem, M, dxs, dxm=None):
    return lib().ora_step_linear(P.ts.shape[0], _p(P.xs), _p(P.ts), _p(P.xm), _p(P.tm), P.nq,
                                 _p(P.rule), _p(_i32(M)), _p(_f64(dxs)),
                                 _p(None if dxm is None else _f64(dxm)))


@dataclass
class StepBound:
    alpha: float
    alpha_lin: float
    alpha_accd: float
    n_swept: int


def ccd_step(P: Problem, M, dxs, dxm=None, s=0.1, use_grid=True) -> StepBound:
    ns = C.c_int64(0)
    al = C.c_double(0.0)
    aa = C.c_double(0.0)
    a = lib().ora_ccd_step(P.Vs, P.ts.shape[0], _p(P.xs), _p(P.ts), P.Vm, P.tm.shape[0], _p(P.xm),
                           _p(P.tm), P.nq, _p(P.rule), _p(_i32(M)), _p(_f64(dxs)),
                           _p(None if dxm is None else _f64(dxm)), float(s), int(use_grid),
                           C.byref(ns), C.byref(al), C.byref(aa))
    return StepBound(a, al.value, aa.value, ns.value)


def swept_count(P: Problem, dxs, dxm=None, pad_rel: float = 0.0, pad_abs: float = 0.0,
                use_grid: bool = True) -> int:
    """Number of (sample point, master triangle) pairs whose boxes over the
    linear motion overlap (the pairs the step bound's additive CCD runs
    over; Eq. (global_ccd) and the additive CCD reading).  A margin pad_rel
    |c| + pad_abs grows every box bound outward (a count for boxes widened
    by rounding); 0 is the definition."""
    return int(lib().ora_swept_count(P.ts.shape[0], _p(P.xs), _p(P.ts), P.tm.shape[0], _p(P.xm), _p(P.tm),
                                     P.nq, _p(P.rule), _p(_f64(dxs)), _p(None if dxm is None else _f64(dxm)),
                                     float(pad_rel), float(pad_abs), int(use_grid)))


def weights(P: Problem) -> np.ndarray:
    """Per-sample mortar weights w_k = 2 A_rest(T) what_q."""
    area = rest_area(P.xs_rest, P.ts)
    return (2.0 * area[:, None] * P.rule[None, :, 2]).ravel()
