"""Oracle: linear-elastic tetrahedra and one implicit Euler step with GMCP
contact (test infrastructure only; FP64, numpy / scipy).

Incremental potential of one step (target x_tilde = x_t + dt v_t):
    E(x) = 1/2 sum_i m_i |x_i - x_tilde_i|^2 / dt^2 + Psi_el(x) + Psi_GMCP(x)
    Psi_el = sum_tets vol (mu eps:eps + lambda/2 tr(eps)^2),  eps = sym(grad u), u = x - X
with linear shape functions (grad N_1..3 = rows of Dm^-1, grad N_0 = -sum),
lumped mass rho vol / 4 per tet vertex, and an optional constant external
load f (the term -f . x).  One body against a prescribed master surface, or
two bodies in contact: the slave body's vertices first, then the master
body's, so the contact's vertex numbering is the bodies'.
Newton with a direct sparse solve,
step capped by the GMCP step bound, Armijo backtracking on the energy with
the iterate's contact samples frozen (the function the assembled gradient
and Hessian belong to); stop when |grad E|_inf <= tol * F_ref.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle import mortar as omortar


def lame(young, poisson):
    mu = young / (2.0 * (1.0 + poisson))
    lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson))
    return mu, lam


def shape_gradients(X, tets):
    """grad N [n_tet, 4, 3] and volumes [n_tet]."""
    p = X[tets]
    Dm = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], axis=2)  # columns
    inv = np.linalg.inv(Dm)
    g = np.empty((tets.shape[0], 4, 3))
    g[:, 1:] = inv            # row a of Dm^-1 = grad N_{a+1}
    g[:, 0] = -inv.sum(axis=1)
    vol = np.abs(np.linalg.det(Dm)) / 6.0
    return g, vol


def stiffness(X, tets, young, poisson):
    """K (3V x 3V, scipy CSR): the Hessian of Psi_el, assembled element by element."""
    mu, lam = lame(young, poisson)
    g, vol = shape_gradients(X, tets)
    n = tets.shape[0]
    I = np.eye(3)
    rows, cols, vals = [], [], []
    for a in range(4):
        for b in range(4):
            dab = np.einsum("ni,ni->n", g[:, a], g[:, b])
            blk = vol[:, None, None] * (mu * dab[:, None, None] * I[None]
                                        + mu * np.einsum("ni,nk->nik", g[:, b], g[:, a])
                                        + lam * np.einsum("ni,nk->nik", g[:, a], g[:, b]))
            for i in range(3):
                for k in range(3):
                    rows.append(3 * tets[:, a] + i)
                    cols.append(3 * tets[:, b] + k)
                    vals.append(blk[:, i, k])
    V = X.shape[0]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * V, 3 * V))


def elastic_energy(X, tets, young, poisson, x):
    """Psi_el evaluated element by element from its definition."""
    mu, lam = lame(young, poisson)
    g, vol = shape_gradients(X, tets)
    u = (x - X)[tets]                                  # [n, 4, 3]
    F = np.einsum("nai,naj->nij", u, g)                # grad u
    eps = 0.5 * (F + np.transpose(F, (0, 2, 1)))
    tr = np.trace(eps, axis1=1, axis2=2)
    psi = mu * np.einsum("nij,nij->n", eps, eps) + 0.5 * lam * tr * tr
    return float(np.sum(vol * psi))


def lumped_mass(X, tets, rho):
    _, vol = shape_gradients(X, tets)
    m = np.zeros(X.shape[0])
    for a in range(4):
        np.add.at(m, tets[:, a], rho * vol / 4.0)
    return m


class Body:
    """fixed: Dirichlet vertices (every component held); held: optional
    [V, 3] mask of further held components (rollers)."""

    def __init__(self, X, tets, top, fixed, young, poisson, rho, dt, held=None):
        self.X = np.asarray(X, float)
        self.tets = np.asarray(tets)
        self.top = np.asarray(top)
        self.fixed = np.zeros(self.X.shape[0], bool)
        self.fixed[np.asarray(fixed)] = True
        self.held = np.repeat(self.fixed[:, None], 3, axis=1)
        if held is not None:
            self.held |= np.asarray(held, bool)
        self.young, self.poisson, self.dt = young, poisson, dt
        self.K = stiffness(self.X, self.tets, young, poisson)
        self.m = lumped_mass(self.X, self.tets, rho)
        self.free = ~self.held.ravel()

    def fem_energy_grad(self, x, x_tilde):
        dt2 = self.dt * self.dt
        u = (x - self.X).ravel()
        Ku = self.K @ u
        dv = (x - x_tilde)
        E = 0.5 * np.sum(self.m[:, None] * dv * dv) / dt2 + 0.5 * u @ Ku
        g = (self.m[:, None] * dv / dt2).ravel() + Ku
        return E, g.reshape(-1, 3)


def stress(X, tets, young, poisson, x):
    """Cauchy stress of every tet (small strain): lambda tr(eps) I + 2 mu eps, [n, 3, 3]."""
    mu, lam = lame(young, poisson)
    g, _ = shape_gradients(X, tets)
    F = np.einsum("nai,naj->nij", (x - X)[tets], g)
    eps = 0.5 * (F + np.transpose(F, (0, 2, 1)))
    tr = np.trace(eps, axis1=1, axis2=2)
    return lam * tr[:, None, None] * np.eye(3)[None] + 2.0 * mu * eps


def newton_step(body: Body, P_of, x_t, v_t, fixed_pos, kappa, dhat, rule_n, xm, tol=1e-6, f_ref=1.0,
                max_newton=60, armijo=1e-4, x_start=None, n_slave=None, f_ext=None, mortar=False):
    """One implicit step; P_of(x) -> oracle.Problem at the positions x.
    One body (n_slave None): the slave surface belongs to the body and the
    master xm is prescribed (kinematic).  Two bodies (n_slave = vertices of
    the slave body): x holds both, the slave's first; the contact acts on
    both (no kinematic master).  f_ext: constant external load [V, 3].
    mortar: clipped mortar face samples (oracle.mortar) instead of
    whole-triangle samples; their step bound is the smaller of Eq. (ccd) over
    the clipped samples and the additive CCD of the rule points.
    Returns (x, stats dict)."""
    two = n_slave is not None
    split = (lambda z: (z[:n_slave], z[n_slave:])) if two else (lambda z: (z, None))
    f_ext = np.zeros_like(x_t) if f_ext is None else np.asarray(f_ext, float)
    dt = body.dt
    fx = body.held
    x_tilde = x_t + dt * v_t
    x_tilde[fx] = fixed_pos[fx]
    y = x_tilde.copy() if x_start is None else x_start.copy()
    y[fx] = fixed_pos[fx]

    def gmcp(x, need_h):
        P = P_of(x)
        if mortar:
            A = omortar.assemble(P, omortar.samples(P), kinematic=not two, with_hessian=need_h)
            return P, None, A
        nr = oracle.narrow(P)
        A = oracle.assemble(P, nr.M, kinematic=not two, project=False, hessian=need_h)
        return P, nr, A

    def frozen(P, nr, A, x):
        xs, xmm = split(x)
        xmm = xm if xmm is None else xmm
        if mortar:
            return omortar.frozen_energy(P, A.active, xs, xmm)
        return oracle.frozen_energy(P, nr.M, nr.bm, xs, xmm)

    def step_bound(P, nr, A, d):
        ds, dm = split(d)
        if not mortar:
            return oracle.ccd_step(P, nr.M, ds, dm).alpha
        none = np.full(P.Ns, -1, np.int32)       # no whole-triangle samples: the CCD part alone
        return min(1.0, omortar.linear_step(P, A.active, ds, dm), oracle.ccd_step(P, none, ds, dm).alpha_accd)

    def hessian(A):
        if not mortar:
            return sp.bsr_matrix((A.val, A.col, A.row_ptr[:V + 1]), shape=(3 * V, 3 * V)) if A.col.size else \
                sp.csr_matrix((3 * V, 3 * V))
        H = sp.lil_matrix((3 * V, 3 * V))
        for (i, j), B in A.blocks.items():
            H[3 * i:3 * i + 3, 3 * j:3 * j + 3] = B
        return H.tocsr()

    V = x_t.shape[0]
    P, nr, A = gmcp(x_t, False)
    a0 = step_bound(P, nr, A, y - x_t)
    x = x_t + a0 * (y - x_t)
    x[fx] = fixed_pos[fx]
    stats = dict(newton_iters=0, assemblies=0, energy_evals=0, start_alpha=a0, residual=np.inf)
    for _ in range(max_newton):
        Ef, gf = body.fem_energy_grad(x, x_tilde)
        Ef -= float(np.sum(f_ext * x))
        P, nr, A = gmcp(x, True)
        stats["assemblies"] += 1
        g = gf - f_ext + A.grad[:V]
        g[fx] = 0.0
        stats["residual"] = np.abs(g).max() / f_ref
        if stats["residual"] <= tol:
            break
        stats["newton_iters"] += 1
        Hb = hessian(A)
        Asys = sp.diags(np.repeat(body.m, 3) / dt ** 2) + body.K + Hb
        fr = body.free
        d = np.zeros(3 * V)
        d[fr] = spla.spsolve(Asys.tocsr()[fr][:, fr].tocsc(), -g.ravel()[fr])
        d = d.reshape(-1, 3)
        slope = float(np.sum(g * d))
        alpha = min(1.0, step_bound(P, nr, A, d))
        # Armijo on the energy with this iterate's samples frozen: the function
        # whose gradient and Hessian the assembly gave (Sec. 4.2)
        E0 = Ef + frozen(P, nr, A, x)
        while True:
            xn = x + alpha * d
            Efn, _ = body.fem_energy_grad(xn, x_tilde)
            En = Efn - float(np.sum(f_ext * xn)) + frozen(P, nr, A, xn)
            stats["energy_evals"] += 1
            # Armijo, or a change below the energy's double-precision resolution
            if En <= E0 + armijo * alpha * slope or abs(En - E0) <= 64 * 2.2e-16 * abs(E0) or alpha < 1e-14:
                break
            alpha *= 0.5
        x = xn
    return x, stats


def patch_test(pt, kappa, mortar=False, rule_n=2, steps=4, tol=1e-10):
    """The contact patch test (Sec. 5, Table 1) solved quasi-statically:
    implicit steps with zero velocity (rho = 1, dt = 1) until the positions
    stop moving.  pt: the two-block scene (upper = slave body, its vertices
    first; rollers u_x = u_y = 0 on pt.roller; lower block's bottom held;
    pressure as nodal loads pt.f_ext).  Returns (x, per-step stats)."""
    Vs = pt.Vs
    held = np.zeros(pt.X.shape, bool)
    held[pt.roller, :2] = True
    body = Body(pt.X, pt.tets, pt.ts, pt.fixed, pt.young, pt.poisson, 1.0, 1.0, held=held)
    P_of = lambda x: oracle.Problem(x[:Vs], pt.ts, x[Vs:], pt.tm, rule_n, kappa, pt.dhat, 0.0, None, pt.X[:Vs])
    x, v = pt.X.copy(), np.zeros_like(pt.X)
    out = []
    for _ in range(steps):
        xn, st = newton_step(body, P_of, x, v, pt.X, kappa, pt.dhat, rule_n, None, tol=tol,
                             f_ref=pt.young * pt.h_top ** 2, max_newton=200, n_slave=Vs, f_ext=pt.f_ext,
                             mortar=mortar)
        out.append(st)
        moved = np.abs(xn - x).max()
        x = xn
        if moved <= 1e-12:
            break
    return x, out
