"""Implicit Euler step of a linear-elastic tet body in contact through GMCP:
Newton on the incremental potential with a CCD-capped backtracking line
search (the IPC solver structure the paper's contact model plugs into).
Each Newton iteration re-selects the contact samples (assembly at the
iterate); the line search tests the energy with those samples frozen, the
function whose gradient and Hessian the assembly returned.

    E(x) = 1/2 |x - x_tilde|^2_M / dt^2 + 1/2 (x - X)^T K (x - X) + Psi_GMCP(x)

The tactile surface (slave) is a boundary of the body; the indenter
(master) is prescribed for the step (kinematic master).  With a contact
context that is not kinematic, two bodies meet: the positions hold the
slave body's vertices first, then the master body's, which is the
contact's own vertex numbering, so its gradient and Hessian act on both
bodies unchanged.  An optional constant external load f adds -f . x.
Held components (Dirichlet vertices, rollers) move to their prescribed
values at the start of the step and stay there.

Every step runs on the GPU library: GMCP broad phase / assembly / step
bound (gmcp.h), FEM energy / gradient and the PCG solve (gmcp_fem.h); this
module holds only the control flow and the bookkeeping of counts.
Convergence: r = |grad E|_inf / F_ref <= tol with F_ref = E_young h^2
(h the element size), which does not depend on the starting point.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch


@dataclass
class StepStats:
    newton_iters: int = 0
    assemblies: int = 0        # full assemblies (energy, gradient, Hessian)
    energy_evals: int = 0      # energy-only evaluations in the line search
    cg_iters: int = 0
    residual: float = float("inf")
    start_alpha: float = 1.0
    converged: bool = False
    alphas: list = field(default_factory=list)
    x0: object = None          # the (filtered) starting point of the Newton iteration
    used_start: bool | None = None  # safeguarded start: the given start beat the plain one


class ImplicitSolver:
    """Newton solver for one body (slave) against a prescribed indenter."""

    def __init__(self, fem, contact, f_ref: float, tol: float = 1e-6, max_newton: int = 60,
                 armijo: float = 1e-4, cg_rtol: float = 1e-3, cg_max: int = 20000, f_ext=None):
        self.fem = fem
        # gmcp Context, float64; kinematic master: slave = body vertices;
        # otherwise slave body then master body (Vs + Vm = body vertices)
        self.contact = contact
        self.two_body = not contact.kinematic
        self.Vs = contact.Vs
        self.f_ext = f_ext
        self.f_ref = f_ref
        self.tol = tol
        self.max_newton = max_newton
        self.armijo = armijo
        self.cg_rtol = cg_rtol
        self.cg_max = cg_max

    # -------------------------------------------------------------- pieces
    def _sm(self, x, xm):
        """(slave, master) positions of the contact."""
        return (x[:self.Vs], x[self.Vs:]) if self.two_body else (x, xm)

    def _ccd(self, x, xm, d) -> float:
        d = d.contiguous()
        if self.two_body:
            a = self.contact.ccd_step(x[:self.Vs], x[self.Vs:], d[:self.Vs], d[self.Vs:])
        else:
            a = self.contact.ccd_step(x, xm, d)
        return float(a.min().item())

    def _ext(self, x) -> float:
        return 0.0 if self.f_ext is None else -float((self.f_ext * x).sum().item())

    def energy(self, x, x_tilde, xm) -> float:
        """Incremental potential with the contact samples re-selected at x."""
        e_fem, _ = self.fem.energy(x, x_tilde, grad=False)
        s, m = self._sm(x, xm)
        self.contact.broadphase(s, m)
        A = self.contact.assemble(s, m, grad=False, hessian=False)
        return float(e_fem.item() + A.energy.sum().item()) + self._ext(x)

    def model_energy(self, x, x_tilde, xm) -> float:
        """Incremental potential with the contact samples of the last
        assembly frozen: the function whose gradient and Hessian the
        assembly returned, so the Armijo test and the descent direction
        agree."""
        e_fem, _ = self.fem.energy(x, x_tilde, grad=False)
        return float(e_fem.item() + self.contact.energy_frozen(*self._sm(x, xm)).sum().item()) + self._ext(x)

    def gradient_system(self, x, x_tilde, xm):
        e_fem, g = self.fem.energy(x, x_tilde, grad=True)
        s, m = self._sm(x, xm)
        self.contact.broadphase(s, m)
        A = self.contact.assemble(s, m, grad=True, hessian=True)
        g = g + A.grad
        if self.f_ext is not None:
            g = g - self.f_ext
        g[self.fem.fixed] = 0.0
        E = float(e_fem.item() + A.energy.sum().item()) + self._ext(x)
        return E, g, A.hessian

    def feasible_start(self, x_t, y, xm) -> tuple:
        """x_t + alpha (y - x_t), alpha from the contact step bound (free
        components; held ones are set afterwards)."""
        d = (y - x_t).contiguous()
        s, m = self._sm(x_t, xm)
        self.contact.broadphase(s, m)
        self.contact.assemble(s, m, grad=False, hessian=False)
        a = self._ccd(x_t, xm, d)
        return x_t + a * d, a

    # ---------------------------------------------------------------- step
    def solve_step(self, x_t, v_t, xm, fixed_pos, x_start=None, safeguard=False, log=None) -> tuple:
        """One implicit step.  fixed_pos: positions of the Dirichlet vertices
        at the end of the step ([V, 3] tensor, only fixed rows are read).
        x_start: optional starting guess (the plain start is x_t + dt v_t);
        it passes the same feasibility filter as the plain start.  With
        safeguard, both filtered starts are evaluated (two energy-only
        evaluations) and the one with the lower incremental potential is
        used.  log(str), optional, receives one line per Newton iteration."""
        st = StepStats()
        fx = self.fem.fixed
        x_tilde = x_t + self.fem.dt * v_t
        x_tilde[fx] = fixed_pos[fx]
        y = x_tilde.clone() if x_start is None else x_start.clone()
        y[fx] = fixed_pos[fx]
        x, st.start_alpha = self.feasible_start(x_t, y, xm)
        x[fx] = fixed_pos[fx]
        if x_start is not None and safeguard:
            xp, ap = self.feasible_start(x_t, x_tilde.clone(), xm)
            xp[fx] = fixed_pos[fx]
            e_given = self.energy(x.contiguous(), x_tilde, xm)
            e_plain = self.energy(xp.contiguous(), x_tilde, xm)
            st.energy_evals += 2
            st.used_start = bool(e_given < e_plain)
            if not st.used_start:
                x, st.start_alpha = xp, ap
        x = x.contiguous()
        st.x0 = x.clone()
        for it in range(self.max_newton):
            E, g, H = self.gradient_system(x, x_tilde, xm)
            st.assemblies += 1
            st.residual = float(g.abs().max().item()) / self.f_ref
            if st.residual <= self.tol:
                st.converged = True
                break
            st.newton_iters += 1
            gn = float(g.norm().item())
            rtol = min(self.cg_rtol, max(1e-10, (st.residual / 10.0)))
            if log:
                log(f"  newton {it}: E {E:.6e} r {st.residual:.3e} active {int(self.contact.status().n_active)} "
                    f"cg rtol {rtol:.1e}")
            d, cg_it, cg_res = self.fem.solve(H, (-g).contiguous(), rtol=rtol, max_iter=self.cg_max)
            st.cg_iters += cg_it
            slope = float((g * d).sum().item())
            if not slope < 0.0:      # not a descent direction: fall back to steepest descent
                d = -g / max(gn, 1e-300)
                slope = float((g * d).sum().item())
            a_ccd = self._ccd(x, xm, d)
            a = min(1.0, a_ccd)
            E0 = self.model_energy(x, x_tilde, xm)
            while True:
                xn = (x + a * d).contiguous()
                En = self.model_energy(xn, x_tilde, xm)
                st.energy_evals += 1
                # Armijo, or a change below the energy's double-precision
                # resolution (near convergence the decrease is smaller than
                # the rounding of E, and the test cannot be decided)
                if En <= E0 + self.armijo * a * slope or abs(En - E0) <= 64 * 2.2e-16 * abs(E0) or a < 1e-14:
                    break
                a *= 0.5
            st.alphas.append(a)
            if log:
                log(f"    cg {cg_it} it, rel res {cg_res:.2e}; step {a:.3e} (bound {a_ccd:.3e}), "
                    f"|d|inf {float(d.abs().max()):.3e}")
            x = xn
        return x, st
