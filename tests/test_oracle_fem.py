"""Pins of the oracle's linear-elastic tetrahedra and implicit step.

* patch test: an affine displacement u = G X gives the energy
  V_total (mu eps:eps + lambda/2 tr(eps)^2) exactly (linear elements
  reproduce affine fields) and zero force at every interior vertex;
* the quadratic form 1/2 u^T K u equals the element-by-element energy;
* rigid translations and infinitesimal rotations are in the null space of K;
* K u equals central differences of the energy;
* the energy of a simple shear, a uniform dilation and a uniaxial strain
  equals the volume times G gamma^2 / 2, 9 K e^2 / 2 and M e^2 / 2 with
  the engineering moduli of an isotropic solid (shear G = E / (2 (1 + nu)),
  bulk K = E / (3 (1 - 2 nu)), P-wave M = E (1 - nu) / ((1 + nu) (1 - 2 nu))),
  which pins the Lame parameters the energy is written with;
* the lumped mass adds up to rho times the volume;
* with the indenter out of reach, the implicit step solves the linear
  system M (x - x_tilde)/dt^2 + K (x - X) = 0 on the free vertices.
"""
import numpy as np
import pytest

from gen import meshes
from oracle import fem


def _block(n=3, nz=2, h=1e-3):
    X, tets, top, bottom = meshes.tet_block(n, n, nz, h)
    return X, tets, top, bottom


def test_patch_test_affine_field():
    X, tets, top, bottom = _block()
    E, nu = 3e5, 0.45
    mu, lam = fem.lame(E, nu)
    G = np.array([[1e-3, 2e-4, -1e-4], [3e-4, -5e-4, 2e-4], [0.0, 1e-4, 7e-4]])
    x = X + X @ G.T
    eps = 0.5 * (G + G.T)
    vol = (3e-3) * (3e-3) * (2e-3)
    psi = mu * np.sum(eps * eps) + 0.5 * lam * np.trace(eps) ** 2
    assert abs(fem.elastic_energy(X, tets, E, nu, x) / (vol * psi) - 1) < 1e-12
    K = fem.stiffness(X, tets, E, nu)
    u = (x - X).ravel()
    assert abs(0.5 * u @ (K @ u) / (vol * psi) - 1) < 1e-12
    f = (K @ u).reshape(-1, 3)
    lo, hi = X.min(0), X.max(0)
    interior = np.all((X > lo + 1e-12) & (X < hi - 1e-12), axis=1)
    assert interior.sum() > 0
    assert np.abs(f[interior]).max() < 1e-12 * np.abs(f).max()


def test_energy_matches_engineering_moduli():
    X, tets, top, bottom = _block()
    vol = (3e-3) * (3e-3) * (2e-3)
    for E, nu in ((3e5, 0.45), (2e11, 0.3), (1e6, 0.0)):
        G = E / (2.0 * (1.0 + nu))
        K = E / (3.0 * (1.0 - 2.0 * nu))
        Mp = E * (1.0 - nu) / ((1.0 + nu) * (1.0 - 2.0 * nu))
        g, e = 2e-3, 1e-3
        shear = X.copy()
        shear[:, 0] += g * X[:, 1]                       # u_x = gamma y
        dil = X * (1.0 + e)                              # u = e X
        uni = X.copy()
        uni[:, 2] *= 1.0 + e                             # u_z = e z
        for x, want in ((shear, G * g * g / 2), (dil, 9.0 * K * e * e / 2), (uni, Mp * e * e / 2)):
            assert abs(fem.elastic_energy(X, tets, E, nu, x) / (vol * want) - 1) < 1e-12


def test_rigid_modes_in_null_space():
    X, tets, _, _ = _block()
    K = fem.stiffness(X, tets, 3e5, 0.45)
    scale = np.abs(K).max()
    for t in np.eye(3):
        assert np.abs(K @ np.tile(t, X.shape[0])).max() < 1e-12 * scale
    for w in np.eye(3):
        u = np.cross(w, X).ravel()
        assert np.abs(K @ u).max() < 1e-10 * scale
    assert abs(K - K.T).max() < 1e-12 * scale


def test_stiffness_is_energy_hessian_fd():
    X, tets, _, _ = _block(n=2, nz=1)
    K = fem.stiffness(X, tets, 3e5, 0.45)
    rng = np.random.default_rng(0)
    x = X + rng.normal(size=X.shape) * 1e-5
    u = (x - X).ravel()
    g = K @ u
    h = 1e-9
    for j in rng.choice(u.size, 12, replace=False):
        xp, xm = x.copy().ravel(), x.copy().ravel()
        xp[j] += h
        xm[j] -= h
        fd = (fem.elastic_energy(X, tets, 3e5, 0.45, xp.reshape(-1, 3))
              - fem.elastic_energy(X, tets, 3e5, 0.45, xm.reshape(-1, 3))) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * np.abs(g).max()


def test_lumped_mass_total():
    X, tets, _, _ = _block()
    m = fem.lumped_mass(X, tets, 1000.0)
    assert abs(m.sum() / (1000.0 * 3e-3 * 3e-3 * 2e-3) - 1) < 1e-12


def test_step_without_contact_solves_linear_system():
    X, tets, top, bottom = _block(n=4, nz=2)
    body = fem.Body(X, tets, top, bottom, 3e5, 0.45, 1000.0, 1e-3)
    from oracle import Problem
    xm, tm = meshes.icosphere(1, 1e-3)
    xm = xm + np.array([2e-3, 2e-3, 2e-3 + 5e-3])    # far above
    P_of = lambda x: Problem(x, top, xm, tm, 2, 1e5, 1e-3, 0.0)
    v = np.zeros_like(X)
    fixed_pos = X.copy()
    fixed_pos[bottom, 2] += 2e-5                        # plate pushed up
    x, st = fem.newton_step(body, P_of, X.copy(), v, fixed_pos, 1e5, 1e-3, 2, xm, tol=1e-10, f_ref=1.0)
    Ef, g = body.fem_energy_grad(x, np.where(body.fixed[:, None], fixed_pos, X))
    g[body.fixed] = 0
    assert np.abs(g).max() < 1e-9
    assert np.allclose(x[bottom], fixed_pos[bottom])
    assert x[:, 2].max() > X[:, 2].max()                 # the push travels up
