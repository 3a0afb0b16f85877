"""Implicit step on the GPU against the oracle (float64 throughout).

* the library's stiffness equals the oracle's element assembly;
* inertial + elastic energy and gradient match;
* PCG solves (M/dt^2 + K + H) d = b like a direct sparse solve;
* three Newton steps of a 16x16x4 gel block pushed against a sphere end at
  the oracle's positions (both converge to |grad E|_inf <= 1e-6 F_ref).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from gen import meshes
from gpu_helpers import need_gpu, to_dev
from oracle import fem as ofem

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

E_Y, NU, RHO, DT = 3e5, 0.45, 1000.0, 1e-3


def _scene(n=16, nz=4, h=3.125e-4, R=3e-3, gap=2e-5):
    X, tets, top, bottom = meshes.tet_block(n, n, nz, h)
    xm, tm = meshes.icosphere(3, R)
    c = np.array([n * h / 2, n * h / 2, nz * h + R + gap])
    xm = xm + c
    return X, tets, top, bottom, xm, tm


def _gpu_parts(X, tets, top, bottom, xm, tm):
    from paper_2605_24339_amd import Context
    from paper_2605_24339_amd.fem import Fem
    f = Fem(X, tets, E_Y, NU, RHO, DT, bottom)
    ctx = Context.single(top, tm, X.shape[0], xm.shape[0], rule_n=2, kappa=1e5, dhat=1e-3,
                         dtype=torch.float64, kinematic=True)
    ctx.build_samples(to_dev(X, torch.float64))
    return f, ctx


def test_stiffness_energy_and_solve_match_oracle():
    need_gpu()
    X, tets, top, bottom, xm, tm = _scene(n=6, nz=3)
    f, ctx = _gpu_parts(X, tets, top, bottom, xm, tm)
    Kg = f.stiffness()
    V = X.shape[0]
    Kd = sp.bsr_matrix((Kg.val.cpu().numpy(), Kg.col.cpu().numpy(), Kg.row_ptr.cpu().numpy()),
                       shape=(3 * V, 3 * V)).toarray()
    Ko = ofem.stiffness(X, tets, E_Y, NU).toarray()
    assert np.abs(Kd - Ko).max() <= 1e-12 * np.abs(Ko).max()
    body = ofem.Body(X, tets, top, bottom, E_Y, NU, RHO, DT)
    rng = np.random.default_rng(1)
    x = X + rng.normal(size=X.shape) * 1e-6
    xt = X + rng.normal(size=X.shape) * 1e-6
    e, g = f.energy(to_dev(x, torch.float64), to_dev(xt, torch.float64))
    Eo, go = body.fem_energy_grad(x, xt)
    go[body.fixed] = 0
    assert abs(e.item() / Eo - 1) < 1e-12
    assert np.abs(g.cpu().numpy() - go).max() <= 1e-12 * np.abs(go).max()
    # solve with a contact Hessian from a real assembly
    xs = to_dev(X, torch.float64)
    XM = to_dev(xm, torch.float64)
    ctx.broadphase(xs, XM)
    A = ctx.assemble(xs, XM)
    assert int(ctx.status().nnzb) > 0
    Hd = sp.bsr_matrix((A.hessian.val.cpu().numpy(), A.hessian.col.cpu().numpy(),
                        A.hessian.row_ptr.cpu().numpy()), shape=(3 * V, 3 * V))
    b = rng.normal(size=(V, 3))
    d, it, rr = f.solve(A.hessian, to_dev(b, torch.float64), rtol=1e-12, max_iter=20000)
    fr = body.free
    Asys = (sp.diags(np.repeat(body.m, 3) / DT ** 2) + body.K + Hd).tocsr()[fr][:, fr]
    dref = np.zeros(3 * V)
    dref[fr] = spla.spsolve(Asys.tocsc(), b.ravel()[fr])
    assert np.abs(d.cpu().numpy().ravel() - dref).max() <= 1e-9 * np.abs(dref).max()
    y = f.apply(A.hessian, to_dev(dref.reshape(-1, 3), torch.float64)).cpu().numpy().ravel()
    assert np.abs(y[fr] - b.ravel()[fr]).max() <= 1e-9 * np.abs(b).max()


def test_newton_steps_match_oracle():
    need_gpu()
    from paper_2605_24339_amd.newton import ImplicitSolver
    h = 3.125e-4
    X, tets, top, bottom, xm, tm = _scene()
    f, ctx = _gpu_parts(X, tets, top, bottom, xm, tm)
    f_ref = E_Y * h * h
    solver = ImplicitSolver(f, ctx, f_ref, tol=1e-6)
    body = ofem.Body(X, tets, top, bottom, E_Y, NU, RHO, DT)
    P_of = lambda x: oracle.Problem(x, top, xm, tm, 2, 1e5, 1e-3, 0.0, None, X)
    XM = to_dev(xm, torch.float64)
    x_g = to_dev(X, torch.float64)
    v_g = torch.zeros_like(x_g)
    x_o, v_o = X.copy(), np.zeros_like(X)
    fixed_pos = X.copy()
    for step in range(3):
        fixed_pos[bottom, 2] += 2e-5
        xn_g, st = solver.solve_step(x_g, v_g, XM, to_dev(fixed_pos, torch.float64))
        assert st.converged, (step, st)
        v_g = (xn_g - x_g) / DT
        x_g = xn_g
        xn_o, so = ofem.newton_step(body, P_of, x_o, v_o, fixed_pos, 1e5, 1e-3, 2, xm, tol=1e-6, f_ref=f_ref)
        assert so["residual"] <= 1e-6
        v_o = (xn_o - x_o) / DT
        x_o = xn_o
        err = np.abs(x_g.cpu().numpy() - x_o).max()
        assert err <= 1e-8, (step, err)
    # the block was pushed into contact
    ctx.broadphase(x_g, XM)
    ctx.assemble(x_g, XM, grad=False, hessian=False)
    assert int(ctx.status().n_active) > 0
