"""The contact patch test on the GPU (Sec. 5, Table 1): two deformable
blocks through the library's two-body Newton solve (FEM + GMCP without a
kinematic master + PCG + CCD line search), against the oracle's
quasi-static solve and the analytical uniform stress sigma_zz = -p.

* held single components (gmcp_fem_constrain): PCG and the operator agree
  with a direct sparse solve of the system with those components removed;
* whole-triangle samples on non-matching meshes: converged positions equal
  the oracle's (both solve to |grad E|_inf <= 1e-10 E h^2), hence the same
  (non-zero) stress errors;
* clipped mortar samples: the uniform stress is exact (to the solver's
  tolerance) for kappa = 1e4, 1e6, 1e8, and the positions equal the
  oracle's mortar solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from gen import workloads
from gpu_helpers import need_gpu, to_dev
from oracle import fem as ofem
from patch_helpers import oracle_patch, stress_errors

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_constrained_components_solve_like_a_reduced_direct_solve():
    need_gpu()
    from paper_2605_24339_amd.fem import Fem
    pt = workloads.patch_test(n_top=4, n_bot=4)
    f = Fem(pt.X, pt.tets, pt.young, pt.poisson, 1.0, 1.0, pt.fixed)
    f.constrain(pt.roller, 1 | 2)
    held = np.zeros(pt.X.shape, bool)
    held[pt.roller, :2] = True
    body = ofem.Body(pt.X, pt.tets, pt.ts, pt.fixed, pt.young, pt.poisson, 1.0, 1.0, held=held)
    assert np.array_equal(f.fixed.cpu().numpy(), body.held)
    V = pt.X.shape[0]
    rng = np.random.default_rng(3)
    b = rng.normal(size=(V, 3))
    d, it, rr = f.solve(None, to_dev(b, torch.float64), rtol=1e-12, max_iter=20000)
    fr = body.free
    A = (sp.diags(np.repeat(body.m, 3)) + body.K).tocsr()[fr][:, fr]
    ref = np.zeros(3 * V)
    ref[fr] = spla.spsolve(A.tocsc(), b.ravel()[fr])
    got = d.cpu().numpy().ravel()
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    assert np.all(got[~fr] == 0.0)
    # the operator removes held rows and columns
    z = rng.normal(size=(V, 3))
    y = f.apply(None, to_dev(z, torch.float64)).cpu().numpy().ravel()
    zf = z.ravel().copy()
    zf[~fr] = 0.0
    yref = (sp.diags(np.repeat(body.m, 3)) + body.K) @ zf
    assert np.abs(y[fr] - yref[fr]).max() <= 1e-12 * np.abs(yref).max()
    assert np.all(y[~fr] == 0.0)


def test_whole_triangle_patch_test_matches_oracle():
    need_gpu()
    from paper_2605_24339_amd import patchtest
    pt = workloads.patch_test(n_top=4, n_bot=6)
    x, st = patchtest.solve(pt, 1e6)
    assert all(s.converged for s in st)
    xo, so = oracle_patch(pt, 1e6)
    err = np.abs(x.cpu().numpy() - xo).max()
    assert err <= 1e-9, err
    e = patchtest.errors(pt, x)
    zz, spur = stress_errors(pt, xo)
    assert abs(e["sigma_zz_max_rel_err"] - zz) <= 1e-6 * zz
    assert abs(e["sigma_spur"] - spur) <= 1e-6 * spur


@pytest.mark.parametrize("kappa", [1e4, 1e6, 1e8])
def test_mortar_patch_test_is_exact(kappa):
    need_gpu()
    from paper_2605_24339_amd import patchtest
    pt = workloads.patch_test(n_top=4, n_bot=6)
    x, st = patchtest.solve(pt, kappa, mortar=True)
    assert all(s.converged for s in st)
    e = patchtest.errors(pt, x)
    assert e["sigma_zz_max_rel_err"] <= 1e-7 and e["sigma_spur"] <= 1e-7 * pt.pressure, e
    if kappa == 1e6:
        xo, _ = oracle_patch(pt, kappa, mortar=True)
        err = np.abs(x.cpu().numpy() - xo).max()
        assert err <= 1e-9, err
