"""Pins of the two-body implicit solve on the contact patch test (Sec. 5,
Table 1): the analytical solution is sigma_zz = -p in both blocks and every
other stress component zero.

* matching interface meshes with whole-triangle samples: every sample's
  master point is the same barycentric point of the opposite triangle, so
  the nodal forces on both sides are the consistent ones and the uniform
  state is exact; the common gap then balances the pressure, kappa B'(g) =
  -p (B' from central differences of the barrier's definition);
* clipped mortar samples integrate over the exact overlaps, so the uniform
  state is exact on non-matching meshes too (the consistency the paper's
  face samples are built for);
* whole-triangle samples on non-matching meshes are not consistent: the
  error is well above the solver's, so the first two pins are not vacuous.
"""
import math

import numpy as np

from gen import workloads
from patch_helpers import oracle_patch, stress_errors


def test_matching_meshes_carry_the_uniform_stress():
    pt = workloads.patch_test(n_top=4, n_bot=4)
    kappa = 1e4
    x, st = oracle_patch(pt, kappa)
    assert all(s["residual"] <= 1e-10 for s in st)
    zz, spur = stress_errors(pt, x)
    assert zz <= 1e-8 and spur <= 1e-8 * pt.pressure
    # the gap is uniform (to the solve's resolution: |grad E| <= 1e-10 E h^2
    # fixes positions to about that over the stiffness E h) and balances the pressure
    gaps = x[:pt.Vs][pt.ts][:, :, 2].ravel().min(), x[:pt.Vs][pt.ts][:, :, 2].ravel().max()
    assert gaps[1] - gaps[0] <= 1e-10
    g = x[:pt.Vs][pt.ts][:, :, 2].min() - x[pt.Vs:][pt.tm][:, :, 2].max()
    eps = pt.dhat
    B = lambda t: -(t - eps) ** 2 * math.log(t / eps)
    h = 1e-9
    assert abs(kappa * (B(g + h) - B(g - h)) / (2 * h) + pt.pressure) <= 1e-5 * pt.pressure


def test_mortar_samples_pass_on_non_matching_meshes():
    pt = workloads.patch_test(n_top=4, n_bot=6)
    x, st = oracle_patch(pt, 1e6, mortar=True)
    assert all(s["residual"] <= 1e-10 for s in st)
    zz, spur = stress_errors(pt, x)
    assert zz <= 1e-8 and spur <= 1e-8 * pt.pressure


def test_whole_triangle_samples_are_not_consistent_on_non_matching_meshes():
    pt = workloads.patch_test(n_top=4, n_bot=6)
    x, st = oracle_patch(pt, 1e4)
    assert all(s["residual"] <= 1e-10 for s in st)
    zz, spur = stress_errors(pt, x)
    assert zz > 1e-3 and spur > 1e-3 * pt.pressure
