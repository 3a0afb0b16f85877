"""Pins of the oracle's quadrature rule, barrier and Hermite step.

Rule: exactness on monomials over the reference triangle, where
int xi^a eta^b = a! b! / (a+b+2)!, positive weights, total 1/2, and the
hand-derived closed form of the 2x2 rule.  Barrier: the IPC log barrier's
closed-form values, its C^2 contact with zero at the support edge, signs on
(0, eps), and derivatives against central differences.  Hermite step: the
values and C^1 ends of Eq. (smoothstep).
"""
import math

import numpy as np
import pytest

import oracle
from oracle.rule import stroud_rule


def _mono(a, b):
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_rule_exact_to_degree_2n_minus_1(n):
    r = stroud_rule(n)
    assert r.shape == (n * n, 3)
    assert np.all(r[:, 2] > 0)
    assert abs(r[:, 2].sum() - 0.5) < 1e-15
    xi, eta, w = r.T
    assert np.all(xi > 0) and np.all(eta > 0) and np.all(xi + eta < 1)
    for a in range(2 * n):
        for b in range(2 * n - a):
            q = np.sum(w * xi ** a * eta ** b)
            assert abs(q - _mono(a, b)) < 1e-15, (a, b)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_rule_not_exact_at_degree_2n(n):
    # the degree bound is sharp: some monomial of degree 2n is missed
    xi, eta, w = stroud_rule(n).T
    errs = [abs(np.sum(w * xi ** a * eta ** (2 * n - a)) - _mono(a, 2 * n - a)) for a in range(2 * n + 1)]
    assert max(errs) > 1e-6


def test_rule_closed_form_n1_n2():
    r1 = stroud_rule(1)
    assert np.allclose(r1, [[1 / 3, 1 / 3, 0.5]], atol=1e-15)
    # Gauss-Jacobi(1,0) on [0,1]: roots of u^2 - 4/5 u + 1/10,
    # weights (9 +- sqrt6)/36; Gauss-Legendre on [0,1]: 1/2 -+ sqrt3/6, 1/2.
    s6, s3 = math.sqrt(6), math.sqrt(3)
    u = [(4 - s6) / 10, (4 + s6) / 10]
    W = [(9 + s6) / 36, (9 - s6) / 36]
    v = [0.5 - s3 / 6, 0.5 + s3 / 6]
    r2 = stroud_rule(2)
    for i in range(2):
        for j in range(2):
            q = i * 2 + j
            assert abs(r2[q, 0] - u[i]) < 1e-15
            assert abs(r2[q, 1] - v[j] * (1 - u[i])) < 1e-15
            assert abs(r2[q, 2] - W[i] * 0.5) < 1e-15


def test_barrier_closed_form_values():
    eps = 1e-3
    g = eps / math.e
    # B(eps/e) = -(eps/e - eps)^2 ln(1/e) = eps^2 (1 - 1/e)^2
    assert abs(oracle.barrier(g, eps) - eps ** 2 * (1 - 1 / math.e) ** 2) < 1e-20
    # B'(g) = -2 (g - eps) ln(g/eps) - (g - eps)^2 / g at g = eps/e
    d = g - eps
    assert abs(oracle.barrier_d1(g, eps) - (2 * d - d * d / g)) < 1e-15
    assert abs(oracle.barrier_d2(g, eps) - (2 - 4 * d / g + d * d / (g * g))) < 1e-12


def test_barrier_zero_at_and_beyond_support():
    eps = 1e-3
    for g in (eps, 1.5 * eps, 10.0):
        assert oracle.barrier(g, eps) == 0.0
        assert oracle.barrier_d1(g, eps) == 0.0
        assert oracle.barrier_d2(g, eps) == 0.0
    # C^2 contact: at g = eps (1 - d) the leading terms are
    # B ~ eps^2 d^3, B' ~ -3 eps d^2, B'' ~ 6 d
    dd = 1e-6
    g = eps * (1 - dd)
    assert abs(oracle.barrier(g, eps) / (eps ** 2 * dd ** 3) - 1) < 1e-4
    assert abs(oracle.barrier_d1(g, eps) / (-3 * eps * dd ** 2) - 1) < 1e-4
    assert abs(oracle.barrier_d2(g, eps) / (6 * dd) - 1) < 1e-4


def test_barrier_signs_on_support():
    eps = 1e-3
    for g in np.geomspace(1e-9, eps * (1 - 1e-9), 200):
        assert oracle.barrier(g, eps) > 0
        assert oracle.barrier_d1(g, eps) < 0
        assert oracle.barrier_d2(g, eps) > 0


def test_barrier_derivatives_central_differences():
    eps = 1e-3
    for g in (2e-5, 1e-4, 4e-4, 9e-4):
        h = g * 1e-5
        fd1 = (oracle.barrier(g + h, eps) - oracle.barrier(g - h, eps)) / (2 * h)
        fd2 = (oracle.barrier_d1(g + h, eps) - oracle.barrier_d1(g - h, eps)) / (2 * h)
        assert abs(fd1 - oracle.barrier_d1(g, eps)) <= 1e-7 * abs(oracle.barrier_d1(g, eps))
        assert abs(fd2 - oracle.barrier_d2(g, eps)) <= 1e-7 * abs(oracle.barrier_d2(g, eps))


def test_hermite_step():
    d = 0.05
    assert oracle.hermite(-1.0, d) == 0.0
    assert oracle.hermite(0.0, d) == 0.0
    assert oracle.hermite(d, d) == 1.0
    assert oracle.hermite(2 * d, d) == 1.0
    assert abs(oracle.hermite(d / 2, d) - 0.5) < 1e-15
    # 3t^2 - 2t^3 at t = 0.25
    assert abs(oracle.hermite(0.25 * d, d) - (3 * 0.0625 - 2 * 0.015625)) < 1e-15
    # C^1: slope -> 0 at both ends
    h = 1e-7 * d
    assert abs((oracle.hermite(h, d) - oracle.hermite(0, d)) / h) < 1e-4
    assert abs((oracle.hermite(d, d) - oracle.hermite(d - h, d)) / h) < 1e-4
