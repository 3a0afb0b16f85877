"""Pins of the oracle's face weight, Hermite step, pressure, selection among
stacked master surfaces and adaptive support radius, each checked against
a property the paper or the mathematics fixes rather than the oracle's own
formula:

* the C^1 Hermite step, Eq. (smoothstep): its end values, the symmetry
  H(x) + H(delta - x) = 1, zero slope at both ends, monotone;
* with a face-weight width delta_T > 0 (samples near master edges get
  gamma < 1): energy, gradient and Hessian do not change under a cyclic
  relabelling of every master triangle's vertices, since f_T of
  Eq. (gamma) takes the smallest of the three master barycentrics,
  whichever vertex it belongs to;
* frozen-sample finite differences of each sample's own energy
  (Eq. (gmcp_potential), the coefficient kappa w gamma read off the
  sample's energy) pin the gradient and Hessian of Sec. 4.2 with gamma < 1;
* force balance: the pressure map weighted by the sample weights along the
  slave normals sums to the slave vertices' summed gradient (the gradient
  of Sec. 4.2 with grad g_k = -beta^s_a n on slave vertex a, the slave
  barycentrics summing to one);
* two master sheets stacked within the support radius: every sample selects
  the nearer one, at exactly its gap (the closest opposing hit);
* Eq. (adaptive_eps): a selected sample contributes if and only if its gap
  is below min(0.9 g_ref, dhat), checked just inside and just outside the
  boundary, in the selection and in the assembly;
* with partial face weights, central differences in the per-sample gap
  offsets pin the pressure loss's gradient and the offset part of the joint
  Hessian-vector product (the derivative of the assembly's dE/ddelta and
  gradient along one offset).
"""
import numpy as np
import pytest

import oracle
from gen import meshes, workloads

DELTA_T = 0.05


def test_hermite_step_properties():
    for delta in (0.05, 0.3, 1.0):
        assert oracle.hermite(0.0, delta) == 0.0 and oracle.hermite(-0.1, delta) == 0.0
        assert oracle.hermite(delta, delta) == 1.0 and oracle.hermite(2 * delta, delta) == 1.0
        xs = np.linspace(0.0, delta, 201)
        H = np.array([oracle.hermite(x, delta) for x in xs])
        assert np.all(np.diff(H) >= 0.0)
        for x in xs:
            assert abs(oracle.hermite(x, delta) + oracle.hermite(delta - x, delta) - 1.0) <= 1e-14
        # zero slope at both ends (C^1 joins with the constant pieces): the
        # one-sided difference quotients vanish linearly with the step
        for h in (1e-3 * delta, 1e-4 * delta):
            assert oracle.hermite(h, delta) / h <= 4.0 * h / delta ** 2
            assert (1.0 - oracle.hermite(delta - h, delta)) / h <= 4.0 * h / delta ** 2
        assert abs(oracle.hermite(0.5 * delta, delta) - 0.5) <= 1e-15


@pytest.fixture(scope="module")
def curved():
    P = workloads.to_problem(workloads.small_indent(delta_T=DELTA_T, fp32=False))
    nr = oracle.narrow(P)
    A = oracle.assemble(P, nr.M)
    return P, nr, A


def test_some_samples_have_partial_face_weight(curved):
    # the pins below need samples with 0 < gamma < 1: master barycentric
    # minimum inside (0, delta_T)
    P, nr, A = curved
    act = np.nonzero(nr.M >= 0)[0]
    mb = nr.bm[act].min(axis=1)
    part = (mb > 0.0) & (mb < DELTA_T)
    assert part.sum() >= 10 and (~part).sum() >= 10


def test_master_vertex_rotation_invariance(curved):
    P, nr, A = curved
    P2 = oracle.Problem(P.xs, P.ts, P.xm, P.tm[:, [1, 2, 0]].copy(), P.rule_n, P.kappa, P.dhat, P.delta_T)
    nr2 = oracle.narrow(P2)
    assert np.array_equal(nr.M, nr2.M)
    act = nr.M >= 0
    assert np.allclose(nr2.bm[act], nr.bm[act][:, [1, 2, 0]], rtol=0, atol=1e-12)
    A2 = oracle.assemble(P2, nr2.M)
    assert abs(A2.energy - A.energy) <= 1e-12 * abs(A.energy)
    assert np.allclose(A2.Ek, A.Ek, rtol=1e-10, atol=1e-14 * np.abs(A.Ek).max())
    assert np.allclose(A2.grad, A.grad, rtol=0, atol=1e-10 * np.abs(A.grad).max())
    assert np.array_equal(A2.row_ptr, A.row_ptr) and np.array_equal(A2.col, A.col)
    assert np.allclose(A2.val, A.val, rtol=0, atol=1e-10 * np.abs(A.val).max())


def _geom(P, k, M):
    T, q = divmod(int(k), P.nq)
    xi, eta = P.rule[q, :2]
    bs = np.array([1.0 - xi - eta, xi, eta])
    g, bm, n = oracle.sample_geom(P, int(k), int(M))
    return T, bs, bm, n, g


def test_frozen_fd_with_partial_face_weight(curved):
    # E_frozen(x) = sum_k (E_k / B(g_k)) B(g_k(x)), with g_k(x) affine in x
    # (normal, barycentrics and coefficient frozen at the assembly state);
    # its first and mixed second differences must match the assembled
    # gradient and Hessian, whatever kappa w gamma the oracle used
    P, nr, A = curved
    act = np.nonzero(nr.M >= 0)[0]
    frozen = []
    for k in act:
        T, bs, bm, n, g = _geom(P, k, nr.M[k])
        coef = A.Ek[k] / oracle.barrier(g, P.dhat)
        frozen.append((T, int(nr.M[k]), bs, bm, n, coef))

    def E(xs, xm):
        tot = 0.0
        for T, M, bs, bm, n, coef in frozen:
            g = n @ (bm @ xm[P.tm[M]] - bs @ xs[P.ts[T]])
            tot += coef * oracle.barrier(g, P.dhat)
        return tot

    def moved(moves):
        xs, xm = P.xs.copy(), P.xm.copy()
        for v, d, h in moves:
            if v < P.Vs:
                xs[v, d] += h
            else:
                xm[v - P.Vs, d] += h
        return E(xs, xm)

    # samples with a partial face weight, smallest and largest gaps among them
    mb = nr.bm[act].min(axis=1)
    part = act[(mb > 0.0) & (mb < DELTA_T)]
    part = part[np.argsort(nr.g[part])]
    H = A.dense_hessian()
    gmax, Hmax = np.abs(A.grad).max(), np.abs(H).max()
    h = 1e-8
    big = 0
    for k in part[[0, len(part) // 2, -1]]:
        T, M = divmod(int(k), P.nq)[0], int(nr.M[k])
        vs = [int(v) for v in P.ts[T]] + [P.Vs + int(v) for v in P.tm[M]]
        for v in (vs[0], vs[4]):
            for d in range(3):
                fd = (moved([(v, d, h)]) - moved([(v, d, -h)])) / (2 * h)
                assert abs(fd - A.grad[v, d]) <= 1e-5 * gmax, (k, v, d, fd, A.grad[v, d])
        for (v, d, u, e) in [(vs[0], 2, vs[1], 2), (vs[0], 2, vs[3], 2), (vs[4], 2, vs[5], 2), (vs[2], 2, vs[2], 2)]:
            fd = (moved([(v, d, h), (u, e, h)]) - moved([(v, d, h), (u, e, -h)]) - moved([(v, d, -h), (u, e, h)])
                  + moved([(v, d, -h), (u, e, -h)])) / (4 * h * h)
            an = H[3 * v + d, 3 * u + e]
            assert abs(fd - an) <= 1e-5 * Hmax, (k, v, d, u, e, fd, an)
            big += abs(an) >= 1e-3 * Hmax
    assert big >= 2


def test_pressure_force_balance(curved):
    P, nr, A = curved
    w = oracle.weights(P)
    F = np.zeros(3)
    for k in np.nonzero(nr.M >= 0)[0]:
        _, _, _, n, _ = _geom(P, k, nr.M[k])
        F += w[k] * A.press[k] * n
    G = A.grad[:P.Vs].sum(axis=0)
    assert np.abs(F).max() > 0.0
    assert np.allclose(F, G, rtol=0, atol=1e-10 * np.abs(G).max())


def _stacked(g1, g2, dhat=1e-3):
    # a flat pad (normal +z) under two flat master sheets facing it (normal
    # -z) at heights g1 < g2, each larger than the pad and meshed unlike it
    xs, ts = meshes.pad(6, 1e-2)
    sheets_x, sheets_t = [], []
    off = 0
    for z, shift in ((g1, 0.11), (g2, 0.23)):
        xm, tm = meshes.pad(5, 1.4e-2)
        xm[:, 0] += shift * 1.4e-2 / 5
        xm[:, 1] += 0.5 * shift * 1.4e-2 / 5
        xm[:, 2] = z
        sheets_x.append(xm)
        sheets_t.append(tm[:, [0, 2, 1]] + off)
        off += xm.shape[0]
    ntri_lower = sheets_t[0].shape[0]
    return (oracle.Problem(xs, ts, np.concatenate(sheets_x), np.concatenate(sheets_t), 2, 1e5, dhat, 0.0),
            ntri_lower)


def test_nearest_of_two_stacked_sheets():
    P, n_lower = _stacked(0.3e-3, 0.6e-3)
    nr = oracle.narrow(P)
    assert np.all(nr.M >= 0) and np.all(nr.M < n_lower)
    assert np.allclose(nr.g, 0.3e-3, rtol=1e-12, atol=0)
    # the upper sheet alone is selected once the lower one leaves the support
    P2, n_lower = _stacked(1.5e-3, 0.6e-3)
    nr2 = oracle.narrow(P2)
    assert np.all(nr2.M >= n_lower)
    assert np.allclose(nr2.g, 0.6e-3, rtol=1e-12, atol=0)


def test_adaptive_support_radius_boundary():
    g0 = 3e-4
    P = workloads.to_problem(workloads.flat_punch(gap=g0))
    nr = oracle.narrow(P)
    assert np.all(nr.M >= 0) and np.allclose(nr.g, g0, rtol=1e-12)
    rng = np.random.default_rng(4)
    inside = rng.random(P.Ns) < 0.5
    # eps_k = min(0.9 g_ref, dhat): just above g0 for the "inside" samples, just below for the others;
    # and g_ref large enough that dhat caps it for every tenth sample
    g_ref = np.where(inside, g0 / 0.9 * (1.0 + 1e-6), g0 / 0.9 * (1.0 - 1e-6))
    capped = np.arange(P.Ns) % 10 == 0
    g_ref[capped] = 1.0
    Pg = oracle.Problem(P.xs, P.ts, P.xm, P.tm, P.rule_n, P.kappa, P.dhat, P.delta_T, g_ref=g_ref)
    sel = oracle.narrow(Pg).M >= 0
    want = inside | capped
    assert np.array_equal(sel, want)
    # the assembly applies the same radius to samples selected without it
    A = oracle.assemble(Pg, nr.M)
    assert np.array_equal(A.Ek > 0.0, want)
    assert np.all(A.c1[~want] == 0.0) and np.all(A.c2[~want] == 0.0)
    # a capped sample's energy is the plain dhat barrier's
    k = int(np.nonzero(capped)[0][0])
    A0 = oracle.assemble(P, nr.M)
    assert A.Ek[k] == A0.Ek[k]


def _partial(P, nr, count=12):
    act = np.nonzero(nr.M >= 0)[0]
    mb = nr.bm[act].min(axis=1)
    part = act[(mb > 0.0) & (mb < DELTA_T)]
    return part[np.linspace(0, len(part) - 1, count).astype(int)]


def test_pressure_loss_offset_gradient_with_partial_face_weight(curved):
    P, nr, A = curved
    rng = np.random.default_rng(6)
    pt = A.press + rng.normal(size=P.Ns) * np.abs(A.press).max() * 0.1
    delta = rng.uniform(-1e-6, 1e-6, size=P.Ns) * (nr.M >= 0)
    _, _, dLdd = oracle.pressure_loss(P, nr.M, pt, delta)
    h = 1e-11
    scale = np.abs(dLdd).max()
    for k in _partial(P, nr):
        dp, dm = delta.copy(), delta.copy()
        dp[k] += h
        dm[k] -= h
        fd = (oracle.pressure_loss(P, nr.M, pt, dp)[0] - oracle.pressure_loss(P, nr.M, pt, dm)[0]) / (2 * h)
        assert abs(fd - dLdd[k]) <= 1e-5 * scale, (k, fd, dLdd[k])


def test_joint_hvp_offset_part(curved):
    # H [0; e_k] = (d/ddelta_k) [dE/dx; dE/ddelta]: the change of the
    # gradient and of c1 = dE/ddelta under a small offset of sample k's gap
    P, nr, A = curved
    h = 1e-10
    vx = np.zeros((P.Vs + P.Vm, 3))
    for k in _partial(P, nr, 6):
        vd = np.zeros(P.Ns)
        vd[k] = 1.0
        ox, od = oracle.hvp(P, nr.M, A.c2, vx, vd)
        dp, dm = np.zeros(P.Ns), np.zeros(P.Ns)
        dp[k], dm[k] = h, -h
        Ap, Am = oracle.assemble(P, nr.M, delta_gap=dp, hessian=False), oracle.assemble(P, nr.M, delta_gap=dm, hessian=False)
        fd_d = (Ap.c1 - Am.c1) / (2 * h)
        fd_x = (Ap.grad - Am.grad) / (2 * h)
        assert abs(od[k] - fd_d[k]) <= 1e-5 * abs(fd_d[k]) and od[k] > 0.0, (k, od[k], fd_d[k])
        assert np.all(od[np.arange(P.Ns) != k] == 0.0)
        assert np.allclose(ox, fd_x, rtol=0, atol=1e-5 * np.abs(fd_x).max()), k
