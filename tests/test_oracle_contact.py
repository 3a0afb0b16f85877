"""Pins of the oracle's contact samples, energy, gradient and Hessian.

* flat punch on a flat pad (non-matching meshes, uniform gap g0): every
  sample has g = g0 and master barycentrics equal to the planar ones; the
  pressure is uniform, -kappa B'(g0); the total normal force is
  kappa |B'(g0)| A_pad; interior nodal forces are equal (the rule is exact
  for the linear hat functions);
* sample weights sum to the tactile area;
* zero energy, gradient and Hessian beyond dhat (bitwise);
* rigid-motion invariance of the energy;
* brute-force and grid candidate search select identically;
* full-energy finite differences of the oracle itself pin the gradient and
  Hessian where the frozen-sample approximation is exact to first order
  (flat punch, motion along the normal); a frozen-sample finite difference
  pins the general scatter (curved indenter);
* the Hessian is symmetric PSD and the eigen-projection of the rank-1
  virtual-point blocks is the identity;
* penetration and degenerate triangles are reported with their index.
"""
import numpy as np
import pytest

import oracle
from gen import meshes, workloads


def _punch(gap=3e-4, **kw):
    w = workloads.flat_punch(gap=gap, **kw)
    return w, workloads.to_problem(w)


def _planar_bary(p, a, b, c):
    # barycentrics of p in the xy-projected triangle (a, b, c), solved directly
    A = np.array([[a[0] - c[0], b[0] - c[0]], [a[1] - c[1], b[1] - c[1]]])
    l0, l1 = np.linalg.solve(A, p[:2] - c[:2])
    return np.array([l0, l1, 1 - l0 - l1])


def test_flat_punch_gaps_barycentrics_pressure():
    g0 = 3e-4
    w, P = _punch(g0)
    nr = oracle.narrow(P, use_grid=False)
    assert np.all(nr.M >= 0)
    assert np.all(nr.flags == 0) or np.all((nr.flags & ~oracle.FLAG_INSIDE) == 0)
    assert np.max(np.abs(nr.g - g0)) < 1e-15
    # sample position from the rule, barycentrics in the hit master triangle
    for k in range(0, P.Ns, 7):
        T, q = divmod(k, P.nq)
        xi, eta = P.rule[q, :2]
        s = P.xs[P.ts[T]]
        p = (1 - xi - eta) * s[0] + xi * s[1] + eta * s[2]
        m = P.xm[P.tm[nr.M[k]]]
        assert np.allclose(nr.bm[k], _planar_bary(p, *m), atol=1e-12)
        assert nr.bm[k].min() >= 0
    A = oracle.assemble(P, nr.M)
    pk = -P.kappa * oracle.barrier_d1(g0, P.dhat)
    assert np.max(np.abs(A.press / pk - 1)) < 1e-12
    # total normal force on the punch = kappa |B'(g0)| A_pad
    area = 1e-2 * 1e-2
    Fz_master = A.grad[P.Vs:, 2].sum()
    assert abs(Fz_master / (P.kappa * oracle.barrier_d1(g0, P.dhat) * area) - 1) < 1e-12
    # action = reaction; no tangential force
    assert abs(A.grad[:P.Vs, 2].sum() + Fz_master) < 1e-12 * abs(Fz_master)
    assert np.max(np.abs(A.grad[:, :2])) < 1e-15 * abs(Fz_master)
    # energy = kappa A B(g0)
    assert abs(A.energy / (P.kappa * area * oracle.barrier(g0, P.dhat)) - 1) < 1e-12
    # interior pad vertices carry equal force (2 A_tri each times pressure)
    n = 8
    ij = np.array([(i, j) for i in range(1, n) for j in range(1, n)])
    interior = ij[:, 0] * (n + 1) + ij[:, 1]
    f = A.grad[interior, 2]
    a_tri = 0.5 * (1e-2 / n) ** 2
    assert np.max(np.abs(f / (-P.kappa * oracle.barrier_d1(g0, P.dhat) * 2 * a_tri) - 1)) < 1e-12


def test_weights_sum_to_tactile_area():
    w = workloads.small_indent(fp32=False)
    P = workloads.to_problem(w)
    wk = oracle.weights(P)
    assert wk.shape == (P.Ns,)
    assert np.all(wk > 0)
    assert abs(wk.sum() / 1e-4 - 1) < 1e-13
    # noisy pad: the total is the sum of the rest triangle areas
    xs, ts = meshes.pad(12, 1e-2, noise=50e-6, rng=np.random.default_rng(5))
    e1 = xs[ts[:, 1]] - xs[ts[:, 0]]
    e2 = xs[ts[:, 2]] - xs[ts[:, 0]]
    tot = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1).sum()
    P2 = oracle.Problem(xs, ts, w.xm, w.tm, rule_n=3)
    assert abs(oracle.weights(P2).sum() / tot - 1) < 1e-13


def test_weights_come_from_the_rest_mesh():
    """A pad stretched in its plane by 1.3 (still flat, still under the
    punch at the same gap) keeps its rest weights: they sum to the rest
    area, the whole-triangle energy is kappa B(g0) times the rest area, and
    so are the clipped mortar samples' weights and energy."""
    from oracle import mortar
    g0 = 3e-4
    w, P0 = _punch(g0)
    xs = P0.xs.copy()
    xs[:, 0] *= 1.3
    P = oracle.Problem(xs, P0.ts, P0.xm, P0.tm, P0.rule_n, P0.kappa, P0.dhat, P0.delta_T, xs_rest=P0.xs)
    rest = 1e-4
    assert abs(oracle.weights(P).sum() / rest - 1) < 1e-12
    nr = oracle.narrow(P)
    assert np.all(nr.M >= 0)
    A = oracle.assemble(P, nr.M, hessian=False)
    assert abs(A.energy / (P.kappa * oracle.barrier(g0, P.dhat) * rest) - 1) < 1e-12
    MA = mortar.assemble(P, mortar.samples(P))
    assert abs(sum(s.w for s in MA.active) / rest - 1) < 1e-12
    assert abs(MA.energy / (P.kappa * oracle.barrier(g0, P.dhat) * rest) - 1) < 1e-12


def test_zero_beyond_dhat_bitwise():
    w, P = _punch(1.5e-3)
    nr = oracle.narrow(P)
    assert np.all(nr.M < 0)
    A = oracle.assemble(P, nr.M)
    assert A.energy == 0.0
    assert np.all(A.grad == 0.0)
    assert A.col.size == 0 and np.all(A.row_ptr == 0)
    # a gap just beyond dhat after imposing the assignment is also exactly zero
    w2, P2 = _punch(P.dhat * (1 + 1e-9))
    M = np.zeros(P2.Ns, np.int32)
    for k in range(P2.Ns):
        nr2 = oracle.narrow(P2.with_positions(xm=P2.xm - [0, 0, 1e-6]))
        M = nr2.M
        break
    A2 = oracle.assemble(P2, M)
    assert A2.energy == 0.0 and np.all(A2.grad == 0.0) and A2.col.size == 0


def test_rigid_motion_invariance(small):
    P = workloads.to_problem(small)
    nr = oracle.narrow(P)
    A = oracle.assemble(P, nr.M)
    R = meshes.random_rotation(np.random.default_rng(7))
    t = np.array([0.3, -0.2, 0.5])
    P2 = oracle.Problem(P.xs @ R.T + t, P.ts, P.xm @ R.T + t, P.tm, P.rule_n, P.kappa, P.dhat)
    nr2 = oracle.narrow(P2)
    safe = (nr.flags == 0) & (nr2.flags == 0)
    assert np.array_equal(nr.M[safe], nr2.M[safe])
    A2 = oracle.assemble(P2, nr2.M)
    assert abs(A2.energy / A.energy - 1) < 1e-9
    # gradient rotates with the body
    assert np.max(np.abs(A2.grad - A.grad @ R.T)) < 1e-6 * np.abs(A.grad).max()


def test_brute_force_equals_grid(small):
    P = workloads.to_problem(small)
    a = oracle.narrow(P, use_grid=False)
    b = oracle.narrow(P, use_grid=True)
    assert np.array_equal(a.M, b.M)
    assert np.array_equal(a.g, b.g)
    assert np.array_equal(a.flags, b.flags)
    # letter-shaped indenter on a coarse noisy pad (sharp edges, walls)
    xs, ts = meshes.pad(24, 1e-2, noise=50e-6, rng=np.random.default_rng(3))
    xm, tm = meshes.letter(refine=3)
    xm = meshes.place_above(xm, xs, 10e-6)
    P2 = oracle.Problem(xs, ts, xm, tm, rule_n=3)
    a = oracle.narrow(P2, use_grid=False)
    b = oracle.narrow(P2, use_grid=True)
    assert (a.M >= 0).sum() > 100
    assert np.array_equal(a.M, b.M) and np.array_equal(a.g, b.g)


def test_selection_is_the_closest_inside_opposing_hit(small):
    # brute force in numpy over every master triangle for a subset of samples
    P = workloads.to_problem(small)
    nr = oracle.narrow(P)
    rng = np.random.default_rng(0)
    for k in rng.choice(P.Ns, 60, replace=False):
        T, q = divmod(int(k), P.nq)
        s = P.xs[P.ts[T]]
        xi, eta = P.rule[q, :2]
        p = (1 - xi - eta) * s[0] + xi * s[1] + eta * s[2]
        n = np.cross(s[1] - s[0], s[2] - s[0])
        n /= np.linalg.norm(n)
        best, bt = -1, np.inf
        for M in range(P.tm.shape[0]):
            m = P.xm[P.tm[M]]
            N = np.cross(m[1] - m[0], m[2] - m[0])
            den = n @ N
            if den >= 0:
                continue
            t = N @ (m[0] - p) / den
            y = p + t * n
            # barycentrics by solving [f1 f2] b = y - m0 in least squares
            F = np.stack([m[1] - m[0], m[2] - m[0]], 1)
            b12 = np.linalg.lstsq(F, y - m[0], rcond=None)[0]
            b = np.array([1 - b12.sum(), *b12])
            if b.min() >= 0 and 0 < t < P.dhat and t < bt:
                best, bt = M, t
        if nr.flags[k] == 0:
            assert nr.M[k] == best
            if best >= 0:
                assert abs(nr.g[k] - bt) < 1e-15


def _frozen_energy(P, nr, A, x_s, x_m):
    # E(x) = sum kappa w gamma B(g_k(x)) with g_k(x) = n_k.(sum bm x_m - sum bs x_s),
    # n_k, bm, bs, w, gamma frozen at the assembly state
    wk = oracle.weights(P)
    E = 0.0
    for k in np.nonzero(nr.M >= 0)[0]:
        T, q = divmod(int(k), P.nq)
        xi, eta = P.rule[q, :2]
        bs = np.array([1 - xi - eta, xi, eta])
        _, bm, n = oracle.sample_geom(P, k, nr.M[k])
        g = n @ (bm @ x_m[P.tm[nr.M[k]]] - bs @ x_s[P.ts[T]])
        E += P.kappa * wk[k] * oracle.barrier(g, P.dhat)
    return E


def test_gradient_hessian_frozen_fd_curved(small):
    P = workloads.to_problem(small)
    nr = oracle.narrow(P)
    A = oracle.assemble(P, nr.M)
    H = A.dense_hessian()
    rng = np.random.default_rng(1)
    act_s = np.unique(P.ts[np.nonzero(nr.M >= 0)[0] // P.nq])
    act_m = np.unique(P.tm[nr.M[nr.M >= 0]])
    h = 1e-8
    x_s, x_m = P.xs.copy(), P.xm.copy()
    for v in list(rng.choice(act_s, 5)) + [P.Vs + int(j) for j in rng.choice(act_m, 5)]:
        for d in range(3):
            def E_at(delta):
                xs2, xm2 = x_s.copy(), x_m.copy()
                if v < P.Vs:
                    xs2[v, d] += delta
                else:
                    xm2[v - P.Vs, d] += delta
                return _frozen_energy(P, nr, A, xs2, xm2)
            fd = (E_at(h) - E_at(-h)) / (2 * h)
            an = A.grad[v, d]
            assert abs(fd - an) <= 1e-5 * np.abs(A.grad).max(), (v, d, fd, an)
    # Hessian: symmetric, PSD, and equal to second differences of the frozen
    # energy (four-point mixed differences, h = 1e-8 m) on entries coupling
    # the slave and master vertices of the samples with the smallest, median
    # and largest active gap
    assert np.max(np.abs(H - H.T)) <= 1e-14 * np.abs(H).max()
    ev = np.linalg.eigvalsh(H)
    assert ev.min() >= -1e-12 * ev.max()

    def E2(moves):
        xs2, xm2 = x_s.copy(), x_m.copy()
        for (v, d, dh) in moves:
            if v < P.Vs:
                xs2[v, d] += dh
            else:
                xm2[v - P.Vs, d] += dh
        return _frozen_energy(P, nr, A, xs2, xm2)

    act = np.nonzero(nr.M >= 0)[0]
    order = act[np.argsort(nr.g[act])]
    h, Hmax, big = 1e-8, np.abs(H).max(), 0
    for k in order[[0, len(order) // 2, -1]]:
        vs = [int(v) for v in P.ts[k // P.nq]] + [P.Vs + int(v) for v in P.tm[nr.M[k]]]
        for (v, d, u, e) in [(vs[0], 2, vs[1], 2), (vs[0], 2, vs[3], 2), (vs[4], 0, vs[5], 2),
                             (vs[2], 1, vs[2], 1), (vs[1], 2, vs[4], 1)]:
            fd = (E2([(v, d, h), (u, e, h)]) - E2([(v, d, h), (u, e, -h)]) - E2([(v, d, -h), (u, e, h)])
                  + E2([(v, d, -h), (u, e, -h)])) / (4 * h * h)
            an = H[3 * v + d, 3 * u + e]
            assert abs(fd - an) <= 1e-5 * Hmax, (v, d, u, e, fd, an)
            big += abs(an) >= 1e-2 * Hmax
    assert big >= 2       # some checked entries are large, so a wrong term would show


def test_gradient_and_hessian_full_fd_flat_punch():
    # flat punch: the frozen approximation is exact to first order for
    # motion along the normal, so the oracle's full energy differentiates to
    # its own gradient and Hessian
    g0 = 2e-4
    w, P = _punch(g0, n_pad=4, n_punch=3)
    nr = oracle.narrow(P)
    A = oracle.assemble(P, nr.M)
    H = A.dense_hessian()
    h = 1e-9
    Vt = P.Vs + P.Vm

    def full(xs, xm):
        Q = P.with_positions(xs, xm)
        return oracle.assemble(Q, oracle.narrow(Q).M)

    for v in range(Vt):
        xs_p, xm_p, xs_m, xm_m = P.xs.copy(), P.xm.copy(), P.xs.copy(), P.xm.copy()
        if v < P.Vs:
            xs_p[v, 2] += h
            xs_m[v, 2] -= h
        else:
            xm_p[v - P.Vs, 2] += h
            xm_m[v - P.Vs, 2] -= h
        Ap, Am = full(xs_p, xm_p), full(xs_m, xm_m)
        fd = (Ap.energy - Am.energy) / (2 * h)
        assert abs(fd - A.grad[v, 2]) <= 1e-6 * np.abs(A.grad[:, 2]).max(), v
        fdH = (Ap.grad[:, 2] - Am.grad[:, 2]) / (2 * h)
        # moving a master vertex along z keeps every hit point's barycentrics
        # (the ray is vertical), so its whole Hessian column is exact; moving a
        # slave vertex tilts n_T, which shifts the master barycentrics at
        # first order - the term the frozen-sample approximation leaves out -
        # so only the slave rows of that column are compared
        rows = slice(None) if v >= P.Vs else slice(0, P.Vs)
        assert np.max(np.abs(fdH[rows] - H[2::3, 3 * v + 2][rows])) <= 1e-5 * np.abs(H).max(), v


def test_psd_projection_of_rank1_blocks_is_identity(small):
    P = workloads.to_problem(small)
    nr = oracle.narrow(P)
    A = oracle.assemble(P, nr.M, project=True)
    B = oracle.assemble(P, nr.M, project=False)
    assert np.max(np.abs(A.val - B.val)) <= 1e-10 * np.abs(B.val).max()
    assert np.all(A.c2[nr.M >= 0] >= 0)
    # a negative coefficient is clamped: the projected block vanishes
    n = np.array([0.0, 0.6, 0.8])
    bm = np.array([0.2, 0.3, 0.5])
    H, cl = oracle.local_block12(-2.0, bm, n)
    assert np.max(np.abs(H)) < 1e-12 and abs(cl - 2.0 * (1 + bm @ bm)) < 1e-12
    H, cl = oracle.local_block12(3.0, bm, n)
    sh = np.array([-1, *bm])
    assert np.allclose(H, 3.0 * np.kron(np.outer(sh, sh), np.outer(n, n)), atol=1e-13)


def test_hvp_equals_bsr_times_vector(small):
    P = workloads.to_problem(small)
    nr = oracle.narrow(P)
    A = oracle.assemble(P, nr.M)
    H = A.dense_hessian()
    v = np.random.default_rng(2).normal(size=(P.Vs + P.Vm, 3))
    ox, od = oracle.hvp(P, nr.M, A.c2, v)
    assert np.max(np.abs(ox.ravel() - H @ v.ravel())) <= 1e-12 * np.abs(H @ v.ravel()).max()


def test_pressure_loss_gradient_fd():
    w, P = _punch(2e-4, n_pad=4, n_punch=3)
    nr = oracle.narrow(P)
    rng = np.random.default_rng(4)
    pt = rng.normal(size=P.Ns) * 10.0
    delta = rng.uniform(-1e-5, 1e-5, size=P.Ns)
    L, dLdx, dLdd = oracle.pressure_loss(P, nr.M, pt, delta)
    h = 1e-10
    for k in range(0, P.Ns, 5):
        dp, dm = delta.copy(), delta.copy()
        dp[k] += h
        dm[k] -= h
        fd = (oracle.pressure_loss(P, nr.M, pt, dp)[0] - oracle.pressure_loss(P, nr.M, pt, dm)[0]) / (2 * h)
        assert abs(fd - dLdd[k]) <= 1e-6 * np.abs(dLdd).max()
    for v in range(P.Vs + P.Vm):
        xs_p, xm_p, xs_m, xm_m = P.xs.copy(), P.xm.copy(), P.xs.copy(), P.xm.copy()
        if v < P.Vs:
            xs_p[v, 2] += h
            xs_m[v, 2] -= h
        else:
            xm_p[v - P.Vs, 2] += h
            xm_m[v - P.Vs, 2] -= h
        Lp = oracle.pressure_loss(P.with_positions(xs_p, xm_p), nr.M, pt, delta)[0]
        Lm = oracle.pressure_loss(P.with_positions(xs_m, xm_m), nr.M, pt, delta)[0]
        assert abs((Lp - Lm) / (2 * h) - dLdx[v, 2]) <= 1e-6 * np.abs(dLdx).max()


def test_penetration_and_degenerate_reported():
    w, P = _punch(-1e-4)
    with pytest.raises(oracle.OracleError) as e:
        oracle.narrow(P)
    assert e.value.code == oracle.E_PENETRATION and e.value.index == 0
    xs = P.xs.copy()
    ts = P.ts.copy()
    ts[5] = [ts[5][0], ts[5][0], ts[5][2]]
    P2 = oracle.Problem(xs, ts, w.xm + [0, 0, 4e-4], w.tm)
    with pytest.raises(oracle.OracleError) as e:
        oracle.narrow(P2)
    assert e.value.code == oracle.E_DEGENERATE and e.value.index == 5


def test_frozen_energy_is_the_assembled_energy_and_gradient():
    """The frozen-sample energy equals the assembled energy at the assembly
    point, its central finite differences give the assembled (frozen)
    gradient, and it is unchanged by a common translation."""
    import oracle
    from gen import workloads
    w = workloads.small_indent(fp32=False)
    P = workloads.to_problem(w)
    nr = oracle.narrow(P)
    A = oracle.assemble(P, nr.M, hessian=False)
    E0 = oracle.frozen_energy(P, nr.M, nr.bm, P.xs, P.xm)
    assert abs(E0 / A.energy - 1) < 1e-12
    rng = np.random.default_rng(5)
    ds = rng.normal(size=P.xs.shape) * 1e-6
    dm = rng.normal(size=P.xm.shape) * 1e-6
    h = 1e-3
    Ep = oracle.frozen_energy(P, nr.M, nr.bm, P.xs + h * ds, P.xm + h * dm)
    Em = oracle.frozen_energy(P, nr.M, nr.bm, P.xs - h * ds, P.xm - h * dm)
    fd = (Ep - Em) / (2 * h)
    an = float(np.sum(A.grad[:P.Vs] * ds) + np.sum(A.grad[P.Vs:] * dm))
    assert abs(fd - an) <= 1e-6 * abs(an)
    t = np.array([1e-3, -2e-3, 5e-4])
    assert abs(oracle.frozen_energy(P, nr.M, nr.bm, P.xs + t, P.xm + t) / E0 - 1) < 1e-12
