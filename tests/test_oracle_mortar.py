"""Pins of the clipped mortar face samples of the oracle (Sec. 4.1 face
samples, Sec. 4.2): the clipping against hand-computed polygons, exact
overlap areas and exact integrals of linear gaps for flat punches (which
whole-triangle samples only approximate), the projection property of every
sample, the gradient against finite differences of the frozen-sample
energy, and Eq. (ccd) over clipped samples against its closed form for
flat surfaces closing along the normal."""
import math

import numpy as np
import pytest

import oracle
from gen import meshes, workloads
from oracle import mortar


def _area(poly):
    a = 0.0
    for i in range(len(poly)):
        p, q = poly[i], poly[(i + 1) % len(poly)]
        a += p[0] * q[1] - q[0] * p[1]
    return abs(a) / 2


def test_clip_against_hand_polygons():
    # a triangle containing the reference triangle clips to it
    out = mortar.clip_by_reference([(-1, -1), (3, -1), (-1, 3)])
    assert abs(_area(out) - 0.5) < 1e-15 and len(out) == 3
    # a triangle inside is unchanged
    tri = [(0.1, 0.1), (0.3, 0.1), (0.1, 0.4)]
    out = mortar.clip_by_reference(tri)
    assert np.allclose(np.array(out), np.array(tri))
    # disjoint
    assert mortar.clip_by_reference([(2, 2), (3, 2), (2, 3)]) == []
    # the square [0.25, 0.75]^2 as two triangles: area above the diagonal u + v = 1 is cut
    sq = [(0.25, 0.25), (0.75, 0.25), (0.75, 0.75), (0.25, 0.75)]
    out = mortar.clip_by_reference(sq)
    assert abs(_area(out) - (0.25 - 0.125)) < 1e-15     # half of the square lies below u + v = 1
    # reversed orientation gives the same area
    assert abs(_area(mortar.clip_by_reference(sq[::-1])) - 0.125) < 1e-15


def _punch_problem(punch_length, n_pad=6, n_punch=5, gap=3e-4, rule_n=2, tilt=0.0):
    w = workloads.flat_punch(n_pad=n_pad, n_punch=n_punch, gap=gap, punch_length=punch_length, rule_n=rule_n)
    xm = w.xm.copy()
    xm[:, 2] += tilt * xm[:, 0]
    return oracle.Problem(w.xs, w.ts, xm, w.tm, rule_n, w.kappa, w.dhat, w.delta_T, None, w.xs), w


@pytest.mark.parametrize("punch,expect", [(1.4e-2, 1e-4), (6e-3, 3.6e-5)])
def test_flat_punch_weights_cover_the_exact_overlap(punch, expect):
    """Punch larger than the pad: the weights sum to the pad area; a
    smaller, shifted, independently meshed punch inside the pad: to the
    punch area.  Every gap equals the uniform gap and E = kappa B(g0) area."""
    P, w = _punch_problem(punch)
    S = mortar.samples(P)
    A = mortar.assemble(P, S)
    tot = sum(s.w for s in A.active)
    assert abs(tot / expect - 1) < 1e-12
    assert all(abs(s.g - 3e-4) < 1e-15 for s in A.active)
    assert abs(A.energy / (P.kappa * oracle.barrier(3e-4, P.dhat) * expect) - 1) < 1e-12
    for s in A.active:        # the master point projects onto the slave point
        xs_k = s.bs @ P.xs[P.ts[s.T]]
        xm_k = s.bm @ P.xm[P.tm[s.M]]
        assert np.linalg.norm(np.cross(xm_k - xs_k, s.n)) < 1e-15
        assert s.bm.min() >= -1e-12 and s.bs.min() >= -1e-12


def test_rotated_punch_overlap_against_lattice_count():
    """A punch rotated by 30 degrees about the pad normal: the weights sum
    to the overlap of the two squares, counted independently on a lattice."""
    P, w = _punch_problem(9e-3, n_pad=5, n_punch=4)
    c, s = math.cos(math.pi / 6), math.sin(math.pi / 6)
    Rz = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    P = oracle.Problem(P.xs, P.ts, P.xm @ Rz.T, P.tm, P.rule_n, P.kappa, P.dhat, 0.0, None, P.xs)
    tot = sum(s_.w for s_ in mortar.assemble(P, mortar.samples(P)).active)
    m = 1500
    t = (np.arange(m) + 0.5) / m * 1e-2 - 5e-3
    X, Y = np.meshgrid(t, t)
    U = c * X + s * Y - 0.13 * 9e-3 / 4          # coordinates in the punch frame (inverse rotation, shift)
    V = -s * X + c * Y - 0.07 * 9e-3 / 4
    inside = (np.abs(U) <= 4.5e-3) & (np.abs(V) <= 4.5e-3)
    ref = inside.mean() * 1e-4
    assert abs(tot / ref - 1) < 2e-3


@pytest.mark.parametrize("rule_n", [1, 2, 3])
def test_linear_gap_integrated_exactly(rule_n):
    """A tilted punch (gap linear in x): sum_k w_k g_k equals the exact
    integral of the gap over the covered pad area for every rule."""
    tilt = 0.02
    P, w = _punch_problem(1.4e-2, rule_n=rule_n, tilt=tilt)
    S = mortar.samples(P)
    tot = sum(s.w * s.g for s in S)
    # pad [-5, 5] mm^2 fully covered: integral of (g0 + tilt x) = g0 * area (x averages to 0 over the pad)
    assert abs(tot / (3e-4 * 1e-4) - 1) < 1e-12
    if rule_n >= 2:      # g x is quadratic: exact from degree 2n - 1 >= 2
        tot_x = sum(s.w * s.g * (s.bs @ P.xs[P.ts[s.T]])[0] for s in S)
        assert abs(tot_x / (tilt * (1e-2) ** 4 / 12) - 1) < 1e-10


def test_gradient_against_frozen_energy_differences():
    P, _ = _punch_problem(6e-3, n_pad=4, n_punch=3, gap=2e-4)
    rng = np.random.default_rng(2)
    P = oracle.Problem(P.xs, P.ts, P.xm + rng.uniform(-2e-5, 2e-5, size=P.xm.shape), P.tm, P.rule_n, P.kappa,
                       P.dhat, 0.0, None, P.xs)
    S = mortar.samples(P)
    A = mortar.assemble(P, S)

    def frozen(xs, xm):
        E = 0.0
        for s in A.active:
            g = s.n @ (s.bm @ xm[P.tm[s.M]] - s.bs @ xs[P.ts[s.T]])
            E += P.kappa * s.w * oracle.barrier(g, P.dhat)
        return E

    ds = rng.normal(size=P.xs.shape) * 1e-6
    dm = rng.normal(size=P.xm.shape) * 1e-6
    h = 1e-3
    fd = (frozen(P.xs + h * ds, P.xm + h * dm) - frozen(P.xs - h * ds, P.xm - h * dm)) / (2 * h)
    an = float(np.sum(A.grad[:P.Vs] * ds) + np.sum(A.grad[P.Vs:] * dm))
    assert abs(fd - an) <= 1e-6 * abs(an)
    # the Hessian blocks are symmetric PSD rank-one sums
    for (i, j), B in A.blocks.items():
        assert np.allclose(B, A.blocks[(j, i)].T, atol=1e-12 * np.abs(B).max())


def test_penetration_reported():
    P, _ = _punch_problem(6e-3, gap=-1e-5)
    with pytest.raises(oracle.OracleError) as e:
        mortar.samples(P)
    assert e.value.code == oracle.E_PENETRATION


def _single_master(heights=(3e-4, 3e-4, 3e-4)):
    """A flat pad under one opposing master triangle (vertices off the pad's edges)."""
    xs, ts = meshes.pad(6, 1e-2)
    xm = np.array([[-3.1e-3, -2.7e-3, heights[0]], [3.3e-3, -1.9e-3, heights[1]], [0.4e-3, 3.6e-3, heights[2]]])
    tm = np.array([[0, 2, 1]])      # normal along -z: opposing the pad
    return oracle.Problem(xs, ts, xm, tm, 2, 1e5, 1e-3, 0.0, None, xs)


def test_edge_and_point_samples_of_one_triangle():
    """Point samples: one per master vertex, at its height, weight 1; edge
    samples: the weights of every edge sum to its length over the pad, and
    sum w g integrates the (linear) gap along the edge exactly."""
    P = _single_master((3e-4, 5e-4, 4e-4))
    S = mortar.samples(P, features=True)
    pts = [s for s in S if s.kind == 0]
    assert sorted(int(s.mv[0]) for s in pts) == [0, 1, 2]
    for s in pts:
        assert s.w == 1.0 and abs(s.g - P.xm[s.mv[0], 2]) < 1e-15
    for a, b in ((0, 1), (1, 2), (0, 2)):
        es = [s for s in S if s.kind == 1 and sorted(s.mv.tolist()) == [a, b]]
        L = np.linalg.norm(P.xm[b] - P.xm[a])
        assert abs(sum(s.w for s in es) / L - 1) < 1e-12
        ref = L * (P.xm[a, 2] + P.xm[b, 2]) / 2
        assert abs(sum(s.w * s.g for s in es) / ref - 1) < 1e-12
        # the master point of every edge sample projects onto its slave point
        for s in es:
            xm_k = s.bm @ P.xm[s.mv]
            xs_k = s.bs @ P.xs[P.ts[s.T]]
            assert np.linalg.norm(np.cross(xm_k - xs_k, s.n)) < 1e-15


def test_edge_weight_vanishes_at_endpoints():
    P = _single_master()
    S = [s for s in mortar.samples(P, features=True) if s.kind == 1]
    for s in S:
        f = mortar.gamma(P, s, delta_e=0.2)
        ref = oracle.hermite(s.eta, 0.2) * oracle.hermite(1 - s.eta, 0.2)
        assert abs(f - ref) < 1e-15
    assert abs(mortar.gamma(P, S[0], delta_e=0.0) - 1.0) == 0.0
    assert oracle.hermite(0.0, 0.2) == 0.0 and oracle.hermite(0.5, 0.2) == 1.0


def test_feature_gradient_against_frozen_energy_differences():
    P = _single_master((3e-4, 5e-4, 4e-4))
    S = mortar.samples(P, features=True)
    ke, kp = 2e2, 1e-2
    A = mortar.assemble(P, S, kappa_edge=ke, kappa_point=kp, delta_e=0.1)
    kap = {2: P.kappa, 1: ke, 0: kp}

    def frozen(xs, xm):
        E = 0.0
        for s in A.active:
            g = s.n @ (s.bm @ xm[s.mv] - s.bs @ xs[P.ts[s.T]])
            E += kap[s.kind] * s.w * mortar.gamma(P, s, 0.1) * oracle.barrier(g, P.dhat)
        return E

    rng = np.random.default_rng(4)
    ds = rng.normal(size=P.xs.shape) * 1e-6
    dm = rng.normal(size=P.xm.shape) * 1e-6
    h = 1e-3
    fd = (frozen(P.xs + h * ds, P.xm + h * dm) - frozen(P.xs - h * ds, P.xm - h * dm)) / (2 * h)
    an = float(np.sum(A.grad[:P.Vs] * ds) + np.sum(A.grad[P.Vs:] * dm))
    assert abs(fd - an) <= 1e-6 * abs(an)
    kinds = {s.kind for s in A.active}
    assert kinds == {0, 1, 2}


def test_reference_gaps_per_slave_triangle_closed_form():
    """Eq. (adaptive_eps) for clipped samples, one reference gap per slave
    triangle: under a punch at uniform gap g0 that covers the pad, the energy
    is sum_T kappa A_T B(g0, eps_T) with eps_T = min(0.9 g_ref[T], dhat) (B = 0
    when g0 >= eps_T), and a triangle whose radius shrinks below the gap
    keeps no active sample."""
    g0 = 3e-4
    w = workloads.flat_punch(gap=g0, n_pad=6, n_punch=5, rule_n=2)
    P = workloads.to_problem(w)
    rng = np.random.default_rng(3)
    g_ref = rng.uniform(0.2e-3, 2e-3, size=P.ts.shape[0])
    eps = np.minimum(0.9 * g_ref, P.dhat)
    assert (eps <= g0).any() and ((eps > g0) & (eps < P.dhat)).any() and (eps == P.dhat).any()
    S = mortar.samples(P, g_ref_tri=g_ref)
    O = mortar.assemble(P, S)
    area = oracle.rest_area(P.xs_rest, P.ts)
    expect = sum(P.kappa * area[T] * oracle.barrier(g0, eps[T]) for T in range(P.ts.shape[0]))
    assert abs(O.energy / expect - 1) <= 1e-10
    active_tris = {s.T for s in O.active}
    assert active_tris == set(np.nonzero(eps > g0)[0].tolist())
    # without reference gaps every triangle has the full radius
    O0 = mortar.assemble(P, mortar.samples(P))
    assert abs(O0.energy / (P.kappa * area.sum() * oracle.barrier(g0, P.dhat)) - 1) <= 1e-10


def test_mortar_linear_step_closed_form():
    """Flat punch at the uniform gap g0, every clipped sample active: a
    closing speed v along the normal (the master moving down, the slave up,
    or both) gives Eq. (ccd)'s bound 0.9 g0 / v for every sample; moving
    apart gives no bound."""
    P, w = _punch_problem(1.4e-2)
    act = mortar.assemble(P, mortar.samples(P)).active
    assert len(act) > 0
    g0 = 3e-4
    zs, zm = np.zeros_like(P.xs), np.zeros_like(P.xm)
    down = zm.copy()
    down[:, 2] = -1e-4
    up = zs.copy()
    up[:, 2] = 5e-5
    assert abs(mortar.linear_step(P, act, zs, down) / (0.9 * g0 / 1e-4) - 1) < 1e-12
    assert abs(mortar.linear_step(P, act, up, zm) / (0.9 * g0 / 5e-5) - 1) < 1e-12
    assert abs(mortar.linear_step(P, act, up, down) / (0.9 * g0 / 1.5e-4) - 1) < 1e-12
    assert mortar.linear_step(P, act, -up, -down) == np.inf
