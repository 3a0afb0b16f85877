"""Pins of the oracle's step bound (linearised gap, Eq. (ccd)/(global_ccd),
and additive CCD over swept pairs).

* point-plane linear motion: alpha = 0.9 g0 / v_n exactly, for both the
  linearised bound and ACCD (s = 0.1);
* a flat punch pushed down by D: alpha = 0.9 g0 / D over every sample;
* a common rigid translation of both surfaces gives alpha = 1;
* point-triangle distance against dense barycentric sampling;
* ACCD never exceeds the exact time of impact, computed independently from
  the coplanarity cubic and an inside test, and stops short of contact;
* grid and brute-force swept-pair enumeration agree.
"""
import numpy as np
import pytest

import oracle
from gen import workloads


def _point_plane(g0=2e-4, v=5e-4):
    # one slave triangle (centroid sample), a big master triangle above it
    xs = np.array([[0.0, 0.0, 0.0], [1e-3, 0.0, 0.0], [0.0, 1e-3, 0.0]])
    ts = np.array([[0, 1, 2]])
    L = 1e-1
    xm = np.array([[-L, -L, g0], [-L, 3 * L, g0], [3 * L, -L, g0]])
    tm = np.array([[0, 1, 2]])   # normal -z (faces the pad)
    P = oracle.Problem(xs, ts, xm, tm, rule_n=1)
    dxs = np.tile([0.0, 0.0, v], (3, 1))
    return P, dxs, np.zeros((3, 3))


def test_point_plane_linear_and_accd_exact():
    g0, v = 2e-4, 5e-4
    P, dxs, dxm = _point_plane(g0, v)
    nr = oracle.narrow(P)
    assert nr.M[0] == 0 and abs(nr.g[0] - g0) < 1e-18
    expect = 0.9 * g0 / v
    assert abs(oracle.step_linear(P, nr.M, dxs, dxm) / expect - 1) < 1e-14
    p = P.xs.mean(axis=0)
    a = oracle.accd(p, [0, 0, v], *[x for m in P.xm for x in (m, np.zeros(3))])
    assert abs(a / expect - 1) < 1e-12
    sb = oracle.ccd_step(P, nr.M, dxs, dxm)
    assert abs(sb.alpha / expect - 1) < 1e-12 and sb.n_swept == 1


def test_flat_punch_pushed_down():
    g0, D = 3e-4, 1e-3
    w = workloads.flat_punch(gap=g0, n_pad=6, n_punch=4)
    P = workloads.to_problem(w)
    nr = oracle.narrow(P)
    dxs = np.zeros_like(P.xs)
    dxm = np.tile([0.0, 0.0, -D], (P.Vm, 1))
    expect = 0.9 * g0 / D
    sb = oracle.ccd_step(P, nr.M, dxs, dxm)
    assert abs(sb.alpha_lin / expect - 1) < 1e-13
    assert abs(sb.alpha_accd / expect - 1) < 1e-12
    assert abs(sb.alpha / expect - 1) < 1e-12
    assert sb.n_swept >= P.Ns


def test_common_translation_gives_one(small):
    P = workloads.to_problem(small)
    nr = oracle.narrow(P)
    d = np.array([1e-4, -2e-4, 3e-4])
    sb = oracle.ccd_step(P, nr.M, np.tile(d, (P.Vs, 1)), np.tile(d, (P.Vm, 1)))
    # the linearised gap rate is zero up to rounding: no finite bound below 1
    assert sb.alpha == 1.0 and sb.alpha_lin > 1e6


def test_point_triangle_distance_dense_sampling():
    rng = np.random.default_rng(8)
    s = np.linspace(0, 1, 401)
    uu, vv = np.meshgrid(s, s)
    keep = uu + vv <= 1
    uu, vv = uu[keep], vv[keep]
    for _ in range(40):
        a, b, c = rng.normal(size=(3, 3))
        p = rng.normal(size=3) * 1.5
        pts = a + uu[:, None] * (b - a) + vv[:, None] * (c - a)
        dmin = np.sqrt(((pts - p) ** 2).sum(1).min())
        d = np.sqrt(oracle.point_tri_dist2(p, a, b, c))
        edge = max(np.linalg.norm(b - a), np.linalg.norm(c - a), np.linalg.norm(c - b))
        assert d <= dmin + 1e-12
        assert dmin - d <= 2.5e-3 * edge


def _exact_toi(p, dp, a, da, b, db, c, dc):
    """Earliest t in [0,1] where the moving point lies in the moving triangle
    (coplanarity cubic + inside test), or None."""
    def f(t):
        A, B, Cc, Pp = a + t * da, b + t * db, c + t * dc, p + t * dp
        return np.linalg.det(np.stack([B - A, Cc - A, Pp - A]))
    ts = np.array([0.0, 1 / 3, 2 / 3, 1.0])
    coef = np.polyfit(ts, [f(t) for t in ts], 3)
    roots = np.roots(coef)
    cands = sorted(r.real for r in roots if abs(r.imag) < 1e-9 and -1e-12 <= r.real <= 1 + 1e-12)
    for t in cands:
        A, B, Cc, Pp = a + t * da, b + t * db, c + t * dc, p + t * dp
        F = np.stack([B - A, Cc - A], 1)
        uv = np.linalg.lstsq(F, Pp - A, rcond=None)[0]
        if uv.min() >= -1e-9 and uv.sum() <= 1 + 1e-9:
            return t
    return None


def test_accd_conservative_against_exact_toi():
    rng = np.random.default_rng(9)
    hits = 0
    for it in range(300):
        a, b, c = rng.normal(size=(3, 3))
        n = np.cross(b - a, c - a)
        n /= np.linalg.norm(n)
        cen = (a + b + c) / 3
        p = cen + n * rng.uniform(0.05, 0.5) + rng.normal(size=3) * 0.3
        dp = -n * rng.uniform(0.2, 1.5) + rng.normal(size=3) * 0.3
        da, db, dc = rng.normal(size=(3, 3)) * 0.1
        toi = _exact_toi(p, dp, a, da, b, db, c, dc)
        al = oracle.accd(p, dp, a, da, b, db, c, dc, 0.1, 1.0)
        assert 0.0 < al <= 1.0
        if toi is not None:
            hits += 1
            assert al <= toi
            # ACCD stops short of contact, at a separation of order s d0
            A, B, Cc, Pp = a + al * da, b + al * db, c + al * dc, p + al * dp
            assert oracle.point_tri_dist2(Pp, A, B, Cc) > 0.0
            assert al >= 0.5 * toi * 0.9 or toi < 1e-3
    assert hits > 50


def test_swept_pairs_grid_equals_brute(small):
    P = workloads.to_problem(small)
    nr = oracle.narrow(P)
    a = oracle.ccd_step(P, nr.M, small.dxs, small.dxm, use_grid=True)
    b = oracle.ccd_step(P, nr.M, small.dxs, small.dxm, use_grid=False)
    assert a.n_swept == b.n_swept and a.alpha == b.alpha and a.alpha_accd == b.alpha_accd
    assert 0 < a.alpha < 1


def test_swept_count_brute_force_tiny():
    """The swept-pair count is the number of (sample point, master triangle)
    pairs whose boxes over t in [0, 1] overlap: brute force over boxes built
    here from the vertex paths, on a small random scene with motion of both
    surfaces; the count equals the step bound's n_swept, and a positive box
    margin can only add pairs."""
    rng = np.random.default_rng(17)
    from gen import meshes
    xs, ts = meshes.pad(4, 2e-3)
    xm = rng.uniform(-1.2e-3, 1.2e-3, size=(12, 3))
    xm[:, 2] = rng.uniform(1e-4, 6e-4, size=12)
    tm = rng.integers(0, 12, size=(10, 3))
    tm = tm[(tm[:, 0] != tm[:, 1]) & (tm[:, 1] != tm[:, 2]) & (tm[:, 0] != tm[:, 2])]
    dxs = rng.uniform(-2e-4, 2e-4, size=xs.shape)
    dxm = rng.uniform(-2e-4, 2e-4, size=xm.shape)
    P = oracle.Problem(xs, ts, xm, tm, rule_n=2)
    # sample points and their paths from the rule written out here
    pts = []
    for T in range(ts.shape[0]):
        for q in range(P.nq):
            xi, eta = P.rule[q, 0], P.rule[q, 1]
            b = np.array([1 - xi - eta, xi, eta])
            p0 = b @ xs[ts[T]]
            p1 = p0 + b @ dxs[ts[T]]
            pts.append((np.minimum(p0, p1), np.maximum(p0, p1)))
    brute = 0
    for t in range(tm.shape[0]):
        ends = np.concatenate([xm[tm[t]], xm[tm[t]] + dxm[tm[t]]])
        lo, hi = ends.min(axis=0), ends.max(axis=0)
        for plo, phi in pts:
            brute += bool(np.all(plo <= hi) and np.all(lo <= phi))
    assert brute > 5
    assert oracle.swept_count(P, dxs, dxm) == brute
    assert oracle.swept_count(P, dxs, dxm, use_grid=False) == brute
    nr = oracle.narrow(P)
    assert oracle.ccd_step(P, nr.M, dxs, dxm).n_swept == brute
    assert oracle.swept_count(P, dxs, dxm, pad_rel=1e-3, pad_abs=1e-5) >= brute
    assert oracle.swept_count(P, dxs, dxm, pad_abs=1.0) == len(pts) * tm.shape[0]


@pytest.mark.parametrize("seed", [3, 5, 8])
def test_swept_count_brute_force_deforming(seed):
    """Exact swept-pair counts on denser scenes whose vertices move
    independently (each sample path depends on all three of its triangle's
    vertex motions), with and without an absolute box margin: a margin d on
    both boxes makes them overlap when every axis gap is at most 2 d."""
    rng = np.random.default_rng(seed)
    from gen import meshes
    xs, ts = meshes.pad(6, 2e-3)
    xm = rng.uniform(-1.2e-3, 1.2e-3, size=(30, 3))
    xm[:, 2] = rng.uniform(5e-5, 4e-4, size=30)
    tm = rng.integers(0, 30, size=(40, 3))
    tm = tm[(tm[:, 0] != tm[:, 1]) & (tm[:, 1] != tm[:, 2]) & (tm[:, 0] != tm[:, 2])]
    dxs = rng.uniform(-3e-4, 3e-4, size=xs.shape)
    dxm = rng.uniform(-3e-4, 3e-4, size=xm.shape)
    P = oracle.Problem(xs, ts, xm, tm, rule_n=3)
    boxes = []
    for T in range(ts.shape[0]):
        for q in range(P.nq):
            xi, eta = P.rule[q, 0], P.rule[q, 1]
            b = np.array([1 - xi - eta, xi, eta])
            p0 = b @ xs[ts[T]]
            p1 = p0 + b @ dxs[ts[T]]
            boxes.append((np.minimum(p0, p1), np.maximum(p0, p1)))
    tri = [(np.concatenate([xm[t], xm[t] + dxm[t]]).min(axis=0), np.concatenate([xm[t], xm[t] + dxm[t]]).max(axis=0))
           for t in tm]
    for pad in (0.0, 2e-5):
        brute = sum(bool(np.all(plo - pad <= hi + pad) and np.all(lo - pad <= phi + pad))
                    for lo, hi in tri for plo, phi in boxes)
        assert brute > 50
        assert oracle.swept_count(P, dxs, dxm, pad_abs=pad) == brute
        assert oracle.swept_count(P, dxs, dxm, pad_abs=pad, use_grid=False) == brute
