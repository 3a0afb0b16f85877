"""Pins of the dual-mesh mapper oracle (Sec. 3, Eqs. (bary_proj), (decomp),
(gram), (bary_interp)) against facts the geometry fixes: dense sampling of
triangles, exact reconstruction at rest, rigid invariance, and the O(h^2)
interpolation error the paper states."""
import numpy as np
import pytest

from gen import meshes
from oracle import dualmesh as dm


def _dense(A, B, C, m=120):
    """Points of a barycentric lattice on one triangle."""
    i, j = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
    keep = i + j <= m
    v, w = i[keep] / m, j[keep] / m
    return A + v[:, None] * (B - A) + w[:, None] * (C - A)


def test_closest_point_against_dense_sampling():
    rng = np.random.default_rng(0)
    for _ in range(60):
        A, B, C = rng.normal(size=(3, 3))
        p = rng.normal(size=3) * 2
        q = dm.closest_points(p, A[None], B[None], C[None])[0]
        S = _dense(A, B, C)
        ds = np.sqrt(((S - p) ** 2).sum(1)).min()
        dq = np.linalg.norm(p - q)
        h = max(np.linalg.norm(B - A), np.linalg.norm(C - A), np.linalg.norm(C - B)) / 120
        assert dq <= ds + 1e-12                      # nothing on the triangle is closer
        assert dq >= ds - h                          # and the lattice gets within a cell of it
        # the returned point lies on the triangle
        u, v, w, off = dm.embed_on(q, np.stack([A, B, C]), np.array([[0, 1, 2]]), 0)
        assert min(u, v, w) >= -1e-9 and abs(off) < 1e-9


def test_nearest_triangle_against_dense_sampling():
    rng = np.random.default_rng(1)
    V, F = meshes.icosphere(1, 1.0)
    V = V * (1 + 0.1 * rng.uniform(-1, 1, size=(V.shape[0], 1)))
    for _ in range(25):
        p = rng.normal(size=3) * 1.3
        t, d2 = dm.nearest_triangle(p, V, F)
        dens = [np.sqrt(((_dense(*V[f], m=40) - p) ** 2).sum(1)).min() for f in F]
        assert np.sqrt(d2) <= min(dens) + 1e-12
        # the sampled argmin is the same triangle unless two are within a lattice cell
        order = np.argsort(dens)
        if dens[order[1]] - dens[order[0]] > 0.05:
            assert t == order[0]


def _mesh_pair(freq_sim, freq_vis=24, rng=None):
    Vs, Fs = meshes.geodesic_sphere(freq_sim, 1.0)
    P, _ = meshes.geodesic_sphere(freq_vis, 1.0)
    if rng is not None:
        P = P * (1 + 0.02 * rng.uniform(-1, 1, size=(P.shape[0], 1)))
    return Vs, Fs, P


def test_reconstruction_at_rest_and_decomposition():
    rng = np.random.default_rng(2)
    Vs, Fs, P = _mesh_pair(4, 10, rng)
    T, B, D, _ = dm.embed(P, Vs, Fs)
    assert np.allclose(B.sum(1), 1.0, atol=1e-14)
    assert np.abs(dm.update(Vs, Fs, T, B, D) - P).max() < 1e-13
    # the offset is the signed distance to the plane of the assigned triangle
    for i in range(0, P.shape[0], 37):
        v0, e1, e2, n = dm.frame(Vs, Fs, T[i])
        assert abs((P[i] - v0) @ n - D[i]) < 1e-14


def test_rigid_invariance():
    rng = np.random.default_rng(3)
    Vs, Fs, P = _mesh_pair(4, 10, rng)
    T, B, D, _ = dm.embed(P, Vs, Fs)
    R = meshes.random_rotation(rng)
    tr = rng.normal(size=3)
    out = dm.update(Vs @ R.T + tr, Fs, T, B, D)
    assert np.abs(out - (P @ R.T + tr)).max() < 1e-12


def _phi(x):
    """A smooth non-affine deformation."""
    return x + 0.15 * np.stack([np.sin(2 * x[:, 1]), np.cos(1.5 * x[:, 2]) * x[:, 0], 0.5 * x[:, 0] * x[:, 1]], 1)


def test_error_is_second_order_in_h():
    """Sphere visual mesh on coarser geodesic simulation meshes: the
    error of the mapped positions against the deformation applied to the
    visual vertices falls by ~4x per halving of h."""
    errs = []
    for f in (4, 8, 16):
        Vs, Fs, P = _mesh_pair(f, 24)
        T, B, D, _ = dm.embed(P, Vs, Fs)
        errs.append(np.abs(dm.update(_phi(Vs), Fs, T, B, D) - _phi(P)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs


@pytest.mark.parametrize("seed", [4])
def test_tie_rule_smaller_index(seed):
    """A point equidistant from two triangles sharing an edge maps to the
    smaller index."""
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float)
    F = np.array([[1, 3, 2], [0, 1, 2]])
    p = np.array([0.5, 0.5, 0.3])                     # above the shared edge's midpoint
    t, d2 = dm.nearest_triangle(p, V, F)
    assert t == 0 and abs(d2 - 0.09) < 1e-15


def test_zero_area_triangle_never_chosen():
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.2, 0.2, 0.0], [0.3, 0.3, 0.0]], float)
    F = np.array([[3, 4, 3], [0, 1, 2]])
    t, d2 = dm.nearest_triangle(np.array([0.25, 0.25, 0.01]), V, F)
    assert t == 1 and abs(d2 - 1e-4) < 1e-15
