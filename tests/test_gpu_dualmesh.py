"""Dual-mesh mapper on the GPU (include/gmcp_dualmesh.h) against the FP64
oracle (Sec. 3, Eqs. (bary_proj), (decomp), (gram), (bary_interp)).

The nearest triangle is unique except at exact ties (a visual vertex whose
nearest point lies on an edge shared by two triangles): there the distance
is compared, and the GPU's triangle must be one of the nearest; the
barycentric coordinates and offset are compared with the oracle evaluated
on the GPU's triangle.  Tolerances: distances and mapping 1e-12 relative to
the mesh size (both sides FP64); the float32 update 2e-6 of the mesh size.
"""
import numpy as np
import pytest

from gen import meshes, workloads
from gpu_helpers import need_gpu
from oracle import dualmesh as odm

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _check_mapping(dmap, P, V, F, idx, scale):
    tri = dmap.tri.cpu().numpy()
    d2 = dmap.dist2.cpu().numpy()
    bary = dmap.bary64.cpu().numpy()
    delta = dmap.delta64.cpu().numpy()
    for i in idx:
        t, od2 = odm.nearest_triangle(P[i], V, F)
        assert abs(np.sqrt(d2[i]) - np.sqrt(od2)) <= 1e-12 * scale, i
        if tri[i] != t:   # a tie: the GPU's triangle must be as near
            q = odm.closest_points(P[i], *(V[F[tri[i]]][:, None, :]))[0]
            assert abs(np.linalg.norm(P[i] - q) - np.sqrt(od2)) <= 1e-12 * scale, (i, t, tri[i])
        u, v, w, dl = odm.embed_on(P[i], V, F, tri[i])
        assert np.abs(bary[i] - (u, v, w)).max() <= 1e-9, i
        assert abs(delta[i] - dl) <= 1e-12 * scale, i


@pytest.mark.parametrize("n_vis,n_sim", [(10, 4), (7, 5)])
def test_small_mapping_and_update_match_oracle(n_vis, n_sim):
    """Every vertex checked; ragged sizes (N and nT not multiples of the
    256-wide tiles)."""
    need_gpu()
    from paper_2605_24339_amd.dualmesh import DualMesh
    rng = np.random.default_rng(n_vis * 10 + n_sim)
    V, F = meshes.geodesic_sphere(n_sim, 1.0)
    V = V * (1 + 0.05 * rng.uniform(-1, 1, size=(V.shape[0], 1)))
    P, _ = meshes.geodesic_sphere(n_vis, 1.0)
    P = (P @ meshes.random_rotation(rng).T) * (1 + 0.03 * rng.uniform(-1, 1, size=(P.shape[0], 1)))
    for dtype in (torch.float64, torch.float32):
        dmap = DualMesh(P, V, F, dtype=dtype)
        _check_mapping(dmap, P, V, F, range(P.shape[0]), 1.0)
        T, B, D = dmap.tri.cpu().numpy(), dmap.bary64.cpu().numpy(), dmap.delta64.cpu().numpy()
        Vd = workloads.smooth_deformation(V, amp=0.1, scale=1.0)
        ref = odm.update(Vd, F, T, B, D)
        out = dmap.update(torch.tensor(Vd, dtype=dtype, device="cuda")).double().cpu().numpy()
        tol = 1e-12 if dtype == torch.float64 else 2e-6
        assert np.abs(out - ref).max() <= tol, dtype
        # at rest the mapping reproduces the visual vertices
        rest = dmap.update(torch.tensor(V, dtype=dtype, device="cuda")).double().cpu().numpy()
        assert np.abs(rest - P).max() <= tol


def test_rigid_invariance_on_gpu():
    need_gpu()
    from paper_2605_24339_amd.dualmesh import DualMesh
    rng = np.random.default_rng(11)
    P, V, F = workloads.dual_mesh(seed=11, sim_freq=8, vis_freq=24, radius=1.0)
    dmap = DualMesh(P, V, F, dtype=torch.float64)
    R = meshes.random_rotation(rng)
    tr = rng.normal(size=3)
    out = dmap.update(torch.tensor(V @ R.T + tr, device="cuda")).cpu().numpy()
    assert np.abs(out - (P @ R.T + tr)).max() < 1e-12


def test_full_size_sampled():
    """655362 visual vertices on a 20480-triangle surface: 400 sampled
    vertices checked one by one against the oracle; the float32 update of
    every vertex against the oracle's formula on the GPU's mapping."""
    need_gpu()
    from paper_2605_24339_amd.dualmesh import DualMesh
    P, V, F = workloads.dual_mesh()
    R = 5e-3
    dmap = DualMesh(P, V, F, dtype=torch.float32)
    rng = np.random.default_rng(0)
    idx = np.concatenate([[0, P.shape[0] - 1], rng.choice(P.shape[0], 398, replace=False)])
    _check_mapping(dmap, P, V, F, idx, R)
    Vd = workloads.smooth_deformation(V)
    out = dmap.update(torch.tensor(Vd, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    T, B, D = dmap.tri.cpu().numpy(), dmap.bary64.cpu().numpy(), dmap.delta64.cpu().numpy()
    # the oracle's update, vectorised over all vertices (same formula)
    a, b, c = Vd[F[T, 0]], Vd[F[T, 1]], Vd[F[T, 2]]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    ref = B[:, :1] * a + B[:, 1:2] * b + B[:, 2:] * c + D[:, None] * n
    assert np.abs(out[idx] - odm.update(Vd, F, T[idx], B[idx], D[idx])).max() <= 2e-6 * R
    assert np.abs(out - ref).max() <= 2e-6 * R


def test_edge_cases():
    need_gpu()
    import ctypes as C

    from paper_2605_24339_amd import _native as N
    from paper_2605_24339_amd.dualmesh import DualMesh, _lib
    # empty visual mesh
    V, F = meshes.icosphere(1, 1.0)
    d = DualMesh(np.zeros((0, 3)), V, F)
    assert d.update(torch.tensor(V, dtype=torch.float32, device="cuda")).shape == (0, 3)
    # no triangles for a non-empty visual mesh
    z = torch.zeros(3, dtype=torch.float64, device="cuda")
    rc = _lib().gmcp_dualmesh_embed(C.c_void_p(z.data_ptr()), 1, C.c_void_p(z.data_ptr()), None, 0, None, None,
                                    None, None, None)
    assert rc == N.GMCP_E_ARG
    # a zero-area triangle is never chosen
    Vz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.2, 0.2, 0.0], [0.3, 0.3, 0.0]], float)
    Fz = np.array([[3, 4, 3], [0, 1, 2]])
    d = DualMesh(np.array([[0.25, 0.25, 0.01]]), Vz, Fz, dtype=torch.float64)
    assert int(d.tri[0]) == 1
