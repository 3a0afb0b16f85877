"""Seeded synthetic surface meshes for the tactile-contact workloads.

Pure geometry (numpy, float64): grids, spheres, an extruded glyph and rigid
poses.  Nothing here evaluates the contact method itself; both the FP64 oracle
and the HIP path consume these arrays.

Conventions
-----------
* SI units (metres).
* Triangles are CCW around their outward normal.  The tactile pad's outward
  normal is +z (it faces the indenter); indenter normals point out of the body.
"""
from __future__ import annotations

import numpy as np


def pad(n: int, length: float = 1e-2, noise: float = 0.0, rng=None):
    """n x n quad grid over [-L/2, L/2]^2 at z = 0, each quad split in two.

    Quad (i, j) with corners v00, v10, v11, v01 becomes (v00, v10, v11) and
    (v00, v11, v01), both CCW seen from +z.  ``noise`` adds a per-vertex z
    offset drawn uniformly from [-noise, noise].
    Returns (x[(n+1)^2, 3] float64, tri[2 n^2, 3] int32).
    """
    t = np.linspace(-length / 2, length / 2, n + 1)
    xx, yy = np.meshgrid(t, t, indexing="xy")          # row = y index
    x = np.stack([xx.ravel(), yy.ravel(), np.zeros(xx.size)], axis=1)
    if noise > 0.0:
        rng = np.random.default_rng(0) if rng is None else rng
        x[:, 2] = rng.uniform(-noise, noise, size=x.shape[0])
    vid = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)   # [iy, ix]
    v00 = vid[:-1, :-1].ravel()
    v10 = vid[:-1, 1:].ravel()
    v11 = vid[1:, 1:].ravel()
    v01 = vid[1:, :-1].ravel()
    tri = np.empty((2 * n * n, 3), dtype=np.int32)
    tri[0::2] = np.stack([v00, v10, v11], axis=1)
    tri[1::2] = np.stack([v00, v11, v01], axis=1)
    return x, tri


def _icosahedron():
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]],
                 dtype=np.int64)
    return v, f


def _weld(points: np.ndarray, tri: np.ndarray, tol: float):
    """Merge coincident vertices (within ``tol``) and reindex triangles."""
    key = np.round(points / tol).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.ravel()
    order = np.argsort(first)              # keep first-seen order for stability
    remap = np.empty_like(order)
    remap[order] = np.arange(order.size)
    new_points = points[first[order]]
    return new_points, remap[inv][tri].astype(np.int32)


def geodesic_sphere(freq: int, radius: float = 1.0):
    """Class-I geodesic sphere: every icosahedron face split into freq^2
    triangles, vertices pushed to the sphere.  20 f^2 triangles, 10 f^2 + 2
    vertices, outward CCW.  freq = 2^s gives the subdivision-s icosphere."""
    v, f = _icosahedron()
    pts = []
    tris = []
    base = 0
    for a, b, c in f:
        A, B, C = v[a], v[b], v[c]
        idx = {}
        local = []
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                k = freq - i - j
                idx[(i, j)] = len(local)
                local.append((k * A + i * B + j * C) / freq)
        for i in range(freq):
            for j in range(freq - i):
                tris.append((base + idx[(i, j)], base + idx[(i + 1, j)], base + idx[(i, j + 1)]))
                if i + j < freq - 1:
                    tris.append((base + idx[(i + 1, j)], base + idx[(i + 1, j + 1)],
                                 base + idx[(i, j + 1)]))
        pts.extend(local)
        base += len(local)
    pts = np.asarray(pts)
    tri = np.asarray(tris, dtype=np.int64)
    pts, tri = _weld(pts, tri, 1e-9)
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    # orient outward: flip faces whose normal points inward
    e1 = pts[tri[:, 1]] - pts[tri[:, 0]]
    e2 = pts[tri[:, 2]] - pts[tri[:, 0]]
    nrm = np.cross(e1, e2)
    inward = np.einsum("ij,ij->i", nrm, pts[tri].mean(axis=1)) < 0
    tri[inward] = tri[inward][:, [0, 2, 1]]
    return pts * radius, tri.astype(np.int32)


def icosphere(subdiv: int, radius: float = 1.0):
    """Icosphere at subdivision level ``subdiv`` (10*4^s + 2 vertices)."""
    return geodesic_sphere(2 ** subdiv, radius)


# 5 x 7 glyph of the capital letter "G", row 0 at the top.
_GLYPH_G = [
    ".###.",
    "#...#",
    "#....",
    "#.###",
    "#...#",
    "#...#",
    ".###.",
]


def _quad_grid(p0, du, dv, k):
    """k x k refined quad p0 + s du + t dv, CCW around du x dv."""
    s = np.linspace(0.0, 1.0, k + 1)
    ss, tt = np.meshgrid(s, s, indexing="ij")
    pts = p0[None, :] + ss.reshape(-1, 1) * du[None, :] + tt.reshape(-1, 1) * dv[None, :]
    vid = np.arange((k + 1) * (k + 1)).reshape(k + 1, k + 1)
    a = vid[:-1, :-1].ravel()
    b = vid[1:, :-1].ravel()
    c = vid[1:, 1:].ravel()
    d = vid[:-1, 1:].ravel()
    tri = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    return pts, tri


def letter(cell: float = 1e-3, depth: float = 4e-3, refine: int = 10, glyph=None):
    """Extruded block letter built from a 5x7 cell glyph.

    The glyph lies in the xy-plane, extruded over z in [0, depth]; the cap at
    z = 0 faces -z.  Every unit face (cap cell or wall cell) is refined into
    ``refine`` x ``refine`` quads.  Returns (x, tri) centred in xy, outward CCW.
    """
    g = _GLYPH_G if glyph is None else glyph
    rows = len(g)
    cols = len(g[0])
    filled = np.array([[ch == "#" for ch in r] for r in g], dtype=bool)[::-1]  # row 0 = bottom (y)
    nz = max(1, int(round(depth / cell)))
    dz = depth / nz
    pts_all, tri_all, base = [], [], 0

    def add(p0, du, dv):
        nonlocal base
        p, t = _quad_grid(np.asarray(p0, float), np.asarray(du, float), np.asarray(dv, float), refine)
        pts_all.append(p)
        tri_all.append(t + base)
        base += p.shape[0]

    X = np.array([cell, 0, 0.0])
    Y = np.array([0, cell, 0.0])
    Z = np.array([0, 0, dz])
    for r in range(rows):
        for c in range(cols):
            if not filled[r, c]:
                continue
            o = np.array([c * cell, r * cell, 0.0])
            add(o, Y, X)                                  # bottom cap, normal -z
            add(o + np.array([0, 0, depth]), X, Y)        # top cap, normal +z
            for kz in range(nz):
                oz = o + kz * Z
                if c == 0 or not filled[r, c - 1]:
                    add(oz, Z, Y)                         # -x wall
                if c == cols - 1 or not filled[r, c + 1]:
                    add(oz + X, Y, Z)                     # +x wall
                if r == 0 or not filled[r - 1, c]:
                    add(oz, X, Z)                         # -y wall
                if r == rows - 1 or not filled[r + 1, c]:
                    add(oz + Y, Z, X)                     # +y wall
    pts = np.concatenate(pts_all)
    tri = np.concatenate(tri_all)
    pts, tri = _weld(pts, tri, cell * 1e-6)
    pts[:, 0] -= cols * cell / 2
    pts[:, 1] -= rows * cell / 2
    return pts, tri


def tet_block(nx: int, ny: int, nz: int, h: float):
    """Box of nx x ny x nz cubes of edge h over [0, nx h] x [0, ny h] x [0, nz h],
    each cube split into 6 tetrahedra along its main diagonal (Kuhn split),
    consistently positively oriented.  Returns (x [V, 3], tets [6 n, 4],
    top [2 nx ny, 3] boundary triangles of the face z = nz h, CCW from +z,
    bottom vertex ids on z = 0)."""
    gx, gy, gz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    x = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], 1).astype(np.float64) * h
    vid = lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    c = [vid(i + (b & 1), j + ((b >> 1) & 1), k + ((b >> 2) & 1)) for b in range(8)]  # corner b = (dx, dy, dz)
    # the six monotone paths from corner 0 to corner 7
    paths = [(1, 3), (1, 5), (2, 3), (2, 6), (4, 5), (4, 6)]
    tets = []
    for a, b in paths:
        tets.append(np.stack([c[0], c[a], c[b], c[7]], 1))
    tets = np.concatenate(tets).astype(np.int64)
    p = x[tets]
    vol = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    flip = vol < 0
    tets[flip] = tets[flip][:, [0, 2, 1, 3]]
    ti, tj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ti, tj = ti.ravel(), tj.ravel()
    v00, v10 = vid(ti, tj, nz), vid(ti + 1, tj, nz)
    v11, v01 = vid(ti + 1, tj + 1, nz), vid(ti, tj + 1, nz)
    top = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)])
    bottom = np.nonzero(x[:, 2] == 0.0)[0]
    return x, tets.astype(np.int32), top.astype(np.int32), bottom.astype(np.int32)


def tet_block_bottom(nx: int, ny: int, nz: int) -> np.ndarray:
    """Boundary triangles of the face z = 0 of ``tet_block(nx, ny, nz, h)``,
    CCW seen from -z (outward), with the same diagonal as the tetrahedra's
    faces there."""
    vid = lambda i, j: (i * (ny + 1) + j) * (nz + 1)
    ti, tj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ti, tj = ti.ravel(), tj.ravel()
    v00, v10 = vid(ti, tj), vid(ti + 1, tj)
    v11, v01 = vid(ti + 1, tj + 1), vid(ti, tj + 1)
    return np.concatenate([np.stack([v00, v11, v10], 1), np.stack([v00, v01, v11], 1)]).astype(np.int32)


def random_rotation(rng) -> np.ndarray:
    """Uniformly distributed rotation matrix (from a normalised quaternion)."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def axis_angle(axis, angle: float) -> np.ndarray:
    """Rotation matrix about unit ``axis`` by ``angle`` (Rodrigues)."""
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)


def perturb_radial(x: np.ndarray, center, rng, n_bumps: int = 3, amp: float = 0.02,
                   width: float = 0.6) -> np.ndarray:
    """Low-frequency radial perturbation: a few Gaussian bumps of relative
    amplitude up to ``amp`` on a sphere-like mesh around ``center``."""
    c = np.asarray(center, float)
    d = x - c
    r = np.linalg.norm(d, axis=1, keepdims=True)
    u = d / r
    scale = np.ones((x.shape[0], 1))
    for _ in range(n_bumps):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        s = rng.uniform(-amp, amp)
        scale[:, 0] += s * np.exp(-((1.0 - u @ axis) / (width * width)))
    return c + u * r * scale


def ball_uniform(rng, n: int, radius: float) -> np.ndarray:
    """n points uniform in a ball: normalised Gaussian direction, radius R U^(1/3)."""
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * (radius * rng.uniform(size=(n, 1)) ** (1.0 / 3.0))


def place_above(x_master: np.ndarray, x_slave: np.ndarray, gap: float) -> np.ndarray:
    """Translate the master along z so its lowest vertex sits ``gap`` above the
    highest slave vertex.  Every master surface point is then at least ``gap``
    above every slave surface point, so no placement can start interpenetrated."""
    dz = x_slave[:, 2].max() + gap - x_master[:, 2].min()
    out = x_master.copy()
    out[:, 2] += dz
    return out
