"""Seeded synthetic tactile-indentation workloads.

Each builder returns a :class:`Workload`: a slave (tactile pad) surface, a
master (indenter) surface, the contact parameters, and a per-vertex search
direction for the step bound.  Positions are generated in float64; with
``fp32=True`` they are rounded to float32 (and kept as float64 arrays), so
the FP64 oracle and the float32 GPU path see the very same coordinates.

Only geometry and random numbers live here; no part of the contact method.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import meshes


@dataclass
class Workload:
    name: str
    xs: np.ndarray           # slave positions [Vs, 3]
    ts: np.ndarray           # slave triangles [Ts, 3] int32
    xm: np.ndarray           # master positions [Vm, 3]
    tm: np.ndarray           # master triangles [Tm, 3] int32
    rule_n: int              # n x n samples per slave triangle
    kappa: float
    dhat: float
    delta_T: float
    dxs: np.ndarray          # search direction, slave [Vs, 3]
    dxm: np.ndarray          # search direction, master [Vm, 3]
    xs_rest: np.ndarray = field(default=None)
    info: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.xs_rest is None:
            self.xs_rest = self.xs

    @property
    def n_samples(self):
        return self.ts.shape[0] * self.rule_n * self.rule_n


def _r32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def _finish(w: Workload, fp32: bool) -> Workload:
    if fp32:
        for k in ("xs", "xm", "dxs", "dxm", "xs_rest"):
            setattr(w, k, _r32(getattr(w, k)))
    return w


def small_indent(seed: int = 1, fp32: bool = True, delta_T: float = 0.0) -> Workload:
    """Plain GMCP case: 16x16 flat pad (512 tris, 10x10 mm), 2x2 samples per
    triangle (2048), icosphere subdivision 3 (642 V / 1280 T, R = 5 mm) with a
    random rotation and a +-0.5 mm lateral offset, lowest vertex 10 um above
    the pad, so sample gaps spread over [10 um, dhat].  dhat = 1 mm,
    kappa = 1e5.  Search direction: every vertex of both meshes moves by a
    vector uniform in a 0.5 mm ball (seed 11)."""
    rng = np.random.default_rng(seed)
    xs, ts = meshes.pad(16, 1e-2)
    xm, tm = meshes.icosphere(3, 5e-3)
    xm = xm @ meshes.random_rotation(rng).T
    off = rng.uniform(-0.5e-3, 0.5e-3, size=2)
    xm[:, 0] += off[0]
    xm[:, 1] += off[1]
    xm = meshes.place_above(xm, xs, 10e-6)
    r2 = np.random.default_rng(11)
    dxs = meshes.ball_uniform(r2, xs.shape[0], 0.5e-3)
    dxm = meshes.ball_uniform(r2, xm.shape[0], 0.5e-3)
    w = Workload("small_indent_16x16_ico3", xs, ts, xm, tm, 2, 1e5, 1e-3, delta_T, dxs, dxm)
    return _finish(w, fp32)


def large_indent(seed: int = 2, fp32: bool = True, indenter: str = "sphere",
                 g_min: float = 10e-6, pad_n: int = 128, rule_n: int = 4) -> Workload:
    """Single large indentation: 128x128 gel pad (32768 tris, 10x10 mm) with
    +-50 um vertex z-noise, 4x4 = 16 samples per triangle (524288 samples),
    pressed by a ~40k-triangle indenter placed g_min above the pad:
      sphere: geodesic sphere, frequency 45 (40500 T), R = 5 mm, three radial
              bumps of up to 2 % R and +-10 um vertex noise;
      letter: extruded 5x7-cell block letter, 4 mm deep, tilted <= 2 deg.
    Search direction: indenter rigid motion of 0.2 mm down plus a 0.2 deg
    rotation about a random horizontal axis; pad vertices uniform in a
    20 um ball."""
    rng = np.random.default_rng(seed)
    xs, ts = meshes.pad(pad_n, 1e-2, noise=50e-6, rng=rng)
    if indenter == "sphere":
        xm, tm = meshes.geodesic_sphere(45, 5e-3)
        xm = meshes.perturb_radial(xm, np.zeros(3), rng, n_bumps=3, amp=0.02)
        xm = xm + rng.uniform(-10e-6, 10e-6, size=xm.shape)
        center = np.zeros(3)
    elif indenter == "letter":
        xm, tm = meshes.letter(cell=1e-3, depth=4e-3, refine=10)
        tilt_axis = np.array([rng.normal(), rng.normal(), 0.0])
        xm = xm @ meshes.axis_angle(tilt_axis, np.deg2rad(rng.uniform(0, 2))).T
        center = xm.mean(axis=0)
    else:
        raise ValueError(indenter)
    xm = meshes.place_above(xm, xs, g_min)
    center = center + (xm.mean(axis=0) - center) if indenter == "letter" else np.array(
        [0.0, 0.0, xm[:, 2].min() + 5e-3])
    ang = np.deg2rad(0.2)
    h = rng.normal(size=2)
    R = meshes.axis_angle([h[0], h[1], 0.0], ang)
    dxm = (xm - center) @ R.T + center - xm
    dxm[:, 2] -= 0.2e-3
    dxs = meshes.ball_uniform(rng, xs.shape[0], 20e-6)
    w = Workload(f"large_indent_{pad_n}x{pad_n}_{indenter}", xs, ts, xm, tm, rule_n, 1e5, 1e-3, 0.0,
                 dxs, dxm, info={"g_min": g_min})
    return _finish(w, fp32)


@dataclass
class Batch:
    """Environments concatenated: global vertex ids, offset tables per env."""
    envs: list
    xs: np.ndarray
    ts: np.ndarray
    xm: np.ndarray
    tm: np.ndarray
    dxs: np.ndarray
    dxm: np.ndarray
    slave_v_off: np.ndarray
    slave_t_off: np.ndarray
    master_v_off: np.ndarray
    master_t_off: np.ndarray

    @property
    def rule_n(self):
        return [w.rule_n for w in self.envs]

    @property
    def n_samples(self):
        return sum(w.n_samples for w in self.envs)


def concat(envs) -> Batch:
    vo = np.cumsum([0] + [w.xs.shape[0] for w in envs])
    to = np.cumsum([0] + [w.ts.shape[0] for w in envs])
    mvo = np.cumsum([0] + [w.xm.shape[0] for w in envs])
    mto = np.cumsum([0] + [w.tm.shape[0] for w in envs])
    return Batch(envs, np.concatenate([w.xs for w in envs]),
                 np.concatenate([w.ts + vo[i] for i, w in enumerate(envs)]).astype(np.int32),
                 np.concatenate([w.xm for w in envs]),
                 np.concatenate([w.tm + mvo[i] for i, w in enumerate(envs)]).astype(np.int32),
                 np.concatenate([w.dxs for w in envs]), np.concatenate([w.dxm for w in envs]),
                 vo, to, mvo, mto)


_GEO_CACHE = {}


def _geo(freq):
    if freq not in _GEO_CACHE:
        _GEO_CACHE[freq] = meshes.geodesic_sphere(freq, 1.0)
    x, t = _GEO_CACHE[freq]
    return x.copy(), t.copy()


def batched(n_env: int = 256, seed: int = 3000, fp32: bool = True, dt: float = 1e-3) -> Batch:
    """Many robot-learning environments of uneven size.  Environment e (seed
    seed + e): pad n x n with n ~ U{32..128} (10 mm, +-50 um noise); n x n
    samples per triangle with n ~ U{2,3,4}; geodesic-sphere indenter of
    frequency ~ U{7..45} (980..40500 triangles), R ~ U[3, 6] mm, uniform
    random rotation, lowest vertex g_min ~ U[0.01, 0.5] dhat above the pad;
    search direction = the indenter's rigid motion over dt with linear
    velocity uniform in a 0.1 m/s ball and angular speed <= 1 rad/s, pad
    vertices uniform in a 20 um ball."""
    envs = []
    for e in range(n_env):
        rng = np.random.default_rng(seed + e)
        n = int(rng.integers(32, 129))
        rule = int(rng.integers(2, 5))
        freq = int(rng.integers(7, 46))
        R = rng.uniform(3e-3, 6e-3)
        dhat = 1e-3
        xs, ts = meshes.pad(n, 1e-2, noise=50e-6, rng=rng)
        xm, tm = _geo(freq)
        xm = (xm @ meshes.random_rotation(rng).T) * R
        xm[:, :2] += rng.uniform(-1e-3, 1e-3, size=2)
        xm = meshes.place_above(xm, xs, rng.uniform(0.01, 0.5) * dhat)
        center = xm.mean(axis=0)
        v = meshes.ball_uniform(rng, 1, 0.1)[0]
        axis = rng.normal(size=3)
        Rot = meshes.axis_angle(axis, rng.uniform(0, 1.0) * dt)
        dxm = (xm - center) @ Rot.T + center - xm + v * dt
        dxs = meshes.ball_uniform(rng, xs.shape[0], 20e-6)
        w = Workload(f"env{e}", xs, ts, xm, tm, rule, 1e5, dhat, 0.0, dxs, dxm)
        envs.append(_finish(w, fp32))
    return concat(envs)


def flat_punch(n_pad: int = 8, n_punch: int = 5, gap: float = 3e-4, length: float = 1e-2,
               punch_length: float = 1.4e-2, rule_n: int = 2, fp32: bool = False) -> Workload:
    """A flat rectangular master, meshed independently of the pad (its grid
    does not match the pad's), parallel to a flat pad at a uniform gap.  The
    punch is larger than the pad so it covers every sample.  Normals: pad +z,
    punch -z (flipped triangle order)."""
    xs, ts = meshes.pad(n_pad, length)
    xm, tm = meshes.pad(n_punch, punch_length)
    tm = tm[:, [0, 2, 1]].copy()
    xm[:, 0] += 0.13 * punch_length / n_punch      # shift so the grids do not line up
    xm[:, 1] += 0.07 * punch_length / n_punch
    xm[:, 2] = gap
    z = np.zeros_like(xs)
    w = Workload("flat_punch", xs, ts, xm, tm, rule_n, 1e5, 1e-3, 0.0, z, np.zeros_like(xm))
    return _finish(w, fp32)


@dataclass
class PatchTest:
    """Two stacked linear-elastic blocks in contact (the contact patch test)."""
    X: np.ndarray          # rest positions [V, 3]: the upper block's vertices, then the lower block's
    tets: np.ndarray       # [n_tet, 4] int32, global vertex ids
    Vs: int                # vertices of the upper block (the slave body)
    ts: np.ndarray         # slave triangles: the upper block's bottom face (outward -z), ids < Vs
    tm: np.ndarray         # master triangles: the lower block's top face (outward +z), ids local to the lower block
    fixed: np.ndarray      # the lower block's bottom-face vertices (global ids): u = 0
    roller: np.ndarray     # the upper block's vertices: u_x = u_y = 0
    f_ext: np.ndarray      # [V, 3] consistent nodal forces of the pressure on the upper block's top face
    pressure: float
    young: float
    poisson: float
    dhat: float
    gap: float
    h_top: float
    h_bot: float


def patch_test(n_top: int = 4, n_bot: int = 6, size: float = 1.0, gap: float = 2e-3, pressure: float = 10.0,
               young: float = 1e3, poisson: float = 0.0, dhat: float = 1e-3) -> PatchTest:
    """The contact patch test of Sec. 5 (Table 1) on synthetic meshes: two
    blocks of size x size x size/2 (cubes of n x n x n/2 cells, six
    tetrahedra each; n even), the upper one meshed with n_top cells per
    side and the lower one with n_bot, so the interface meshes do not match
    when n_top != n_bot.  The upper block starts ``gap`` above the lower
    one; its top face carries a uniform pressure (nodal forces p A / 3 per
    adjacent face triangle, -z); the lower block's bottom face is held and
    the upper block moves only along z (u_x = u_y = 0), as in the paper."""
    if n_top % 2 or n_bot % 2:
        raise ValueError("block resolutions must be even (height = half the side)")
    ht, hb = size / n_top, size / n_bot
    Xu, Tu, top_u, _ = meshes.tet_block(n_top, n_top, n_top // 2, ht)
    Xl, Tl, top_l, bot_l = meshes.tet_block(n_bot, n_bot, n_bot // 2, hb)
    Xu = Xu + np.array([0.0, 0.0, size / 2 + gap])
    Vs = Xu.shape[0]
    X = np.concatenate([Xu, Xl])
    tets = np.concatenate([Tu, Tl + Vs]).astype(np.int32)
    ts = meshes.tet_block_bottom(n_top, n_top, n_top // 2)
    f = np.zeros_like(X)
    p = Xu[top_u]
    area = 0.5 * np.linalg.norm(np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), axis=1)
    for j in range(3):
        np.add.at(f[:, 2], top_u[:, j], -pressure * area / 3.0)
    return PatchTest(X, tets, Vs, ts, top_l.astype(np.int32), (bot_l + Vs).astype(np.int32),
                     np.arange(Vs, dtype=np.int32), f, pressure, young, poisson, dhat, gap, ht, hb)


def to_problem(w: Workload):
    """Oracle problem built from a workload (for tests and the CPU baseline)."""
    from oracle import Problem
    return Problem(w.xs, w.ts, w.xm, w.tm, w.rule_n, w.kappa, w.dhat, w.delta_T, None, w.xs_rest)


def dual_mesh(seed: int = 7, sim_freq: int = 32, vis_freq: int = 256, radius: float = 5e-3):
    """A visual mesh riding on a coarser simulation surface: the simulation
    surface is a geodesic sphere of frequency ``sim_freq`` (20 f^2
    triangles; 20480 at f = 32), the visual vertices those of a geodesic
    sphere of frequency ``vis_freq`` (10 f^2 + 2; 655362 at f = 256) with a
    uniform radial perturbation of +-0.5 % (surface detail), randomly
    rotated so the two meshes do not share vertices.  Returns
    (P [N][3], V [nV][3], F [nT][3] int32), float64."""
    rng = np.random.default_rng(seed)
    V, F = _geo(sim_freq)
    V = V * radius
    P, _ = _geo(vis_freq)
    P = (P @ meshes.random_rotation(rng).T) * radius * (1 + rng.uniform(-5e-3, 5e-3, size=(P.shape[0], 1)))
    return P, V, F


def smooth_deformation(x: np.ndarray, amp: float = 0.1, scale: float = 5e-3) -> np.ndarray:
    """A smooth non-affine deformation of points x (used to move the
    simulation surface in dual-mesh tests)."""
    y = x / scale
    d = np.stack([np.sin(2 * y[:, 1]), np.cos(1.5 * y[:, 2]) * y[:, 0], 0.5 * y[:, 0] * y[:, 1]], axis=1)
    return x + amp * scale * d
