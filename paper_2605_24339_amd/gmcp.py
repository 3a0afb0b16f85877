"""Python front end of the GMCP HIP library.

Thin marshalling over the C ABI (include/gmcp.h): torch tensors provide
device memory and the HIP stream; every step of the hot path runs in the
library's kernels.  There is no CPU fallback: without the built library or
a GPU every call raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _native as N


class GMCPError(RuntimeError):
    def __init__(self, code: int, index: int = -1, where: str = ""):
        super().__init__(f"{where}: {N.strerror(code)} (code {code}, index {index})")
        self.code = code
        self.index = index


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(rc: int, where: str):
    if rc != N.GMCP_OK:
        raise GMCPError(rc, -1, where)


@dataclass
class BSR:
    row_ptr: torch.Tensor   # [V+1] int32
    col: torch.Tensor       # [nnzb] int32
    val: torch.Tensor       # [nnzb, 3, 3]

    def to_dense(self) -> torch.Tensor:
        V = self.row_ptr.numel() - 1
        rows = torch.repeat_interleave(torch.arange(V, device=self.col.device),
                                       (self.row_ptr[1:] - self.row_ptr[:-1]).long())
        H = torch.zeros(3 * V, 3 * V, dtype=self.val.dtype, device=self.val.device)
        for a in range(3):
            for b in range(3):
                H[3 * rows + a, 3 * self.col.long() + b] = self.val[:, a, b]
        return H


@dataclass
class Assembly:
    energy: torch.Tensor          # [n_env]
    grad: torch.Tensor | None     # [V, 3]
    hessian: BSR | None


class Context:
    """One GMCP problem (possibly many environments) resident on one GPU.

    Meshes are concatenated over environments; triangle vertex ids are global
    (slave ids in [0, Vs), master ids in [0, Vm)).  Per-environment arrays:
    rule_n (n in 1..4, n*n samples per slave triangle), kappa, dhat
    (eps_max), delta_T (face transition width), cell (broad-phase cell size,
    0 = automatic).  mortar=True uses clipped mortar face samples (every
    opposing pair's projected overlap, fan-triangulated, n x n rule per
    sub-triangle) instead of one whole-triangle rule per slave triangle;
    features=True adds edge and point samples of the opposing master
    triangles (stiffnesses kappa_edge, kappa_point, edge transition width
    delta_e per environment).
    """

    def __init__(self, slave_tri, master_tri, slave_v_off, slave_t_off, master_v_off, master_t_off,
                 rule_n, kappa, dhat, delta_T, cell=None, dtype=torch.float32, kinematic=False,
                 caps: dict | None = None, device="cuda", mortar: bool = False, features: bool = False,
                 kappa_edge=None, kappa_point=None, delta_e=None):
        N.lib()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dtype = dtype
        self.kinematic = bool(kinematic)
        self._side = None          # second stream of the overlapped step (created on first use)
        self._profiling = False
        self._tuning = None        # launch shapes (gmcp_set_tuning), kept across re-creation
        self.mortar = bool(mortar) or bool(features)
        self.features = bool(features)
        self.ts = torch.as_tensor(slave_tri, dtype=torch.int32).to(self.device).contiguous()
        self.tm = torch.as_tensor(master_tri, dtype=torch.int32).to(self.device).contiguous()
        self.n_env = len(rule_n)
        as_i32 = lambda v: (C.c_int32 * len(v))(*[int(x) for x in v])
        as_f64 = lambda v: (C.c_double * len(v))(*[float(x) for x in v])
        self._keep = dict(svo=as_i32(slave_v_off), sto=as_i32(slave_t_off), mvo=as_i32(master_v_off),
                          mto=as_i32(master_t_off), rule=as_i32(rule_n), kappa=as_f64(kappa),
                          dhat=as_f64(dhat), dT=as_f64(delta_T),
                          cell=as_f64(cell if cell is not None else [0.0] * self.n_env),
                          ke=as_f64(kappa_edge if kappa_edge is not None else [0.0] * self.n_env),
                          kp=as_f64(kappa_point if kappa_point is not None else [0.0] * self.n_env),
                          de=as_f64(delta_e if delta_e is not None else [0.0] * self.n_env))
        k = self._keep
        flags = ((N.GMCP_F64 if dtype == torch.float64 else 0) | (N.GMCP_KINEMATIC_MASTER if kinematic else 0)
                 | (N.GMCP_MORTAR if self.mortar else 0) | (N.GMCP_FEATURES if self.features else 0))
        cast = lambda a, t: C.cast(a, C.POINTER(t))
        self.layout = N.Layout(self.n_env, cast(k["svo"], C.c_int32), cast(k["sto"], C.c_int32),
                               cast(k["mvo"], C.c_int32), cast(k["mto"], C.c_int32),
                               cast(k["rule"], C.c_int32), cast(k["kappa"], C.c_double),
                               cast(k["dhat"], C.c_double), cast(k["dT"], C.c_double),
                               cast(k["cell"], C.c_double), flags, cast(k["ke"], C.c_double),
                               cast(k["kp"], C.c_double), cast(k["de"], C.c_double))
        self.Vs, self.Ts = int(slave_v_off[-1]), int(slave_t_off[-1])
        self.Vm, self.Tm = int(master_v_off[-1]), int(master_t_off[-1])
        self.Ns = sum((int(slave_t_off[e + 1]) - int(slave_t_off[e])) * int(rule_n[e]) ** 2
                      for e in range(self.n_env))
        self.V = self.Vs if kinematic else self.Vs + self.Vm
        # grid cell budget: 2 per triangle (the support radius usually sets
        # the cell size; a budget of 8 per triangle only made the cell-count
        # scans longer: 256-environment step 6.07 -> 6.01 ms at 2)
        c = dict(grid_cells=2 * (self.Ts + self.Tm) + 4096 * self.n_env,
                 grid_items=16 * self.Tm + 4096, candidates=16 * self.Ts + 4096,
                 active=(3 * self.Ns if self.mortar else self.Ns) + 64, pairs=self.Ns // 2 + 1024,
                 row_entries=256)
        if caps:
            c.update(caps)
        self.caps = c
        self.cap_nnzb = 24 * c["pairs"] + 1024
        self._ctx = None
        self._x_rest = None
        self._last_x = None
        self._create()

    # ------------------------------------------------------------------ setup
    def _create(self):
        if self._ctx is not None:
            N.lib().gmcp_destroy(self._ctx)
            self._ctx = None
        c = self.caps
        self._caps_s = N.Caps(c["grid_cells"], c["grid_items"], c["candidates"], c["active"], c["pairs"],
                              c["row_entries"])
        size = N.lib().gmcp_workspace_size(C.byref(self.layout), C.byref(self._caps_s))
        if size == 0:
            raise GMCPError(N.GMCP_E_ARG, -1, "gmcp_workspace_size")
        self.workspace = torch.empty(size + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        ctx = C.c_void_p()
        rc = N.lib().gmcp_create(C.byref(ctx), C.byref(self.layout), C.byref(self._caps_s),
                                 _ptr(self.ts), _ptr(self.tm), C.c_void_p(aligned), size, self._stream())
        _check(rc, "gmcp_create")
        self._ctx = ctx
        self.energy = torch.zeros(self.n_env, dtype=self.dtype, device=self.device)
        self.grad = torch.zeros(self.V, 3, dtype=self.dtype, device=self.device)
        self.row_ptr = torch.zeros(self.V + 1, dtype=torch.int32, device=self.device)
        self.col = torch.zeros(self.cap_nnzb, dtype=torch.int32, device=self.device)
        self.val = torch.zeros(self.cap_nnzb, 3, 3, dtype=self.dtype, device=self.device)
        self.alpha = torch.ones(self.n_env, dtype=self.dtype, device=self.device)
        self._bsr = N.Bsr(_ptr(self.row_ptr), _ptr(self.col), _ptr(self.val), self.cap_nnzb)
        if self._tuning is not None:
            _check(N.lib().gmcp_set_tuning(self._ctx, C.byref(self._tuning)), "gmcp_set_tuning")
        if self._x_rest is not None:
            self.build_samples(self._x_rest)

    def __del__(self):
        try:
            if self._ctx is not None:
                N.lib().gmcp_destroy(self._ctx)
        except Exception:
            pass

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _bind(self):
        _check(N.lib().gmcp_set_stream(self._ctx, self._stream()), "gmcp_set_stream")

    def _x(self, x, n, name):
        if x is None:
            return None
        if x.dtype != self.dtype or x.device != self.device or not x.is_contiguous() or tuple(x.shape) != (n, 3):
            raise ValueError(f"{name}: expected contiguous [{n}, 3] {self.dtype} on {self.device}, "
                             f"got {tuple(x.shape)} {x.dtype} {x.device}")
        return x

    def _vec(self, v, n, name):
        if v is None:
            return None
        if v.dtype != self.dtype or v.device != self.device or not v.is_contiguous() or v.numel() != n:
            raise ValueError(f"{name}: expected contiguous [{n}] {self.dtype} on {self.device}")
        return v

    TUNING_FIELDS = ("query_blocks", "light_row_bound", "light_row_blocks", "heavy_row_blocks")

    def set_tuning(self, **shapes):
        """Launch shapes of the list-walking kernels (gmcp_tuning; 0 = the
        default); fields not given keep their current value."""
        cur = self._tuning if self._tuning is not None else N.Tuning(0, 0, 0, 0)
        vals = {f: int(shapes.get(f, getattr(cur, f))) for f in self.TUNING_FIELDS}
        t = N.Tuning(*[vals[f] for f in self.TUNING_FIELDS])
        _check(N.lib().gmcp_set_tuning(self._ctx, C.byref(t)), "gmcp_set_tuning")
        self._tuning = t

    def tuning(self) -> dict:
        """Launch shapes in effect (defaults filled in)."""
        t = N.Tuning()
        _check(N.lib().gmcp_get_tuning(self._ctx, C.byref(t)), "gmcp_get_tuning")
        return {f: int(getattr(t, f)) for f in self.TUNING_FIELDS}

    def status(self) -> N.StatusInfo:
        info = N.StatusInfo()
        _check(N.lib().gmcp_status(self._ctx, C.byref(info)), "gmcp_status")
        return info

    def _raise_or_grow(self, info, where) -> bool:
        """True if capacities were grown (caller retries); raises on other errors."""
        if info.code == N.GMCP_OK:
            return False
        if info.code != N.GMCP_E_CAPACITY:
            raise GMCPError(info.code, info.index, where)
        need = info.need
        grew = False
        for key, val in (("grid_items", need.grid_items), ("candidates", need.candidates),
                         ("active", need.active), ("pairs", need.pairs)):
            if val > self.caps[key]:
                self.caps[key] = int(val * 1.25) + 1024
                grew = True
        if info.nnzb > self.cap_nnzb:
            self.cap_nnzb = int(info.nnzb * 1.25) + 1024
            grew = True
        if need.row_entries > self.caps["row_entries"]:
            if self.caps["row_entries"] >= 4096:
                raise GMCPError(N.GMCP_E_CAPACITY, -1,
                                f"{where}: a BSR row has more than 4096 distinct columns")
            self.caps["row_entries"] = min(4096, int(need.row_entries))
            grew = True
        if not grew:
            raise GMCPError(info.code, info.index, where)
        self._create()
        return True

    # --------------------------------------------------------------- the path
    def build_samples(self, x_rest, weights: bool = False):
        """Rest areas, Morton-ordered tiles; returns sample weights w_k if asked."""
        x_rest = self._x(x_rest, self.Vs, "x_rest")
        self._x_rest = x_rest
        self._bind()
        w = torch.empty(self.Ns, dtype=self.dtype, device=self.device) if weights else None
        _check(N.lib().gmcp_build_samples(self._ctx, _ptr(x_rest), _ptr(w)), "gmcp_build_samples")
        return w

    def broadphase(self, xs, xm, check: bool = True):
        xs = self._x(xs, self.Vs, "x_slave")
        xm = self._x(xm, self.Vm, "x_master")
        for _ in range(4):
            self._bind()
            _check(N.lib().gmcp_broadphase(self._ctx, _ptr(xs), _ptr(xm)), "gmcp_broadphase")
            self._last_x = (xs, xm)
            if not check or not self._raise_or_grow(self.status(), "gmcp_broadphase"):
                return
        raise GMCPError(N.GMCP_E_CAPACITY, -1, "gmcp_broadphase: capacities did not settle")

    def assemble(self, xs, xm, g_ref=None, delta_gap=None, grad: bool = True, hessian: bool = True,
                 check: bool = True) -> Assembly:
        xs = self._x(xs, self.Vs, "x_slave")
        xm = self._x(xm, self.Vm, "x_master")
        g_ref = self._vec(g_ref, self.Ts if self.mortar else self.Ns, "g_ref")
        delta_gap = self._vec(delta_gap, self.Ns, "delta_gap")
        for _ in range(6):  # capacities only grow; a row table grows to its final size at once
            self._bind()
            rc = N.lib().gmcp_assemble(self._ctx, _ptr(xs), _ptr(xm), _ptr(g_ref), _ptr(delta_gap),
                                       _ptr(self.energy), _ptr(self.grad) if grad else None,
                                       C.byref(self._bsr) if hessian else None)
            _check(rc, "gmcp_assemble")
            if not check:
                return Assembly(self.energy, self.grad if grad else None,
                                BSR(self.row_ptr, self.col, self.val) if hessian else None)
            info = self.status()
            if not self._raise_or_grow(info, "gmcp_assemble"):
                H = None
                if hessian:
                    nb = int(info.nnzb)
                    H = BSR(self.row_ptr, self.col[:nb], self.val[:nb])
                return Assembly(self.energy, self.grad if grad else None, H)
            self.broadphase(xs, xm, check=True)
        raise GMCPError(N.GMCP_E_CAPACITY, -1, "gmcp_assemble: capacities did not settle")

    def ccd_step(self, xs, xm, dxs, dxm=None, check: bool = True) -> torch.Tensor:
        xs = self._x(xs, self.Vs, "x_slave")
        xm = self._x(xm, self.Vm, "x_master")
        dxs = self._x(dxs, self.Vs, "dx_slave")
        dxm = self._x(dxm, self.Vm, "dx_master")
        for _ in range(4):
            self._bind()
            _check(N.lib().gmcp_ccd_step(self._ctx, _ptr(xs), _ptr(xm), _ptr(dxs), _ptr(dxm), _ptr(self.alpha)),
                   "gmcp_ccd_step")
            if not check or not self._raise_or_grow(self.status(), "gmcp_ccd_step"):
                return self.alpha
            self.broadphase(xs, xm)
            self.assemble(xs, xm, grad=False, hessian=False)
        raise GMCPError(N.GMCP_E_CAPACITY, -1, "gmcp_ccd_step: capacities did not settle")

    def ccd_swept(self, xs, xm, dxs, dxm=None):
        """First part of the step bound (swept grid + additive CCD) on the
        current stream; no capacity check (see ``step``)."""
        xs = self._x(xs, self.Vs, "x_slave")
        xm = self._x(xm, self.Vm, "x_master")
        dxs = self._x(dxs, self.Vs, "dx_slave")
        dxm = self._x(dxm, self.Vm, "dx_master")
        self._bind()
        _check(N.lib().gmcp_ccd_swept(self._ctx, _ptr(xs), _ptr(xm), _ptr(dxs), _ptr(dxm)), "gmcp_ccd_swept")

    def ccd_finish(self, dxs, dxm=None) -> torch.Tensor:
        """Second part of the step bound (Eq. (ccd) over the assembled samples)."""
        dxs = self._x(dxs, self.Vs, "dx_slave")
        dxm = self._x(dxm, self.Vm, "dx_master")
        self._bind()
        _check(N.lib().gmcp_ccd_finish(self._ctx, _ptr(dxs), _ptr(dxm), _ptr(self.alpha)), "gmcp_ccd_finish")
        return self.alpha

    def step(self, xs, xm, dxs, dxm=None, check: bool = False):
        """One pass of the whole hot path: broad phase, assembly (energy,
        gradient, BSR Hessian), step bound.  Unchecked and not profiled, the
        step bound's swept part (grid + additive CCD, independent of the
        assembly) runs on a second stream, forked from the current one after
        the broad phase and joined back before the final bound, so it overlaps
        the assembly (also inside a captured graph); the broad phase, whose
        query walks its list with a grid sized to the whole device, runs
        alone."""
        if check or self._profiling:
            self.broadphase(xs, xm, check=check)
            A = self.assemble(xs, xm, check=check)
            alpha = self.ccd_step(xs, xm, dxs, dxm, check=check)
            return A, alpha
        main = torch.cuda.current_stream(self.device)
        if self._side is None:
            self._side = torch.cuda.Stream(self.device)  # default priority
        self.broadphase(xs, xm, check=False)
        self._side.wait_stream(main)
        with torch.cuda.stream(self._side):
            self.ccd_swept(xs, xm, dxs, dxm)
        A = self.assemble(xs, xm, check=False)
        main.wait_stream(self._side)
        alpha = self.ccd_finish(dxs, dxm)
        return A, alpha

    def capture(self, xs, xm, dxs, dxm=None) -> "torch.cuda.CUDAGraph":
        """Capture one full step into a HIP graph.  ``graph.replay()`` re-runs
        it on whatever the same input tensors hold; outputs land in this
        context's energy / grad / BSR / alpha buffers.  Capacities are settled
        by a checked step first (no host synchronisation inside the graph)."""
        self.step(xs, xm, dxs, dxm, check=True)
        torch.cuda.synchronize(self.device)
        side = torch.cuda.Stream(self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            self.step(xs, xm, dxs, dxm)
        torch.cuda.current_stream(self.device).wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(xs, xm, dxs, dxm)
        self._bind()
        return g

    def hvp(self, vx, vd=None):
        vx = self._x(vx, self.V, "v_x")
        vd = self._vec(vd, self.Ns, "v_d")
        ox = torch.empty(self.V, 3, dtype=self.dtype, device=self.device)
        # clipped mortar samples have no fixed ids: no per-sample part
        od = None if self.mortar else torch.empty(self.Ns, dtype=self.dtype, device=self.device)
        self._bind()
        _check(N.lib().gmcp_hvp(self._ctx, _ptr(vx), _ptr(vd), _ptr(ox), _ptr(od)), "gmcp_hvp")
        return ox, od

    def row_classes(self) -> dict:
        """Light / heavy BSR rows and their blocks in the last assembly (synchronises)."""
        out = (C.c_int64 * 4)()
        self._bind()
        _check(N.lib().gmcp_row_classes(self._ctx, out, _ptr(self.row_ptr)), "gmcp_row_classes")
        return dict(rows_light=out[0], rows_heavy=out[1], nnzb_light=out[2], nnzb_heavy=out[3])

    def energy_frozen(self, xs, xm) -> torch.Tensor:
        """Energy [n_env] of the last assembly's samples at positions (xs, xm),
        every sample frozen (gradient at the assembly point = assembled gradient)."""
        xs = self._x(xs, self.Vs, "x_slave")
        xm = self._x(xm, self.Vm, "x_master")
        out = torch.empty(self.n_env, dtype=self.dtype, device=self.device)
        self._bind()
        _check(N.lib().gmcp_energy_frozen(self._ctx, _ptr(xs), _ptr(xm), _ptr(out)), "gmcp_energy_frozen")
        return out

    def sample_results(self):
        M = torch.empty(self.Ns, dtype=torch.int32, device=self.device)
        mk = lambda *s: torch.empty(*s, dtype=self.dtype, device=self.device)
        g, bm, c1, c2, p = mk(self.Ns), mk(self.Ns, 3), mk(self.Ns), mk(self.Ns), mk(self.Ns)
        self._bind()
        _check(N.lib().gmcp_sample_results(self._ctx, _ptr(M), _ptr(g), _ptr(bm), _ptr(c1), _ptr(c2), _ptr(p)),
               "gmcp_sample_results")
        return dict(M=M, g=g, bm=bm, c1=c1, c2=c2, p=p)

    def pairs(self):
        """(slave triangle, master triangle) of every contact pair of the last
        assembly: int32 tensors T [n], M [n] in storage order."""
        n = int(self.status().n_pairs)
        T = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        M = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        self._bind()
        _check(N.lib().gmcp_pairs(self._ctx, _ptr(T), _ptr(M), n), "gmcp_pairs")
        return T[:n], M[:n]

    def candidates(self):
        info = self.status()
        n = int(info.n_candidates)
        off = torch.empty(self.Ts + 1, dtype=torch.int32, device=self.device)
        cand = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        self._bind()
        _check(N.lib().gmcp_candidates(self._ctx, _ptr(off), _ptr(cand), n), "gmcp_candidates")
        return off, cand[:n]

    def profile(self, enable: bool = True):
        """Start (clears) or stop per-stage HIP-event timing on this context's
        stream (steps then run their stages in order on one stream)."""
        _check(N.lib().gmcp_profile(self._ctx, int(enable)), "gmcp_profile")
        self._profiling = bool(enable)

    def profile_read(self) -> dict:
        """{stage: (total_ms, occurrences)} since the last profile(True); synchronises."""
        n = N.lib().gmcp_profile_stages()
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        _check(N.lib().gmcp_profile_read(self._ctx, ms, cnt), "gmcp_profile_read")
        return {N.lib().gmcp_profile_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(n)}

    # ------------------------------------------------------------ convenience
    @classmethod
    def single(cls, slave_tri, master_tri, n_slave_verts: int, n_master_verts: int, rule_n: int = 2,
               kappa: float = 1e5, dhat: float = 1e-3, delta_T: float = 0.0, cell: float = 0.0,
               dtype=torch.float32, kinematic: bool = False, caps=None, device="cuda", mortar: bool = False,
               features: bool = False, kappa_edge: float = 0.0, kappa_point: float = 0.0, delta_e: float = 0.0):
        Ts = int(len(slave_tri))
        Tm = int(len(master_tri))
        return cls(slave_tri, master_tri, [0, n_slave_verts], [0, Ts], [0, n_master_verts], [0, Tm],
                   [rule_n], [kappa], [dhat], [delta_T], [cell], dtype=dtype, kinematic=kinematic, caps=caps,
                   device=device, mortar=mortar, features=features, kappa_edge=[kappa_edge],
                   kappa_point=[kappa_point], delta_e=[delta_e])
