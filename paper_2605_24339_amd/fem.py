"""Binding of the implicit-step system (include/gmcp_fem.h): linear-elastic
tetrahedra, lumped mass, block-Jacobi PCG on M/dt^2 + K + H_contact."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N
from .gmcp import BSR, GMCPError, _check, _ptr


def _lib():
    L = N.lib()
    if not getattr(L, "_fem_typed", False):
        P = C.c_void_p
        L.gmcp_fem_workspace_size.restype = C.c_size_t
        L.gmcp_fem_workspace_size.argtypes = [P, C.c_int64, C.c_int64]
        L.gmcp_fem_create.restype = C.c_int
        L.gmcp_fem_create.argtypes = [C.POINTER(P), P, C.c_int64, C.c_int64, P, C.c_double, C.c_double,
                                      C.c_double, C.c_double, P, C.c_int64, P, C.c_size_t, P]
        L.gmcp_fem_destroy.restype = None
        L.gmcp_fem_destroy.argtypes = [P]
        L.gmcp_fem_constrain.restype = C.c_int
        L.gmcp_fem_constrain.argtypes = [P, P, C.c_int64, C.c_int]
        L.gmcp_fem_set_stream.restype = C.c_int
        L.gmcp_fem_set_stream.argtypes = [P, P]
        L.gmcp_fem_nnzb.restype = C.c_int64
        L.gmcp_fem_nnzb.argtypes = [P]
        L.gmcp_fem_stiffness.restype = C.c_int
        L.gmcp_fem_stiffness.argtypes = [P, P, P, P]
        L.gmcp_fem_energy.restype = C.c_int
        L.gmcp_fem_energy.argtypes = [P, P, P, P, P]
        L.gmcp_fem_apply.restype = C.c_int
        L.gmcp_fem_apply.argtypes = [P, P, P, P, P, P]
        L.gmcp_fem_solve.restype = C.c_int
        L.gmcp_fem_solve.argtypes = [P, P, P, P, P, P, C.c_double, C.c_int, C.POINTER(C.c_int),
                                     C.POINTER(C.c_double)]
        L._fem_typed = True
    return L


class Fem:
    def __init__(self, X_rest, tets, young, poisson, density, dt, fixed, device="cuda"):
        L = _lib()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        X = np.ascontiguousarray(X_rest, dtype=np.float64)
        T = np.ascontiguousarray(tets, dtype=np.int32)
        F = np.ascontiguousarray(fixed, dtype=np.int32)
        self.V, self.n_tet, self.dt = X.shape[0], T.shape[0], float(dt)
        size = L.gmcp_fem_workspace_size(T.ctypes.data, T.shape[0], X.shape[0])
        if size == 0:
            raise GMCPError(N.GMCP_E_ARG, -1, "gmcp_fem_workspace_size")
        self.workspace = torch.empty(size + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        h = C.c_void_p()
        rc = L.gmcp_fem_create(C.byref(h), T.ctypes.data, T.shape[0], X.shape[0], X.ctypes.data, float(young),
                               float(poisson), float(density), float(dt), F.ctypes.data, F.shape[0],
                               C.c_void_p(aligned), size, self._stream())
        _check(rc, "gmcp_fem_create")
        self._h = h
        self.X = torch.tensor(X, device=self.device)
        # held displacement components [V, 3] (whole Dirichlet vertices, rollers)
        self.fixed = torch.zeros(self.V, 3, dtype=torch.bool, device=self.device)
        self.fixed[torch.tensor(F, dtype=torch.long, device=self.device)] = True
        self._e = torch.zeros(1, dtype=torch.float64, device=self.device)

    def __del__(self):
        try:
            _lib().gmcp_fem_destroy(self._h)
        except Exception:
            pass

    def constrain(self, verts, mask: int):
        """Hold components of vertices: mask bit d (1 = x, 2 = y, 4 = z)."""
        V = np.ascontiguousarray(verts, dtype=np.int32)
        self._bind()
        _check(_lib().gmcp_fem_constrain(self._h, V.ctypes.data, V.shape[0], int(mask)), "gmcp_fem_constrain")
        idx = torch.tensor(V, dtype=torch.long, device=self.device)
        for d in range(3):
            if (mask >> d) & 1:
                self.fixed[idx, d] = True

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _bind(self):
        _check(_lib().gmcp_fem_set_stream(self._h, self._stream()), "gmcp_fem_set_stream")

    def stiffness(self) -> BSR:
        nnzb = _lib().gmcp_fem_nnzb(self._h)
        rp = torch.empty(self.V + 1, dtype=torch.int32, device=self.device)
        col = torch.empty(nnzb, dtype=torch.int32, device=self.device)
        val = torch.empty(nnzb, 3, 3, dtype=torch.float64, device=self.device)
        self._bind()
        _check(_lib().gmcp_fem_stiffness(self._h, _ptr(rp), _ptr(col), _ptr(val)), "gmcp_fem_stiffness")
        return BSR(rp, col, val)

    def energy(self, x, x_tilde, grad: bool = True):
        g = torch.empty(self.V, 3, dtype=torch.float64, device=self.device) if grad else None
        self._bind()
        _check(_lib().gmcp_fem_energy(self._h, _ptr(x), _ptr(x_tilde), _ptr(self._e), _ptr(g)), "gmcp_fem_energy")
        return self._e.clone(), g

    @staticmethod
    def _h_ptrs(H):
        # no contact blocks: H is absent (an empty tensor has no storage, so
        # its pointer would be null next to a valid row_ptr)
        if H is None or H.col.numel() == 0:
            return None, None, None
        return _ptr(H.row_ptr), _ptr(H.col), _ptr(H.val)

    def apply(self, H, x):
        y = torch.empty_like(x)
        self._bind()
        _check(_lib().gmcp_fem_apply(self._h, *self._h_ptrs(H), _ptr(x), _ptr(y)), "gmcp_fem_apply")
        return y

    def solve(self, H, rhs, rtol=1e-8, max_iter=5000):
        x = torch.empty_like(rhs)
        it = C.c_int(0)
        rr = C.c_double(0.0)
        self._bind()
        _check(_lib().gmcp_fem_solve(self._h, *self._h_ptrs(H), _ptr(rhs.contiguous()), _ptr(x), float(rtol),
                                     int(max_iter), C.byref(it), C.byref(rr)), "gmcp_fem_solve")
        return x, it.value, rr.value
