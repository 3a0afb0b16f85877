"""Dual-mesh mapper (include/gmcp_dualmesh.h): a visual mesh embedded on the
simulation surface once, then moved with it every frame.

``DualMesh(P, V, F)`` runs the precomputation on the GPU (nearest triangle,
barycentric coordinates, normal offset, FP64); ``update(Vd)`` maps deformed
simulation positions to visual positions.  Argument marshalling only.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _native as N
from .gmcp import _check, _ptr


def _lib():
    L = N.lib()
    if not getattr(L, "_dualmesh_typed", False):
        P = C.c_void_p
        L.gmcp_dualmesh_embed.restype = C.c_int
        L.gmcp_dualmesh_embed.argtypes = [P, C.c_int64, P, P, C.c_int64, P, P, P, P, P]
        L.gmcp_dualmesh_update.restype = C.c_int
        L.gmcp_dualmesh_update.argtypes = [P, P, P, P, P, C.c_int64, P, C.c_uint32, P]
        L._dualmesh_typed = True
    return L


def _stream(dev):
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


class DualMesh:
    """Mapping (tri, bary, delta) of visual vertices P [N][3] on the
    simulation surface (V [nV][3], F [nT][3]).  ``dtype`` is the precision
    of the per-frame update (the mapping is computed in float64)."""

    def __init__(self, P, V, F, dtype=torch.float32, device="cuda"):
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.dev, self.dtype = dev, dtype
        td = lambda a: torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous()
        P, V = td(P), td(V)
        self.F = torch.as_tensor(F, dtype=torch.int32).to(dev).contiguous()
        self.N = P.shape[0]
        self.tri = torch.empty(self.N, dtype=torch.int32, device=dev)
        bary = torch.empty(self.N, 3, dtype=torch.float64, device=dev)
        delta = torch.empty(self.N, dtype=torch.float64, device=dev)
        self.dist2 = torch.empty(self.N, dtype=torch.float64, device=dev)
        _check(_lib().gmcp_dualmesh_embed(_ptr(P), self.N, _ptr(V), _ptr(self.F), self.F.shape[0], _ptr(self.tri),
                                          _ptr(bary), _ptr(delta), _ptr(self.dist2), _stream(dev)),
               "gmcp_dualmesh_embed")
        self.bary64, self.delta64 = bary, delta
        self.bary = bary.to(dtype).contiguous()
        self.delta = delta.to(dtype).contiguous()

    def update(self, Vd, out=None):
        """Visual positions [N][3] for deformed simulation positions Vd."""
        Vd = Vd.contiguous()
        if Vd.dtype != self.dtype:
            raise TypeError(f"Vd must be {self.dtype}")
        if out is None:
            out = torch.empty(self.N, 3, dtype=self.dtype, device=self.dev)
        flags = N.GMCP_F64 if self.dtype == torch.float64 else 0
        _check(_lib().gmcp_dualmesh_update(_ptr(Vd), _ptr(self.F), _ptr(self.tri), _ptr(self.bary), _ptr(self.delta),
                                           self.N, _ptr(out), flags, _stream(self.dev)), "gmcp_dualmesh_update")
        return out
