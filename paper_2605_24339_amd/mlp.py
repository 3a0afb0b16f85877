"""Learned warm start for the implicit Newton step (include/gmcp_mlp.h).

A per-vertex MLP maps (position, velocity, previous correction) to the
correction d = x* - (x_t + dt v_t) of the coming step; the Newton solve then
starts from x_t + dt v_t + d (after the same contact step-bound filter as
the plain start) and its converged solution measures the start's error.  Forward,
backward, loss and Adam run in the library's kernels (matrix cores, bf16
operands, float32 accumulation); this module holds parameters, feature
scaling and the training loop.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N
from .gmcp import GMCPError, _check, _ptr

N_IN, N_OUT, PAD = 9, 3, 16


def _lib():
    L = N.lib()
    if not getattr(L, "_mlp_typed", False):
        P = C.c_void_p
        L.gmcp_mlp_param_count.restype = C.c_int64
        L.gmcp_mlp_param_count.argtypes = []
        L.gmcp_mlp_work_bytes.restype = C.c_size_t
        L.gmcp_mlp_work_bytes.argtypes = [C.c_int64]
        L.gmcp_mlp_forward.restype = C.c_int
        L.gmcp_mlp_forward.argtypes = [P, P, C.c_int64, P, P, P]
        L.gmcp_mlp_backward.restype = C.c_int
        L.gmcp_mlp_backward.argtypes = [P, P, P, P, C.c_int64, P, P, C.c_size_t, P]
        L.gmcp_mlp_mse.restype = C.c_int
        L.gmcp_mlp_mse.argtypes = [P, P, C.c_int64, C.c_int, P, P, P, C.c_size_t, P]
        L.gmcp_mlp_mse_noalloc.restype = C.c_int
        L.gmcp_mlp_mse_noalloc.argtypes = [P, P, C.c_int64, C.c_int, P, P, P]
        L.gmcp_mlp_mse_noalloc_max_rows.restype = C.c_int64
        L.gmcp_mlp_mse_noalloc_max_rows.argtypes = []
        L.gmcp_mlp_adam.restype = C.c_int
        L.gmcp_mlp_adam.argtypes = [P, P, P, P, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int, P]
        L.gmcp_gemm_bf16.restype = C.c_int
        L.gmcp_gemm_bf16.argtypes = [P, C.c_int, C.c_int, P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P,
                                     C.c_int, P]
        L._mlp_typed = True
    return L


def _stream(dev):
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def gemm_bf16(A, B, transA=False, transB=False):
    """C = op(A) op(B) on the matrix cores (float32 in/out, bf16 operands)."""
    A = A.contiguous()
    B = B.contiguous()
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N_ = B.shape[0] if transB else B.shape[1]
    out = torch.empty(M, N_, dtype=torch.float32, device=A.device)
    _check(_lib().gmcp_gemm_bf16(_ptr(A), A.shape[1], int(transA), _ptr(B), B.shape[1], int(transB), M, N_, K,
                                 _ptr(out), N_, _stream(A.device)), "gmcp_gemm_bf16")
    return out


class MLP:
    """Parameters (float32, device) and the kernel calls around them."""

    def __init__(self, params: torch.Tensor):
        self.n = int(_lib().gmcp_mlp_param_count())
        if params.numel() != self.n or params.dtype != torch.float32:
            raise ValueError(f"expected {self.n} float32 parameters")
        self.p = params.contiguous()
        self.dev = params.device
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.step = 0

    def forward(self, x, act=None):
        B = x.shape[0]
        y = torch.empty(B, PAD, dtype=torch.float32, device=self.dev)
        act = torch.empty(B, 6 * 128, dtype=torch.float32, device=self.dev) if act is None else act
        _check(_lib().gmcp_mlp_forward(_ptr(self.p), _ptr(x), B, _ptr(y), _ptr(act), _stream(self.dev)),
               "gmcp_mlp_forward")
        return y, act

    def predict(self, x):
        """y [B][16] = MLP(x) without saving activations (inference)."""
        B = x.shape[0]
        y = torch.empty(B, PAD, dtype=torch.float32, device=self.dev)
        _check(_lib().gmcp_mlp_forward(_ptr(self.p), _ptr(x), B, _ptr(y), None, _stream(self.dev)),
               "gmcp_mlp_forward")
        return y

    def backward(self, x, act, dy):
        B = x.shape[0]
        g = torch.empty_like(self.p)
        wb = int(_lib().gmcp_mlp_work_bytes(B))
        work = torch.empty(wb // 4 + 64, dtype=torch.float32, device=self.dev)
        _check(_lib().gmcp_mlp_backward(_ptr(self.p), _ptr(x), _ptr(act), _ptr(dy), B, _ptr(g), _ptr(work), wb,
                                        _stream(self.dev)), "gmcp_mlp_backward")
        return g

    def mse(self, y, t, n_out=N_OUT):
        B = y.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=self.dev)
        dy = torch.empty_like(y)
        nbytes = 4 * ((B * PAD + 255) // 256 + 1)
        work = torch.empty(nbytes // 4, dtype=torch.float32, device=self.dev)
        _check(_lib().gmcp_mlp_mse(_ptr(y), _ptr(t), B, n_out, _ptr(loss), _ptr(dy), _ptr(work), nbytes,
                                   _stream(self.dev)), "gmcp_mlp_mse")
        return loss, dy

    def adam(self, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _check(_lib().gmcp_mlp_adam(_ptr(self.p), _ptr(g), _ptr(self.m), _ptr(self.v), self.n, lr, b1, b2, eps,
                                    self.step, _stream(self.dev)), "gmcp_mlp_adam")

    def train(self, X, T, epochs=3, batch=65536, lr=1e-3, seed=0, log=None, lr_min=None):
        """Minibatch Adam on rows (X [R][16], T [R][16] device tensors); with
        lr_min the rate follows a cosine from lr down to lr_min over the run."""
        R = X.shape[0]
        gen = torch.Generator(device="cpu").manual_seed(seed)
        hist = []
        act = torch.empty(batch, 6 * 128, dtype=torch.float32, device=self.dev)
        total = max(1, epochs * (R // batch))
        k = 0
        for ep in range(epochs):
            perm = torch.randperm(R, generator=gen).to(self.dev)
            tot, ns, nb = 0.0, 0, 0
            for i in range(0, R - batch + 1, batch):
                idx = perm[i:i + batch]
                xb, tb = X[idx].contiguous(), T[idx].contiguous()
                y, a = self.forward(xb, act)
                loss, dy = self.mse(y, tb)
                g = self.backward(xb, a, dy)
                rate = lr if lr_min is None else lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * k / total))
                self.adam(g, lr=float(rate))
                k += 1
                if nb % 16 == 0:          # sampled batch losses (a host sync each)
                    tot += float(loss.item())
                    ns += 1
                nb += 1
            hist.append(tot / max(ns, 1))
            if log:
                log(f"epoch {ep}: {nb} batches")
        return hist


def targets(x_star, x_t, v_t, dt, h):
    V = x_t.shape[0]
    t = torch.zeros(V, PAD, dtype=torch.float32, device=x_t.device)
    t[:, 0:3] = ((x_star - (x_t + dt * v_t)) / h).float()
    return t
