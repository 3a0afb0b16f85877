"""Differentiable GMCP energy.

``gmcp_energy(backend, x_s, x_m, delta)`` returns the total barrier energy
E(x, delta) of Eq. (gmcp_potential), where delta is a per-sample offset
added to every selected sample's gap (delta = 0 gives the plain energy).

* backward ("force kernel"): dE/dx is the assembled gradient, dE/ddelta_k
  is c1_k = kappa w_k gamma_k B'(g_k) - both produced by the assembly;
* double backward: the joint Hessian-vector product of the library, with
  the samples of the assembly frozen (the paper's gradient / Hessian
  approximation, Sec. 4.2).

The per-sample contact pressure of the tactile map is p = -dE/ddelta / w,
so a loss on p is differentiated through the double backward.

``backend`` is any object with the methods of :class:`Context` used here
(broadphase, assemble, sample_results, hvp, Vs, Vm, Ns); the product
passes a :class:`Context`.  The samples stay frozen between a forward and
its backward passes: do not assemble the same context in between.
"""
from __future__ import annotations

import torch


class _Force(torch.autograd.Function):
    """(x_s, x_m, delta, scale) -> scale * (dE/dx_s, dE/dx_m, dE/ddelta)."""

    @staticmethod
    def forward(ctx, x_s, x_m, delta, scale, backend, g_s, g_m, c1):
        ctx.backend = backend
        ctx.save_for_backward(scale, g_s, g_m, c1)
        return scale * g_s, scale * g_m, scale * c1

    @staticmethod
    def backward(ctx, go_s, go_m, go_d):
        scale, g_s, g_m, c1 = ctx.saved_tensors
        be = ctx.backend
        z = lambda t, like: torch.zeros_like(like) if t is None else t
        go_s, go_m, go_d = z(go_s, g_s), z(go_m, g_m), z(go_d, c1)
        if be.kinematic:
            vx = go_s.contiguous()
        else:
            vx = torch.cat([go_s, go_m], 0).contiguous()
        hx, hd = be.hvp(vx, go_d.contiguous())
        d_scale = (go_s * g_s).sum() + (go_m * g_m).sum() + (go_d * c1).sum()
        h_s = hx[:be.Vs]
        h_m = torch.zeros_like(g_m) if be.kinematic else hx[be.Vs:]
        return scale * h_s, scale * h_m, scale * hd, d_scale.reshape(scale.shape), None, None, None, None


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x_s, x_m, delta, backend):
        backend.broadphase(x_s, x_m)
        A = backend.assemble(x_s, x_m, delta_gap=delta, grad=True, hessian=False)
        S = backend.sample_results()
        g = A.grad.clone()
        ctx.backend = backend
        g_s = g[:backend.Vs]
        g_m = torch.zeros_like(x_m) if backend.kinematic else g[backend.Vs:]
        ctx.save_for_backward(x_s, x_m, delta, g_s, g_m, S["c1"].clone())
        return A.energy.sum().clone()

    @staticmethod
    def backward(ctx, gE):
        x_s, x_m, delta, g_s, g_m, c1 = ctx.saved_tensors
        scale = gE.reshape(())
        f_s, f_m, f_d = _Force.apply(x_s, x_m, delta, scale, ctx.backend, g_s, g_m, c1)
        return f_s, f_m, f_d, None


def gmcp_energy(backend, x_s, x_m, delta=None):
    """Total GMCP energy (sum over environments), differentiable twice."""
    if delta is None:
        delta = torch.zeros(backend.Ns, dtype=x_s.dtype, device=x_s.device)
    return _Energy.apply(x_s, x_m, delta, backend)


def pressure_map(backend, x_s, x_m, delta, weights):
    """p_k = -dE/ddelta_k / w_k as a differentiable function of (x, delta)."""
    if not delta.requires_grad:
        delta = delta.detach().requires_grad_(True)
    E = gmcp_energy(backend, x_s, x_m, delta)
    (dE_dd,) = torch.autograd.grad(E, delta, create_graph=True)
    return -dE_dd / weights
