"""A stand-in backend with the Context methods the autograd wrapper uses,
evaluated by the FP64 oracle on the CPU (test infrastructure: lets the
autograd plumbing be checked without a GPU)."""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np
import torch

import oracle


class OracleBackend:
    def __init__(self, w, kinematic=False):
        self.w = w
        self.kinematic = kinematic
        self.Vs, self.Vm = w.xs.shape[0], w.xm.shape[0]
        self.Ns = w.ts.shape[0] * w.rule_n ** 2
        self._P = None

    def _problem(self, xs, xm):
        w = self.w
        return oracle.Problem(xs.detach().cpu().numpy(), w.ts, xm.detach().cpu().numpy(), w.tm, w.rule_n,
                              w.kappa, w.dhat, w.delta_T, None, w.xs_rest)

    def broadphase(self, xs, xm):
        self._P = self._problem(xs, xm)
        self._M = oracle.narrow(self._P).M

    def assemble(self, xs, xm, delta_gap=None, grad=True, hessian=False):
        dg = None if delta_gap is None else delta_gap.detach().cpu().numpy()
        A = oracle.assemble(self._P, self._M, delta_gap=dg, kinematic=self.kinematic, hessian=False)
        self._A = A
        g = A.grad[:self.Vs] if self.kinematic else A.grad
        return SimpleNamespace(energy=torch.tensor([A.energy], dtype=torch.float64),
                               grad=torch.tensor(g, dtype=torch.float64), hessian=None)

    def sample_results(self):
        return dict(c1=torch.tensor(self._A.c1), c2=torch.tensor(self._A.c2),
                    M=torch.tensor(self._M), p=torch.tensor(self._A.press))

    def hvp(self, vx, vd=None):
        v = vx.detach().cpu().numpy()
        if self.kinematic:
            v = np.concatenate([v, np.zeros((self.Vm, 3))])
        ox, od = oracle.hvp(self._P, self._M, self._A.c2, v,
                            None if vd is None else vd.detach().cpu().numpy())
        if self.kinematic:
            ox = ox[:self.Vs]
        return torch.tensor(ox), torch.tensor(od)
