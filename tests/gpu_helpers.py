"""Shared helpers of the GPU parity tests: run a workload through the HIP
library and through the FP64 oracle, and compare what is unique.

Comparison rules
* selection (which master triangle each sample takes) must be bit-exact on
  every sample the oracle does not flag as ambiguous for float32;
* energy, gradient, Hessian and pressures are compared with the oracle run
  on the GPU's assignment for the flagged samples, so only arithmetic is
  measured there;
* BSR blocks are compared on the union of both patterns (a block missing on
  one side counts as zero), as a Frobenius-norm relative error.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2605_24339_amd import _native
    _native.lib()  # raises (fails the test) if the HIP library was not built


def to_dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def make_ctx(w, dtype, **kw):
    from paper_2605_24339_amd import Context
    return Context.single(w.ts, w.tm, w.xs.shape[0], w.xm.shape[0], rule_n=w.rule_n, kappa=w.kappa,
                          dhat=w.dhat, delta_T=w.delta_T, dtype=dtype, **kw)


def run_gpu(w, dtype=None, ccd=True, **kw):
    dtype = dtype or torch.float32
    ctx = make_ctx(w, dtype, **kw)
    xs, xm = to_dev(w.xs, dtype), to_dev(w.xm, dtype)
    wts = ctx.build_samples(to_dev(w.xs_rest, dtype), weights=True)
    ctx.broadphase(xs, xm)
    A = ctx.assemble(xs, xm)
    S = ctx.sample_results()
    out = dict(ctx=ctx, xs=xs, xm=xm, energy=A.energy.double().cpu().numpy(),
               grad=A.grad.double().cpu().numpy(), row_ptr=A.hessian.row_ptr.cpu().numpy(),
               col=A.hessian.col.cpu().numpy(), val=A.hessian.val.double().cpu().numpy(),
               M=S["M"].cpu().numpy(), g=S["g"].double().cpu().numpy(), bm=S["bm"].double().cpu().numpy(),
               c1=S["c1"].double().cpu().numpy(), c2=S["c2"].double().cpu().numpy(),
               p=S["p"].double().cpu().numpy(), w=wts.double().cpu().numpy(), status=ctx.status())
    if ccd:
        a = ctx.ccd_step(xs, xm, to_dev(w.dxs, dtype), to_dev(w.dxm, dtype))
        out["alpha"] = float(a[0].item())
        out["ccd_status"] = ctx.status()
    return out


def run_oracle(w, M_gpu=None, ccd=True, project=False):
    P = oracle.Problem(w.xs, w.ts, w.xm, w.tm, w.rule_n, w.kappa, w.dhat, w.delta_T, None, w.xs_rest)
    nr = oracle.narrow(P)
    M = nr.M.copy()
    flagged = nr.flags != 0
    if M_gpu is not None:
        M[flagged] = M_gpu[flagged]
    A = oracle.assemble(P, M, project=project)
    out = dict(P=P, nr=nr, M=M, flagged=flagged, A=A)
    if ccd:
        out["sb"] = oracle.ccd_step(P, M, w.dxs, w.dxm)
    return out


def bsr_dict(row_ptr, col, val):
    d = {}
    for r in range(len(row_ptr) - 1):
        for j in range(row_ptr[r], row_ptr[r + 1]):
            d[(r, int(col[j]))] = val[j].reshape(3, 3)
    return d


def bsr_rel_error(gpu_rp, gpu_col, gpu_val, ora_rp, ora_col, ora_val):
    G = bsr_dict(gpu_rp, gpu_col, gpu_val)
    O = bsr_dict(ora_rp, ora_col, ora_val)
    keys = set(G) | set(O)
    z = np.zeros((3, 3))
    num = sum(float(np.sum((G.get(k, z) - O.get(k, z)) ** 2)) for k in keys)
    den = sum(float(np.sum(O[k] ** 2)) for k in O)
    return np.sqrt(num / den) if den > 0 else np.sqrt(num)


def rel_fro(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / den if den > 0 else np.linalg.norm(a)
