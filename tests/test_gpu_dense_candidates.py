"""Coarse slave triangles over a finely meshed master: the kernels' paths for
many master triangles per slave triangle.

* Clipped mortar samples (Sec. 4.1 face samples) with more than 64
  candidates per slave triangle, so that the mortar kernel takes its pairs
  in several chunks of 64. The energy is checked against the closed form
  kappa B(g0) A for a uniform gap. The energy, gradient and BSR Hessian are
  checked against the oracle. A repeated assembly must be bitwise equal.
* The step bound (Eq. (ccd) + additive CCD) when a slave triangle's swept
  box meets more master triangles than its LDS list holds (256 for the 4x4
  rule). The kernel then walks each point's own cells. Alpha must not
  exceed the oracle's and must be within 1e-3 of it.
"""
import numpy as np
import pytest

import oracle
from gen import workloads
from gpu_helpers import bsr_rel_error, need_gpu, rel_fro, run_gpu, run_oracle, to_dev
from oracle import mortar as om

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _oracle_bsr(blocks, V):
    keys = sorted(blocks)
    row_ptr = np.zeros(V + 1, np.int64)
    for (i, _) in keys:
        row_ptr[i + 1] += 1
    row_ptr = np.cumsum(row_ptr)
    col = np.array([j for (_, j) in keys], np.int64)
    val = np.array([blocks[k] for k in keys]).reshape(-1, 9) if keys else np.zeros((0, 9))
    return row_ptr, col, val


def test_mortar_many_candidates_per_triangle():
    need_gpu()
    from paper_2605_24339_amd import Context
    # 8 slave triangles (5 mm legs) under a 24 x 24 punch (0.58 mm cells)
    w = workloads.flat_punch(n_pad=2, n_punch=24, gap=3e-4, punch_length=1.4e-2, rule_n=4, fp32=True)
    ctx = Context.single(w.ts, w.tm, w.xs.shape[0], w.xm.shape[0], rule_n=w.rule_n, kappa=w.kappa, dhat=w.dhat,
                         delta_T=w.delta_T, dtype=torch.float32, mortar=True)
    xs, xm = to_dev(w.xs, torch.float32), to_dev(w.xm, torch.float32)
    ctx.build_samples(to_dev(w.xs_rest, torch.float32))
    ctx.broadphase(xs, xm)
    A = ctx.assemble(xs, xm)
    st = ctx.status()
    assert st.code == 0, st.code
    off, _ = ctx.candidates()
    counts = np.diff(off.cpu().numpy())
    assert counts.max() > 64, counts          # more than one chunk of 64 pairs
    assert counts.max() <= 512
    # uniform gap under the whole pad: E = kappa B(g0) A_pad
    ref = w.kappa * oracle.barrier(3e-4, w.dhat) * 1e-4
    E = float(A.energy.double().sum())
    assert abs(E / ref - 1) <= 1e-5
    # against the oracle's clipped samples
    P = workloads.to_problem(w)
    O = om.assemble(P, om.samples(P))
    assert abs(int(st.n_active) - len(O.active)) <= 2
    assert abs(E / O.energy - 1) <= 1e-5
    assert rel_fro(A.grad.double().cpu().numpy(), O.grad) <= 1e-4
    rp, col, val = _oracle_bsr(O.blocks, P.Vs + P.Vm)
    H = A.hessian
    assert bsr_rel_error(H.row_ptr.cpu().numpy(), H.col.cpu().numpy(), H.val.double().cpu().numpy().reshape(-1, 9),
                         rp, col, val) <= 1e-4
    # the same inputs give the same bits
    e1, g1, v1 = A.energy.clone(), A.grad.clone(), A.hessian.val.clone()
    ctx.broadphase(xs, xm)
    A2 = ctx.assemble(xs, xm)
    assert torch.equal(e1, A2.energy) and torch.equal(g1, A2.grad) and torch.equal(v1, A2.hessian.val)


def test_step_bound_when_the_swept_list_overflows():
    need_gpu()
    # 32 slave triangles (2.5 mm legs, 16 points each; at most 200 candidates
    # each, within the broad phase's 512) moving up into a 48 x 48 punch
    # (0.29 mm cells) and 3 mm sideways
    w = workloads.flat_punch(n_pad=4, n_punch=48, gap=3e-4, punch_length=1.4e-2, rule_n=4, fp32=True)
    rng = np.random.default_rng(7)
    w.dxs = np.zeros_like(w.xs)
    w.dxs[:, 2] = 6e-4 * (1 + 0.1 * rng.random(w.xs.shape[0]))
    w.dxs[:, 0] = 3e-3
    w.dxm = np.zeros_like(w.xm)
    # the swept boxes of the slave triangles meet more master triangles than
    # a list holds (256 with four triangles per tile)
    lo_m = np.minimum.reduce([w.xm[w.tm[:, k]] for k in range(3)])
    hi_m = np.maximum.reduce([w.xm[w.tm[:, k]] for k in range(3)])
    most = 0
    for t in w.ts:
        p = np.concatenate([w.xs[t], w.xs[t] + w.dxs[t]])
        lo, hi = p.min(0), p.max(0)
        meet = np.all((lo_m <= hi) & (hi_m >= lo), axis=1)
        most = max(most, int(meet.sum()))
    assert most > 256, most
    G = run_gpu(w, torch.float32)
    assert G["ccd_status"].code == 0
    O = run_oracle(w, G["M"])
    sb = O["sb"]
    assert sb.alpha < 1.0
    assert G["alpha"] <= sb.alpha, (G["alpha"], sb.alpha)
    assert (sb.alpha - G["alpha"]) / sb.alpha <= 1e-3, (G["alpha"], sb.alpha)
