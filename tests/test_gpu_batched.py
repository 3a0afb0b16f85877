"""Batched environments and graph capture on the GPU.

* A captured step replayed several times, with eager library work and
  synchronisations between replays, equals the eager step bit for bit on
  every replay, also after the inputs change in place.
* The step bound split in two calls (swept part on a second stream,
  overlapping the broad phase and assembly) equals the one-call step bound
  bit for bit; the second call without the first is rejected.
* The 256-environment batch (uneven pads, rules, indenters) runs in one
  launch sequence; sampled environments (always the smallest and the
  largest) match the FP64 oracle (energy, gradient, BSR Hessian, step
  bound, selection outside the ambiguity band).
"""
import numpy as np
import pytest

import oracle
from gen import workloads
from gpu_helpers import need_gpu, rel_fro, to_dev

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _batch_ctx(B, dtype=torch.float32, cell=None):
    from paper_2605_24339_amd import Context
    E = len(B.envs)
    return Context(B.ts, B.tm, B.slave_v_off, B.slave_t_off, B.master_v_off, B.master_t_off, B.rule_n,
                   [w.kappa for w in B.envs], [w.dhat for w in B.envs], [w.delta_T for w in B.envs],
                   cell if cell is not None else [0.0] * E, dtype=dtype)


def _snapshot(ctx, nnzb):
    return (ctx.energy.clone(), ctx.grad.clone(), ctx.row_ptr.clone(), ctx.col[:nnzb].clone(),
            ctx.val[:nnzb].clone(), ctx.alpha.clone())


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def test_graph_replay_matches_eager():
    need_gpu()
    w = workloads.small_indent()
    from gpu_helpers import make_ctx
    ctx = make_ctx(w, torch.float32)
    xs, xm = to_dev(w.xs, torch.float32), to_dev(w.xm, torch.float32)
    dxs, dxm = to_dev(w.dxs, torch.float32), to_dev(w.dxm, torch.float32)
    ctx.build_samples(xs)
    g = ctx.capture(xs, xm, dxs, dxm)
    ctx.step(xs, xm, dxs, dxm, check=True)
    nnzb = int(ctx.status().nnzb)
    eager = _snapshot(ctx, nnzb)
    for r in range(4):
        ctx.val.zero_()
        ctx.energy.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert int(ctx.status().nnzb) == nnzb
        assert _same(_snapshot(ctx, nnzb), eager), f"replay {r}"
        ctx.step(xs, xm, dxs, dxm)  # eager work between replays
        torch.cuda.synchronize()
    # new positions written in place (indenter moved sideways and up, away
    # from the pad): replay == eager on the new input
    xm.add_(torch.tensor([2e-5, -1e-5, 3e-5], device="cuda"))
    g.replay()
    torch.cuda.synchronize()
    nn2 = int(ctx.status().nnzb)
    rep = _snapshot(ctx, nn2)
    ctx.step(xs, xm, dxs, dxm, check=True)
    assert _same(_snapshot(ctx, nn2), rep)


def test_overlapped_step_bound_matches_sequential():
    need_gpu()
    from paper_2605_24339_amd import GMCPError, _native
    from gpu_helpers import make_ctx
    w = workloads.large_indent()
    ctx = make_ctx(w, torch.float32)
    xs, xm = to_dev(w.xs, torch.float32), to_dev(w.xm, torch.float32)
    dxs, dxm = to_dev(w.dxs, torch.float32), to_dev(w.dxm, torch.float32)
    ctx.build_samples(xs)
    ctx.step(xs, xm, dxs, dxm, check=True)          # sequential, one-call step bound
    torch.cuda.synchronize()
    nnzb = int(ctx.status().nnzb)
    seq = _snapshot(ctx, nnzb)
    n_swept = int(ctx.status().n_swept)
    for _ in range(3):
        ctx.alpha.fill_(-1.0)
        ctx.step(xs, xm, dxs, dxm)                  # overlapped: swept part on the side stream
        torch.cuda.synchronize()
        st = ctx.status()
        assert st.code == 0 and int(st.nnzb) == nnzb and int(st.n_swept) == n_swept
        assert _same(_snapshot(ctx, nnzb), seq)
    with pytest.raises(GMCPError) as e:             # finish without a swept part
        ctx.ccd_finish(dxs, dxm)
    assert e.value.code == _native.GMCP_E_ARG


def _env_bsr(B, e, row_ptr, col, val):
    """Environment e's rows of the batch's BSR (global numbering: every
    slave vertex, then every master vertex) in the environment's own
    numbering (its slave vertices, then its master vertices)."""
    Vs = B.xs.shape[0]
    s0, s1 = B.slave_v_off[e], B.slave_v_off[e + 1]
    m0, m1 = B.master_v_off[e], B.master_v_off[e + 1]
    rows = list(range(s0, s1)) + list(range(Vs + m0, Vs + m1))
    ns = s1 - s0

    def local(c):
        c = c.astype(np.int64)
        out = np.where(c < Vs, c - s0, c - Vs - m0 + ns)
        ok = np.where(c < Vs, (c >= s0) & (c < s1), (c >= Vs + m0) & (c < Vs + m1))
        assert ok.all(), "a block couples two environments"
        return out

    rp, cl, vl = [0], [], []
    for r in rows:
        a, b = row_ptr[r], row_ptr[r + 1]
        cl.append(local(col[a:b]))
        vl.append(val[a:b])
        rp.append(rp[-1] + (b - a))
    return np.array(rp), np.concatenate(cl), np.concatenate(vl)


def test_batch_256_envs_sampled_parity():
    """Sampled environments of the batch, always including the ones with
    the fewest and the most samples: selection, energy, gradient, BSR
    Hessian (blocks of the environment's own rows, no block coupling two
    environments) and step bound against the oracle."""
    need_gpu()
    from gpu_helpers import bsr_rel_error
    B = workloads.batched()
    ctx = _batch_ctx(B)
    X, XM = to_dev(B.xs, torch.float32), to_dev(B.xm, torch.float32)
    ctx.build_samples(X)
    A, alpha = ctx.step(X, XM, to_dev(B.dxs, torch.float32), to_dev(B.dxm, torch.float32), check=True)
    st = ctx.status()
    assert st.code == 0
    E = A.energy.double().cpu().numpy()
    al = alpha.double().cpu().numpy()
    grad = A.grad.double().cpu().numpy()
    H = A.hessian
    row_ptr, col, val = H.row_ptr.cpu().numpy(), H.col.cpu().numpy(), H.val.double().cpu().numpy()
    M = ctx.sample_results()["M"].cpu().numpy()
    samp0 = np.cumsum([0] + [w.n_samples for w in B.envs])
    ns = np.array([w.n_samples for w in B.envs])
    rng = np.random.default_rng(0)
    pick = set(rng.choice(len(B.envs), 6, replace=False).tolist()) | {int(ns.argmin()), int(ns.argmax())}
    for e in sorted(pick):
        w = B.envs[e]
        P = workloads.to_problem(w)
        nr = oracle.narrow(P)
        Me = M[samp0[e]:samp0[e + 1]]
        Me = np.where(Me >= 0, Me - B.master_t_off[e], -1)
        ok = nr.flags == 0
        assert np.array_equal(Me[ok], nr.M[ok]), e
        Mx = nr.M.copy()
        Mx[~ok] = Me[~ok]
        Ar = oracle.assemble(P, Mx, project=False)
        if Ar.energy > 0:
            assert abs(E[e] / Ar.energy - 1) <= 1e-5, e
        else:
            assert E[e] == 0.0
        gs = grad[B.slave_v_off[e]:B.slave_v_off[e + 1]]
        gm = grad[B.xs.shape[0] + B.master_v_off[e]:B.xs.shape[0] + B.master_v_off[e + 1]]
        assert rel_fro(np.concatenate([gs, gm]), Ar.grad) <= 1e-4, e
        rp, cl, vl = _env_bsr(B, e, row_ptr, col, val)
        assert bsr_rel_error(rp, cl, vl, Ar.row_ptr, Ar.col, Ar.val) <= 1e-4, e
        sb = oracle.ccd_step(P, Mx, w.dxs, w.dxm)
        assert al[e] <= sb.alpha and (sb.alpha - al[e]) / sb.alpha <= 1e-3, (e, al[e], sb.alpha)
