"""Differentiable GMCP: the autograd wrapper's backward (force) and double
backward (HVP) against finite differences and the oracle's closed-form
pressure-loss gradient.

CPU tests drive the wrapper with an oracle-backed stand-in backend (FP64):
gradcheck / gradgradcheck in the gap offsets (exact: the selection does not
depend on them), and the pressure-loss gradient in x against the oracle's
closed form (itself pinned by finite differences).  The GPU test runs the
product backend at full size (pressure-map workload, minimum gap 100 um)
and compares with the oracle to 1e-4.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from gen import workloads  # noqa: E402
from oracle_backend import OracleBackend  # noqa: E402
from paper_2605_24339_amd.autograd import gmcp_energy, pressure_map  # noqa: E402


def _small():
    w = workloads.flat_punch(gap=2e-4, n_pad=4, n_punch=3)
    return w


def test_energy_backward_in_gap_offsets_gradcheck():
    w = _small()
    be = OracleBackend(w)
    xs = torch.tensor(w.xs)
    xm = torch.tensor(w.xm)
    d0 = torch.tensor(np.random.default_rng(1).uniform(-2e-5, 2e-5, be.Ns), requires_grad=True)
    f = lambda d: gmcp_energy(be, xs, xm, d) * 1e6
    assert torch.autograd.gradcheck(f, (d0,), eps=1e-9, atol=1e-6, rtol=1e-5)
    assert torch.autograd.gradgradcheck(f, (d0,), eps=1e-9, atol=1e-5, rtol=1e-4)


def test_pressure_loss_gradient_matches_oracle_closed_form():
    w = workloads.small_indent(fp32=False)
    be = OracleBackend(w)
    P = workloads.to_problem(w)
    nr = oracle.narrow(P)
    rng = np.random.default_rng(2)
    ptarget = rng.uniform(0, 50, size=be.Ns)
    wts = torch.tensor(oracle.weights(P))
    xs = torch.tensor(w.xs, requires_grad=True)
    xm = torch.tensor(w.xm, requires_grad=True)
    delta = torch.zeros(be.Ns, dtype=torch.float64, requires_grad=True)
    p = pressure_map(be, xs, xm, delta, wts)
    L = 0.5 * ((p - torch.tensor(ptarget)) ** 2).sum()
    L.backward()
    Lr, dLdx, dLdd = oracle.pressure_loss(P, nr.M, ptarget)
    assert abs(L.item() / Lr - 1) < 1e-12
    g = np.concatenate([xs.grad.numpy(), xm.grad.numpy()])
    assert np.linalg.norm(g - dLdx) <= 1e-10 * np.linalg.norm(dLdx)
    assert np.linalg.norm(delta.grad.numpy() - dLdd) <= 1e-10 * np.linalg.norm(dLdd)


@pytest.mark.gpu
def test_pressure_loss_gradient_gpu_full_size():
    from gpu_helpers import make_ctx, need_gpu, to_dev
    need_gpu()
    w = workloads.large_indent(g_min=100e-6)
    ctx = make_ctx(w, torch.float32)
    xs = to_dev(w.xs, torch.float32).requires_grad_(True)
    xm = to_dev(w.xm, torch.float32).requires_grad_(True)
    wts = ctx.build_samples(xs.detach(), weights=True)
    P = workloads.to_problem(w)
    # target: the oracle's map at an offset indenter pose, with 1 % noise
    Pt = P.with_positions(xm=P.xm + np.array([1e-4, -1e-4, -5e-5]))
    nt = oracle.narrow(Pt)
    At = oracle.assemble(Pt, nt.M, hessian=False)
    rng = np.random.default_rng(4)
    ptarget = At.press * (1 + 0.01 * rng.normal(size=P.Ns))
    delta = torch.zeros(ctx.Ns, dtype=torch.float32, device="cuda", requires_grad=True)
    p = pressure_map(ctx, xs, xm, delta, wts)
    L = 0.5 * ((p - to_dev(ptarget, torch.float32)) ** 2).sum()
    L.backward()
    M = ctx.sample_results()["M"].cpu().numpy()
    nr = oracle.narrow(P)
    Mx = nr.M.copy()
    Mx[nr.flags != 0] = M[nr.flags != 0]
    Lr, dLdx, dLdd = oracle.pressure_loss(P, Mx, ptarget)
    assert abs(L.item() / Lr - 1) < 1e-4
    g = np.concatenate([xs.grad.double().cpu().numpy(), xm.grad.double().cpu().numpy()])
    assert np.linalg.norm(g - dLdx) <= 1e-4 * np.linalg.norm(dLdx)
    assert np.linalg.norm(delta.grad.double().cpu().numpy() - dLdd) <= 1e-4 * np.linalg.norm(dLdd)
