"""BSR rows with more distinct columns than the row kernels' first tables
hold (Sec. 4.2 Hessian scatter).

A fine pad (48 x 48 quads, one sample per triangle) under a punch of two
master triangles that covers it: each of the punch's four vertices couples
to about 1200-2400 slave vertices, so its BSR row needs the largest table
(4096 slots).  The first assemblies report a capacity error from those rows;
the binding grows the table once, to the row's insertion count (4096
slots), and the grown result must match the oracle, in float and double."""
import numpy as np
import pytest

import oracle
from gen import workloads
from gpu_helpers import bsr_rel_error, make_ctx, need_gpu, rel_fro, to_dev

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_rows_beyond_2048_columns_after_growth(dtype):
    need_gpu()
    fp32 = dtype == "f32"
    tdt = torch.float32 if fp32 else torch.float64
    w = workloads.flat_punch(gap=3e-4, n_pad=48, n_punch=1, rule_n=1, fp32=fp32)
    P = workloads.to_problem(w)
    nr = oracle.narrow(P)
    O = oracle.assemble(P, nr.M, project=False)
    rl = np.diff(O.row_ptr)
    assert rl.max() > 2048 and (rl > 512).sum() == 4
    ctx = make_ctx(w, tdt)
    assert ctx.caps["row_entries"] < 512
    xs, xm = to_dev(w.xs, tdt), to_dev(w.xm, tdt)
    ctx.build_samples(to_dev(w.xs_rest, tdt))
    ctx.broadphase(xs, xm)
    A = ctx.assemble(xs, xm)
    assert ctx.caps["row_entries"] == 4096
    assert ctx.status().code == 0
    M = ctx.sample_results()["M"].cpu().numpy()
    assert np.array_equal(M[nr.flags == 0], nr.M[nr.flags == 0])
    te, tg = (1e-5, 1e-4) if fp32 else (1e-10, 1e-10)
    assert abs(float(A.energy.double().sum()) / O.energy - 1) <= te
    assert rel_fro(A.grad.double().cpu().numpy(), O.grad) <= tg
    H = A.hessian
    rp = H.row_ptr.cpu().numpy()
    assert np.array_equal(np.diff(rp), rl)
    assert bsr_rel_error(rp, H.col.cpu().numpy(), H.val.double().cpu().numpy(), O.row_ptr, O.col, O.val) <= tg
    # a second assembly on the grown context reports no error and repeats bit for bit
    v1 = H.val.clone()
    ctx.broadphase(xs, xm)
    A2 = ctx.assemble(xs, xm)
    assert torch.equal(A2.hessian.val, v1)
