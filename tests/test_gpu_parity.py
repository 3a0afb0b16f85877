"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (float32 path): energy 1e-5 relative; gradient and BSR Hessian
1e-4 relative (Frobenius); step bound never above the oracle's and within
1e-3 of it; selection bit-exact outside the oracle's ambiguity band.  The
float64 path must agree to 1e-10 (same definition, different rounding).
"""
import numpy as np
import pytest

from gen import meshes, workloads
from gpu_helpers import bsr_rel_error, make_ctx, need_gpu, rel_fro, run_gpu, run_oracle, to_dev

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _check(w, dtype, tol_e, tol_g, tol_h, ccd=True, min_active=1):
    need_gpu()
    G = run_gpu(w, dtype, ccd=ccd)
    assert G["status"].code == 0, G["status"].code
    O = run_oracle(w, G["M"], ccd=ccd)
    nr, A = O["nr"], O["A"]
    ok = ~O["flagged"]
    # selection
    assert np.array_equal(G["M"][ok], nr.M[ok]), int((G["M"][ok] != nr.M[ok]).sum())
    act = G["M"] >= 0
    assert act.sum() >= min_active
    assert int(G["status"].n_active) == int(act.sum())
    # sample weights, gaps, barycentrics, coefficients
    wk = (2.0 * oracle_area(O) [:, None] * O["P"].rule[None, :, 2]).ravel()
    assert np.max(np.abs(G["w"] - wk)) <= 1e-6 * wk.max()
    a = act & ok
    gap_ref = np.array([_gap(O, k) for k in np.nonzero(a)[0][:4000]])
    idx = np.nonzero(a)[0][:4000]
    assert np.max(np.abs(G["g"][idx] - gap_ref)) <= 1e-6 * w.dhat
    assert np.max(np.abs(G["c1"] - A.c1)) <= tol_g * np.abs(A.c1).max()
    assert np.max(np.abs(G["c2"] - A.c2)) <= tol_h * np.abs(A.c2).max()
    assert np.max(np.abs(G["p"] - A.press)) <= tol_g * np.abs(A.press).max()
    # energy, gradient, Hessian
    assert abs(G["energy"][0] / A.energy - 1) <= tol_e, (G["energy"][0], A.energy)
    assert rel_fro(G["grad"], A.grad) <= tol_g
    assert bsr_rel_error(G["row_ptr"], G["col"], G["val"], A.row_ptr, A.col, A.val) <= tol_h
    # rows of the BSR: sorted, unique columns
    rp, col = G["row_ptr"], G["col"]
    for r in range(len(rp) - 1):
        c = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(c) > 0)
    # contact pairs: the distinct (slave triangle, master triangle) of the
    # active samples, from the oracle's selection (the HIP path's choice
    # only on the flagged samples)
    T, Mp = (t.cpu().numpy() for t in G["ctx"].pairs())
    nq = w.rule_n ** 2
    ka = np.nonzero(O["M"] >= 0)[0]
    ref = {(int(k // nq), int(O["M"][k])) for k in ka}
    got = list(zip(T.tolist(), Mp.tolist()))
    assert len(got) == len(set(got)) == int(G["status"].n_pairs)
    assert set(got) == ref
    if ccd:
        sb = O["sb"]
        ag = G["alpha"]
        assert ag <= sb.alpha, (ag, sb.alpha)
        assert (sb.alpha - ag) / sb.alpha <= 1e-3, (ag, sb.alpha)
        check_swept_count(O["P"], w, int(G["ccd_status"].n_swept))
    return G, O


# Float32 swept boxes: every bound is widened outward by 4e-7 of its
# magnitude, and the point's start is formed with a few roundings of the
# scene's coordinates (|x| <= 2e-2 m here, so each rounding is below 1e-9 m).
# The oracle's count with boxes shrunk and grown by a margin that covers
# both brackets the float count.
SWEPT_REL, SWEPT_ABS = 1e-6, 2e-9


def check_swept_count(P, w, n_gpu):
    """The step bound's swept (sample point, master triangle) pair count
    lies between the oracle's counts for boxes shrunk and grown by the float
    margin (the definition: boxes over the linear motion overlap), and that
    bracket is narrow."""
    import oracle
    lo = oracle.swept_count(P, w.dxs, w.dxm, -SWEPT_REL, -SWEPT_ABS)
    hi = oracle.swept_count(P, w.dxs, w.dxm, SWEPT_REL, SWEPT_ABS)
    exact = oracle.swept_count(P, w.dxs, w.dxm)
    assert lo <= exact <= hi
    assert lo <= n_gpu <= hi, (lo, n_gpu, hi)
    assert hi - lo <= max(2, 2e-3 * exact), (lo, hi)


def oracle_area(O):
    import oracle
    return oracle.rest_area(O["P"].xs_rest, O["P"].ts)


def _gap(O, k):
    import oracle
    return oracle.sample_geom(O["P"], int(k), int(O["M"][k]))[0]


def test_small_indent_fp32():
    _check(workloads.small_indent(), torch.float32, 1e-5, 1e-4, 1e-4, min_active=300)


def test_small_indent_fp64():
    w = workloads.small_indent(fp32=False)
    need_gpu()
    G = run_gpu(w, torch.float64)
    O = run_oracle(w, G["M"])
    A = O["A"]
    assert np.array_equal(G["M"], O["nr"].M)
    assert abs(G["energy"][0] / A.energy - 1) <= 1e-10
    assert rel_fro(G["grad"], A.grad) <= 1e-10
    assert bsr_rel_error(G["row_ptr"], G["col"], G["val"], A.row_ptr, A.col, A.val) <= 1e-10
    assert G["alpha"] <= O["sb"].alpha and (O["sb"].alpha - G["alpha"]) / O["sb"].alpha <= 1e-3
    check_swept_count(O["P"], w, int(G["ccd_status"].n_swept))


def test_small_indent_face_weight_fp32():
    _check(workloads.small_indent(delta_T=0.05), torch.float32, 1e-5, 1e-4, 1e-4, min_active=300)


@pytest.mark.parametrize("rule_n", [1, 3])
def test_ragged_rules(rule_n):
    # 9 samples per triangle: 7 triangles per wave (one idle lane), ragged tail
    w = workloads.small_indent()
    w.rule_n = rule_n
    _check(w, torch.float32, 1e-5, 1e-4, 1e-4, min_active=50)


def test_large_indent_sphere_full_size():
    _check(workloads.large_indent(), torch.float32, 1e-5, 1e-4, 1e-4, min_active=50000)


def test_large_indent_letter_full_size():
    _check(workloads.large_indent(seed=22, indenter="letter"), torch.float32, 1e-5, 1e-4, 1e-4,
           min_active=50000)


def test_flat_punch_uniform_pressure_fp32():
    need_gpu()
    g0 = 3e-4
    w = workloads.flat_punch(gap=g0, n_pad=16, n_punch=7, fp32=True)
    G = run_gpu(w, torch.float32, ccd=False)
    import oracle
    pk = -w.kappa * oracle.barrier_d1(g0, w.dhat)
    assert np.all(G["M"] >= 0)
    assert np.max(np.abs(G["p"] / pk - 1)) <= 1e-5
    Fz = G["grad"][w.xs.shape[0]:, 2].sum()
    assert abs(Fz / (w.kappa * oracle.barrier_d1(g0, w.dhat) * 1e-4) - 1) <= 1e-5


def test_zero_beyond_dhat_bitwise():
    need_gpu()
    w = workloads.flat_punch(gap=1.5e-3, fp32=True)
    G = run_gpu(w, torch.float32)
    assert np.all(G["M"] < 0)
    assert G["energy"][0] == 0.0
    assert np.all(G["grad"] == 0.0)
    assert G["row_ptr"][-1] == 0
    assert G["alpha"] == 1.0 or G["alpha"] > 0


def test_penetration_reported():
    need_gpu()
    from paper_2605_24339_amd import GMCPError
    import oracle
    w = workloads.flat_punch(gap=-1e-4, fp32=True)
    with pytest.raises(GMCPError) as e:
        run_gpu(w, torch.float32, ccd=False)
    P = workloads.to_problem(w)
    with pytest.raises(oracle.OracleError) as eo:
        oracle.narrow(P)
    assert e.value.code == 3 and e.value.index == eo.value.index


def test_deterministic_bitwise():
    need_gpu()
    w = workloads.large_indent(pad_n=64, rule_n=3)
    G1 = run_gpu(w, torch.float32)
    ctx = G1["ctx"]
    xs, xm = G1["xs"], G1["xm"]
    ctx.broadphase(xs, xm)
    A = ctx.assemble(xs, xm)
    assert np.array_equal(A.energy.double().cpu().numpy(), G1["energy"])
    assert np.array_equal(A.grad.double().cpu().numpy(), G1["grad"])
    assert np.array_equal(A.hessian.col.cpu().numpy(), G1["col"])
    assert np.array_equal(A.hessian.val.double().cpu().numpy(), G1["val"])
    a2 = ctx.ccd_step(xs, xm, to_dev(w.dxs, torch.float32), to_dev(w.dxm, torch.float32))
    assert float(a2[0].item()) == G1["alpha"]


def test_candidates_cover_selection():
    need_gpu()
    w = workloads.large_indent(seed=22, indenter="letter", pad_n=64, rule_n=2)
    G = run_gpu(w, torch.float32, ccd=False)
    off, cand = G["ctx"].candidates()
    off, cand = off.cpu().numpy(), cand.cpu().numpy()
    O = run_oracle(w, G["M"], ccd=False)
    nq = w.rule_n ** 2
    for k in np.nonzero(O["nr"].M >= 0)[0]:
        T = k // nq
        lst = cand[off[T]:off[T + 1]]
        assert O["nr"].M[k] in lst
        assert np.all(np.diff(lst) > 0)


def test_hvp_matches_bsr():
    need_gpu()
    w = workloads.small_indent()
    G = run_gpu(w, torch.float32, ccd=False)
    ctx = G["ctx"]
    V = ctx.V
    rng = np.random.default_rng(3)
    v = rng.normal(size=(V, 3))
    vd = rng.normal(size=ctx.Ns) * 1e-4
    ox, od = ctx.hvp(to_dev(v, torch.float32), to_dev(vd, torch.float32))
    import oracle
    O = run_oracle(w, G["M"], ccd=False)
    rx, rd = oracle.hvp(O["P"], O["M"], O["A"].c2, v, vd)
    assert rel_fro(ox.double().cpu().numpy(), rx) <= 1e-4
    assert rel_fro(od.double().cpu().numpy(), rd) <= 1e-4


def test_batched_environments_match_single():
    need_gpu()
    from paper_2605_24339_amd import Context
    ws = [workloads.small_indent(seed=s) for s in (1, 5, 9)]
    ws[1].rule_n = 3
    ws[2].rule_n = 4
    xs = np.concatenate([w.xs for w in ws])
    xm = np.concatenate([w.xm for w in ws])
    vo = np.cumsum([0] + [w.xs.shape[0] for w in ws])
    to = np.cumsum([0] + [w.ts.shape[0] for w in ws])
    mvo = np.cumsum([0] + [w.xm.shape[0] for w in ws])
    mto = np.cumsum([0] + [w.tm.shape[0] for w in ws])
    ts = np.concatenate([w.ts + vo[i] for i, w in enumerate(ws)])
    tm = np.concatenate([w.tm + mvo[i] for i, w in enumerate(ws)])
    ctx = Context(ts, tm, vo, to, mvo, mto, [w.rule_n for w in ws], [w.kappa for w in ws],
                  [w.dhat for w in ws], [w.delta_T for w in ws], dtype=torch.float32)
    X, XM = to_dev(xs, torch.float32), to_dev(xm, torch.float32)
    ctx.build_samples(X)
    ctx.broadphase(X, XM)
    A = ctx.assemble(X, XM)
    alpha = ctx.ccd_step(X, XM, to_dev(np.concatenate([w.dxs for w in ws]), torch.float32),
                         to_dev(np.concatenate([w.dxm for w in ws]), torch.float32))
    E = A.energy.double().cpu().numpy()
    al = alpha.double().cpu().numpy()
    for i, w in enumerate(ws):
        G = run_gpu(w, torch.float32)
        assert abs(E[i] / G["energy"][0] - 1) <= 1e-6
        assert al[i] == G["alpha"]
        gi = A.grad.double().cpu().numpy()[vo[i]:vo[i + 1]]
        assert rel_fro(gi, G["grad"][:w.xs.shape[0]]) <= 1e-6


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_reference_gaps_and_gap_offsets(dtype):
    """Per-sample support radius eps_k = min(0.9 g_ref_k, dhat) (Eq.
    (adaptive_eps)) from caller-supplied reference gaps, plus per-sample gap
    offsets added after selection; selection, energy, gradient and Hessian
    against the oracle given the same arrays."""
    need_gpu()
    import oracle
    fp32 = dtype == "f32"
    tdt = torch.float32 if fp32 else torch.float64
    w = workloads.small_indent(fp32=fp32)
    rng = np.random.default_rng(8)
    Ns = w.ts.shape[0] * w.rule_n ** 2
    g_ref = rng.uniform(0.2, 2.0, size=Ns) * w.dhat
    dgap = rng.uniform(0.0, 1e-6, size=Ns)
    if fp32:
        g_ref = g_ref.astype(np.float32).astype(np.float64)
        dgap = dgap.astype(np.float32).astype(np.float64)
    ctx = make_ctx(w, tdt)
    xs, xm = to_dev(w.xs, tdt), to_dev(w.xm, tdt)
    ctx.build_samples(to_dev(w.xs_rest, tdt))
    ctx.broadphase(xs, xm)
    A = ctx.assemble(xs, xm, g_ref=to_dev(g_ref, tdt), delta_gap=to_dev(dgap, tdt))
    Mg = ctx.sample_results()["M"].cpu().numpy()
    P = oracle.Problem(w.xs, w.ts, w.xm, w.tm, w.rule_n, w.kappa, w.dhat, w.delta_T, g_ref, w.xs_rest)
    nr = oracle.narrow(P)
    M = nr.M.copy()
    fl = nr.flags != 0
    M[fl] = Mg[fl]
    assert np.array_equal(Mg[~fl], nr.M[~fl])
    # the reference gaps removed some of the plain run's contacts
    plain = oracle.narrow(oracle.Problem(w.xs, w.ts, w.xm, w.tm, w.rule_n, w.kappa, w.dhat, w.delta_T, None,
                                         w.xs_rest))
    assert (nr.M >= 0).sum() < (plain.M >= 0).sum() and (nr.M >= 0).sum() > 100
    O = oracle.assemble(P, M, delta_gap=dgap, project=False)
    te, tg = (1e-5, 1e-4) if fp32 else (1e-10, 1e-10)
    assert abs(float(A.energy.double().sum().item()) / O.energy - 1) <= te
    assert rel_fro(A.grad.double().cpu().numpy(), O.grad) <= tg
    H = A.hessian
    assert bsr_rel_error(H.row_ptr.cpu().numpy(), H.col.cpu().numpy(), H.val.double().cpu().numpy(), O.row_ptr,
                         O.col, O.val) <= tg


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_frozen_energy_matches_oracle(dtype):
    """gmcp_energy_frozen: at the assembly point it is the assembled energy;
    at displaced positions it matches the oracle's frozen-sample energy
    evaluated on the same selection."""
    need_gpu()
    import oracle
    fp32 = dtype == "f32"
    tdt = torch.float32 if fp32 else torch.float64
    w = workloads.small_indent(fp32=fp32)
    G = run_gpu(w, tdt, ccd=False)
    ctx = G["ctx"]
    tol = 1e-5 if fp32 else 1e-10
    e0 = float(ctx.energy_frozen(G["xs"], G["xm"]).double().sum().item())
    assert abs(e0 / G["energy"].sum() - 1) <= tol
    rng = np.random.default_rng(9)
    xs1 = w.xs + rng.uniform(-2e-6, 2e-6, size=w.xs.shape)
    xm1 = w.xm + rng.uniform(-2e-6, 2e-6, size=w.xm.shape)
    if fp32:
        xs1, xm1 = xs1.astype(np.float32).astype(np.float64), xm1.astype(np.float32).astype(np.float64)
    e1 = float(ctx.energy_frozen(to_dev(xs1, tdt), to_dev(xm1, tdt)).double().sum().item())
    # the oracle's own selection and barycentrics; on the samples it flags as
    # ambiguous it takes the HIP path's master triangle and computes their
    # barycentrics itself
    O = run_oracle(w, G["M"], ccd=False)
    P, M = O["P"], O["M"]
    bm = O["nr"].bm.copy()
    for k in np.nonzero(O["flagged"] & (M >= 0))[0]:
        bm[k] = oracle.sample_geom(P, int(k), int(M[k]))[1]
    ref = oracle.frozen_energy(P, M, bm, xs1, xm1)
    assert abs(e1 / ref - 1) <= (1e-4 if fp32 else 1e-10)
    assert abs(e1 / e0 - 1) > 1e-4        # the displacement changed the energy
