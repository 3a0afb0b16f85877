#!/usr/bin/env python3
"""Throughput of the GMCP hot path on one MI355X.

One step = one pass of the whole path over the resident input: broad phase,
assembly (selection, barrier, energy, gradient, BSR Hessian) and the step
bound (linearised gap + additive CCD).  Headline workload: the batch of 256
environments of uneven size (pads of 32x32 to 128x128 quads, 2x2 to 4x4
samples per triangle, 980 to 40500-triangle indenters; 35.5 M samples),
float32, captured once into a HIP graph and replayed; the broad-phase cell
size is chosen by the autotuner first.  The single large indentation
(128x128 pad, 524288 samples, 40500-triangle sphere) is measured the same
way beside it.

Algorithmic bytes per step follow the scope's definition: positions,
triangles, rest areas, gradient, BSR values + columns + row pointers and
energies for the assembly; positions and displacements, triangles, the
20-byte active-sample records and the bounds for the step bound.  The
counts they need (active samples, BSR blocks) and the swept-pair count of
the CCD rate are the oracle's (tests/golden/unit_counts.json, written by a
script that calls only the oracle), so neither depends on the HIP path.

Prints one JSON line: samples/s over the timed steps (inputs already in
HBM), per-kernel HIP-event times, the roofline of the dominant kernel and of
the whole step, the same figures for the single large indentation, and the
FP64 oracle's throughput on the host cores (a reported baseline, not the
target).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GMCP samples/s (E+grad+Hess) & CCD pairs/s, % HBM peak; Newton iters learned vs plain"
HBM_PEAK_GBS = 8000.0
# kernels that one profiled stage brackets exactly (candidates for the
# roofline); the additive CCD stage also holds its tile prepass, so it is
# not one of them
KERNEL_STAGES = {"query": "k_query_f32", "cand_move": "k_cand_move", "narrow": "k_narrow_f32",
                 "rows_count": "k_rows<float, 0, false>", "rows_fill": "k_rows<float, 1, false>",
                 "rows_count_heavy": "k_rows<float, 0, true>", "rows_fill_heavy": "k_rows<float, 1, true>",
                 "ccd_linear": "k_ccd_linear<float>"}


# sources of the step's kernels and launches (the traffic counters of a
# kernel are reported only while these are unchanged)
STEP_SOURCES = ("common.h", "util.hip", "broadphase.hip", "assemble.hip", "ccd.hip", "host.cpp")


def src_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2605_24339_amd", "csrc")
    for f in STEP_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def unit_counts(workload: str) -> dict | None:
    """The oracle's counts for a workload (active samples, BSR blocks, swept
    pairs, mesh sizes), if stored and written from the current generator
    and oracle sources."""
    p = os.path.join(ROOT, "tests", "golden", "unit_counts.json")
    if not os.path.exists(p):
        return None
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    try:
        import make_unit_counts as muc
    finally:
        sys.path.pop(0)
    with open(p) as fh:
        d = json.load(fh)
    if d.get("source_hash") != muc.source_hash():
        return None
    return d.get(workload)


def step_bytes(c: dict) -> dict:
    """Algorithmic bytes of one step (float32, 4-byte ids): the assembly
    reads positions, triangles and rest areas and writes the gradient, the
    BSR (3x3 values + column per block, row pointers) and the energies; the
    step bound reads positions and displacements, triangles and the 20-byte
    record of every active sample and writes the bounds."""
    V = c["Vs"] + c["Vm"]
    T = c["Ts"] + c["Tm"]
    b_asm = 12 * V + 12 * T + 4 * c["Ts"] + 12 * V + 40 * c["nnzb"] + 4 * (V + 1) + 4 * c["n_env"]
    b_ccd = 24 * V + 12 * T + 20 * c["active"] + 4 * c["n_env"]
    return {"assembly": int(b_asm), "step_bound": int(b_ccd), "total": int(b_asm + b_ccd),
            "per_sample": (b_asm + b_ccd) / c["samples"]}


def time_replays(g, steps: int, stream) -> float:
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def measure(name, envs, batch, steps, warmup, dev, tune_cache=None, mortar=False, features=None):
    """Autotune, capture, time; per-kernel stage times; roofline of the
    dominant kernel.  features = (kappa_edge, kappa_point, delta_e) adds the
    edge and point samples to the clipped face samples."""
    import numpy as np
    import torch

    from paper_2605_24339_amd import Context, autotune

    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    xs, xm, dxs, dxm = t(batch.xs), t(batch.xm), t(batch.dxs), t(batch.dxm)

    def make(cells):
        fe = {} if features is None else dict(features=True, kappa_edge=[features[0]] * len(envs),
                                              kappa_point=[features[1]] * len(envs),
                                              delta_e=[features[2]] * len(envs))
        return Context(batch.ts, batch.tm, batch.slave_v_off, batch.slave_t_off, batch.master_v_off,
                       batch.master_t_off, [w.rule_n for w in envs], [w.kappa for w in envs],
                       [w.dhat for w in envs], [w.delta_T for w in envs], cells, dtype=torch.float32,
                       device=dev, mortar=mortar, **fe)

    cells, tuning, table = autotune.tune(make, envs, (xs, xm, dxs, dxm), cache=tune_cache if not mortar else None,
                                         scales=autotune.SCALES if not mortar else (0.0,),
                                         shapes=autotune.SHAPES if not mortar else None)
    ctx = make(cells)
    ctx.set_tuning(**tuning)
    ctx.build_samples(xs)
    g = ctx.capture(xs, xm, dxs, dxm)
    stream = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        g.replay()
    ms = time_replays(g, steps, stream)
    st = ctx.status()
    if st.code != 0:
        raise SystemExit(f"{name}: status {st.code} after the timed steps")
    ctx.profile(True)
    for _ in range(max(3, min(steps, 20))):
        ctx.step(xs, xm, dxs, dxm)
    prof = ctx.profile_read()
    ctx.profile(False)
    st = ctx.status()
    stages = {k: v[0] / v[1] for k, v in prof.items() if v[1] > 0}
    Ns = sum(w.n_samples for w in envs)
    gpu = dict(n_env=len(envs), Vs=int(batch.xs.shape[0]), Vm=int(batch.xm.shape[0]), Ts=int(batch.ts.shape[0]),
               Tm=int(batch.tm.shape[0]), samples=int(Ns), active=int(st.n_active), nnzb=int(st.nnzb),
               swept=int(st.n_swept), pairs=int(st.n_pairs), candidates=int(st.n_candidates))
    ora = None if mortar else unit_counts(name)
    counts = ora if ora is not None else gpu
    sb = step_bytes(counts)
    kern = {k: v for k, v in stages.items() if k in KERNEL_STAGES}
    dom = max(kern, key=kern.get)
    traffic = load_traffic(name)
    dom_traffic = traffic.get("kernels", {}).get(KERNEL_STAGES[dom]) if traffic else None
    achieved = sb["total"] / (kern[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": None if dom_traffic is None else round(dom_traffic),
            "kernel": KERNEL_STAGES[dom], "stage": dom, "avg_ms": round(kern[dom], 5),
            "algorithmic_bytes": sb["total"], "bytes_per_sample": round(sb["per_sample"], 3),
            "samples_per_launch": int(Ns)}
    step_gbs = sb["total"] / (ms * 1e-3) / 1e9
    roof_step = {"bound": "hbm", "achieved": round(step_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(step_gbs / HBM_PEAK_GBS, 5),
                 "traffic": None if not traffic else round(traffic["step_bytes"]),
                 "algorithmic_bytes": sb, "ms": round(ms, 5)}
    ccd_ms = stages.get("ccd_linear", 0) + stages.get("ccd_grid", 0) + stages.get("ccd_accd", 0)
    return dict(ms=ms, value=Ns / (ms * 1e-3), samples=Ns, stages={k: round(v, 5) for k, v in stages.items()},
                roofline=roof, roofline_step=roof_step, gpu_counts=gpu, counts=counts,
                counts_source="oracle" if ora is not None else "gpu", ccd_ms=ccd_ms, autotune=table,
                tuning=ctx.tuning(), cells=cells[:4])


def load_traffic(workload: str) -> dict | None:
    """Measured HBM traffic of the workload's kernels (rocprofv3 counters,
    copy-calibrated; profiles/traffic.json), if taken on the current step
    sources: {"kernels": {name: bytes per launch}, "step_bytes": bytes per
    step}."""
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tf):
        return None
    with open(tf) as fh:
        rec = json.load(fh).get(workload)
    if not rec or rec.get("src_hash") != src_hash():
        return None
    return rec


def _event_ms(fn, reps: int) -> float:
    import torch
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def measure_autograd(w, dev, reps: int = 10) -> dict:
    """Differentiable GMCP on the same workload: a pressure-map loss, its
    forward (broad phase + assembly), backward (force kernel) and double
    backward (Hessian-vector product) per iteration."""
    import numpy as np
    import torch

    from paper_2605_24339_amd import Context
    from paper_2605_24339_amd.autograd import pressure_map
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    ctx = Context.single(w.ts, w.tm, w.xs.shape[0], w.xm.shape[0], rule_n=w.rule_n, kappa=w.kappa, dhat=w.dhat,
                         dtype=torch.float32, device=dev)
    xs, xm = t(w.xs).requires_grad_(True), t(w.xm).requires_grad_(True)
    wts = ctx.build_samples(xs.detach(), weights=True)
    target = torch.zeros(ctx.Ns, dtype=torch.float32, device=dev)
    delta = torch.zeros(ctx.Ns, dtype=torch.float32, device=dev, requires_grad=True)

    def it():
        p = pressure_map(ctx, xs, xm, delta, wts)
        L = 0.5 * ((p - target) ** 2).sum()
        L.backward()

    ms = _event_ms(it, reps)
    return {"workload": w.name, "ms_per_iteration": ms, "samples_per_s": ctx.Ns / (ms * 1e-3),
            "what": "pressure-map loss: forward, force backward, HVP double backward, autograd bookkeeping"}


def measure_mlp(dev, batch: int = 65536, reps: int = 20) -> dict:
    """Warm-start MLP: one training step (forward, MSE, backward, Adam) and
    the bf16 matrix-core GEMM of a hidden layer."""
    import torch

    from paper_2605_24339_amd.mlp import MLP, PAD, gemm_bf16
    from paper_2605_24339_amd.warmstart import init_params
    g = torch.Generator(device="cpu").manual_seed(0)
    X = torch.randn(batch, PAD, generator=g).to(dev)
    T = torch.randn(batch, PAD, generator=g).to(dev)
    net = MLP(init_params(0, dev))
    act = torch.empty(batch, 6 * 128, dtype=torch.float32, device=dev)

    def step():
        y, a = net.forward(X, act)
        _, dy = net.mse(y, T)
        net.adam(net.backward(X, a, dy))

    ms = _event_ms(step, reps)
    # fused forward (one launch, activations in registers): inference and
    # the training forward that saves the activations
    Bi = 1 << 18
    Xi = torch.randn(Bi, PAD, generator=g).to(dev)
    Xi[:, 9:] = 0.0
    inf_ms = _event_ms(lambda: net.predict(Xi), reps)
    acti = torch.empty(Bi, 6 * 128, dtype=torch.float32, device=dev)
    fwd_ms = _event_ms(lambda: net.forward(Xi, acti), reps)
    useful = 2 * (9 * 128 + 2 * 128 * 128 + 128 * 3)            # per row, the real network
    executed = 2 * (16 * 128 + 2 * 128 * 128 + 128 * 32)        # per row, padded MFMA tiles
    inf_tf = Bi * useful / (inf_ms * 1e-3) / 1e12
    fused = {"rows": Bi, "inference_ms": inf_ms, "inference_rows_per_s": Bi / (inf_ms * 1e-3),
             "inference_tflops_useful": inf_tf, "inference_tflops_executed": Bi * executed / (inf_ms * 1e-3) / 1e12,
             "mfma_peak_tflops": 2500.0, "frac_mfma_peak_executed": Bi * executed / (inf_ms * 1e-3) / 1e12 / 2500.0,
             "inference_gbs": Bi * 128 / (inf_ms * 1e-3) / 1e9,
             "forward_saving_activations_ms": fwd_ms,
             "forward_saving_activations_gbs": Bi * (128 + 4 * 768) / (fwd_ms * 1e-3) / 1e9,
             "note": "inference reads 64 B and writes 64 B per row; the training forward also writes 3 KiB of "
                     "activations per row (HBM-bound)"}
    flops = 3 * 2 * batch * (PAD * 128 + 2 * 128 * 128 + 128 * PAD)
    Mg, Ng, Kg = 1 << 18, 128, 128
    A = torch.randn(Mg, Kg, generator=g).to(dev)
    B = torch.randn(Kg, Ng, generator=g).to(dev)
    gms = _event_ms(lambda: gemm_bf16(A, B), reps)
    tf = 2 * Mg * Ng * Kg / (gms * 1e-3) / 1e12
    return {"train_rows_per_s": batch / (ms * 1e-3), "train_step_ms": ms, "batch": batch,
            "train_tflops": flops / (ms * 1e-3) / 1e12, "fused_forward": fused,
            "gemm": {"M": Mg, "N": Ng, "K": Kg, "ms": gms, "tflops": tf, "mfma_peak_tflops": 2500.0,
                     "gbs": 4 * (Mg * Kg + Kg * Ng + Mg * Ng) / (gms * 1e-3) / 1e9, "hbm_peak_gbs": HBM_PEAK_GBS,
                     "note": "float32 operands converted to bf16 on load, float32 out: HBM-bound at K = 128"}}


WARMSTART_CHECKPOINT = os.path.join(ROOT, "paper_2605_24339_amd", "data", "warmstart_mlp.npz")


def measure_warmstart(steps: int = 100, seeds=(5045, 5046)) -> dict | None:
    """Newton iterations and assemblies per implicit step to reach the
    1e-6 residual, plain start (x_t + dt v_t) against the learned start
    (the committed network, trained on tap trajectories 5000..5019), on
    held-out tap trajectories of the gel block; both starts pass the same
    step-bound filter, the learned one also the energy safeguard."""
    if not os.path.exists(WARMSTART_CHECKPOINT):
        return None
    from paper_2605_24339_amd import warmstart as W
    net, scaler = W.load_checkpoint(WARMSTART_CHECKPOINT)
    plain, learned = [], []
    t0 = time.perf_counter()
    for sd in seeds:
        sc = W.Scene(sd)
        plain += W.run_trajectory(sc, steps, None, keep=False)
        learned += W.run_trajectory(sc, steps, net, keep=False, scaler=scaler, safeguard=True)
    P, L = W.summarize(plain), W.summarize(learned)
    out = {"workload": "64x64x8-cube gel block (38025 vertices) tapped by a sphere at 10-100 mm/s, dt = 1 ms, "
                       f"held-out trajectories {list(seeds)}, {steps} steps each, residual 1e-6",
           "newton_plain": P["newton"]["mean"], "newton_learned": L["newton"]["mean"],
           "assemblies_plain": P["assemblies"]["mean"], "assemblies_learned": L["assemblies"]["mean"],
           "energy_evals_plain": P["energy_evals"]["mean"], "energy_evals_learned": L["energy_evals"]["mean"],
           "all_converged": bool(P["all_converged"] and L["all_converged"]),
           "learned_start_chosen": L["learned_start_chosen"], "seconds": time.perf_counter() - t0}
    out["newton_ratio_learned_over_plain"] = out["newton_learned"] / out["newton_plain"]
    return out


def measure_dualmesh(dev, reps: int = 50) -> dict:
    """Dual-mesh mapper: the one-off embedding and the per-frame update of
    655362 visual vertices on a 20480-triangle surface (float32 update)."""
    import numpy as np
    import torch

    from gen import workloads
    from paper_2605_24339_amd.dualmesh import DualMesh
    P, V, F = workloads.dual_mesh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dm = DualMesh(P, V, F, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    embed_s = time.perf_counter() - t0
    Vd = torch.tensor(workloads.smooth_deformation(V), dtype=torch.float32, device=dev)
    out = torch.empty(P.shape[0], 3, dtype=torch.float32, device=dev)
    ms = _event_ms(lambda: dm.update(Vd, out), reps)
    N, nV, nT = P.shape[0], V.shape[0], F.shape[0]
    byts = 32 * N + 12 * nV + 12 * nT       # tri, bary, delta, out per vertex; surface read once
    gbs = byts / (ms * 1e-3) / 1e9
    return {"visual_vertices": N, "sim_triangles": nT, "embed_s": embed_s, "update_ms": ms,
            "update_vertices_per_s": N / (ms * 1e-3), "update_bytes": byts, "update_gbs": gbs,
            "update_frac_hbm": gbs / HBM_PEAK_GBS}


def measure_patch(dev) -> dict:
    """Contact patch test (two deformable blocks, non-matching interface):
    Table 1's errors for both face-sample kinds and kappa = 1e4, 1e6, 1e8,
    with the wall time of each quasi-static GPU solve."""
    from paper_2605_24339_amd import patchtest
    patchtest.run(n_top=4, n_bot=6, kappas=(1e6,), device=dev)      # warm-up (library loads, allocator)
    return patchtest.run(n_top=4, n_bot=6, device=dev)


def cpu_patch(kappa: float = 1e6) -> dict:
    """The oracle's quasi-static patch-test solves on the same scene."""
    from gen import workloads
    from oracle import fem as ofem
    pt = workloads.patch_test(n_top=4, n_bot=6)
    out = {}
    for mortar in (False, True):
        t0 = time.perf_counter()
        ofem.patch_test(pt, kappa, mortar=mortar)
        out["clipped mortar" if mortar else "whole triangle"] = time.perf_counter() - t0
    return {"kappa": kappa, "seconds": out, "what": "FP64 oracle: Newton with direct sparse solves, 4x4x2 on "
                                                    "6x6x3 cube blocks (one quasi-static solve per sample kind)"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads() -> int:
    """Host threads the oracle may use: the process's CPU share (the
    OMP_NUM_THREADS limit when set, else the affinity mask)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    return min(n, int(env)) if env and env.isdigit() and int(env) > 0 else n


def cpu_baseline(envs, budget_s: float, threads: int) -> dict:
    """The FP64 oracle as it stands (built -O3 -march=native for this host)
    on a bounded sample of the workload: full passes (narrow phase,
    assembly with the BSR Hessian, step bound) over the environments in
    order, until the time budget is spent; samples/s over the passes done."""
    import oracle
    from gen import workloads
    oracle.use_library(oracle_native_lib())
    oracle.set_threads(threads)
    problems = {}
    done, n_pass, busy = 0, 0, 0.0
    while busy < budget_s:
        i = n_pass % len(envs)
        w = envs[i]
        if i not in problems:               # problem set-up is not timed
            problems[i] = workloads.to_problem(w)
        P = problems[i]
        t0 = time.perf_counter()
        nr = oracle.narrow(P)
        oracle.assemble(P, nr.M, project=False)
        oracle.ccd_step(P, nr.M, w.dxs, w.dxm)
        busy += time.perf_counter() - t0
        done += P.Ns
        n_pass += 1
    what = (f"environments 0..{min(n_pass, len(envs)) - 1} of the {len(envs)}" if len(envs) > 1
            else "the whole workload")
    return {"value": done / busy, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_pass} full passes (narrow phase + assembly with BSR + step bound) over {what} "
                      f"({done} samples), FP64, {threads} thread(s), {busy:.1f} s"}


_NATIVE = None


def oracle_native_lib() -> str:
    global _NATIVE
    if _NATIVE is None:
        from oracle import build as obuild
        _NATIVE = obuild.build_native()
    return _NATIVE


def _counter_means(path: str, counter: str) -> dict:
    """Mean value of one rocprofv3 --pmc counter per kernel name (CSV)."""
    import csv
    import re
    acc = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "")
            name = re.sub(r"\(.*", "", re.sub(r"^void ", "", name)).split("::")[-1]
            a = acc.setdefault(name, [0.0, 0])
            a[0] += float(r["Counter_Value"])
            a[1] += 1
    return {k: v[0] / v[1] for k, v in acc.items()}


def ingest_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, workload, ref_kernel="k_narrow_f32"):
    """HBM traffic of every kernel of a workload's step from two counter runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
    same counter reads for a plain device copy of known size.  Launches per
    step are the dispatches of one step (between the last two launches of
    ref_kernel, once per step).  Stored in profiles/traffic.json under the
    current source hash."""
    import csv
    copy_bytes = 4 * 64 * 1024 * 1024
    cf = _counter_means(copy_fetch_csv, "FETCH_SIZE")
    cw = _counter_means(copy_write_csv, "WRITE_SIZE")
    ck = max(cf, key=cf.get)                    # the copy kernel is the largest dispatch
    f_scale = copy_bytes / (cf[ck] * 1024.0)
    w_scale = copy_bytes / (cw[ck] * 1024.0)
    f = _counter_means(fetch_csv, "FETCH_SIZE")
    w = _counter_means(write_csv, "WRITE_SIZE")

    def step_launches(path):
        """Launches of each kernel in one step: the dispatches from the
        second-to-last launch of ref_kernel (once per step) to the last."""
        import re
        seq = []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != "FETCH_SIZE":
                    continue
                name = r["Kernel_Name"].replace("(anonymous namespace)::", "")
                name = re.sub(r"\(.*", "", re.sub(r"^void ", "", name)).split("::")[-1]
                seq.append((int(r["Dispatch_Id"]), name))
        seq.sort()
        ref = [i for i, (_, n) in enumerate(seq) if n == ref_kernel]
        n = {}
        for _, k in seq[ref[-2]:ref[-1]]:
            n[k] = n.get(k, 0) + 1
        return n

    per_step = step_launches(fetch_csv)
    kernels = {k: f[k] * 1024.0 * f_scale + w.get(k, 0.0) * 1024.0 * w_scale for k in f}
    step = sum(kernels[k] * per_step.get(k, 0) for k in kernels)
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    known = {}
    if os.path.exists(tf):
        with open(tf) as fh:
            known = json.load(fh)
    known[workload] = {"src_hash": src_hash(), "kernels": {k: round(v) for k, v in kernels.items()
                                                           if k.startswith("k_")},
                       "launches_per_step": per_step,
                       "step_bytes": round(step), "copy_kernel": ck, "fetch_scale": f_scale, "write_scale": w_scale}
    with open(tf, "w") as fh:
        json.dump(known, fh, indent=1)
    print(json.dumps({"workload": workload, "step_bytes": round(step),
                      "kernels": sorted(((round(v), k) for k, v in kernels.items()), reverse=True)[:12]}))


def _workload_line(r: dict, name: str) -> dict:
    """Figures of one measured workload."""
    c = r["counts"]
    ccd_pairs = c["active"] + c["swept"]
    return {"workload": name, "samples": r["samples"], "value": r["value"], "unit": "samples/s",
            "ms_per_step": r["ms"], "active_samples_per_s": c["active"] / (r["ms"] * 1e-3),
            "ccd_pairs_per_s": ccd_pairs / (r["ccd_ms"] * 1e-3) if r["ccd_ms"] > 0 else None,
            "ccd_ms": r["ccd_ms"], "counts": c, "counts_source": r["counts_source"], "gpu_counts": r["gpu_counts"],
            "stage_ms": r["stages"], "autotune_ms": r["autotune"], "tuning": r["tuning"], "roofline": r["roofline"],
            "roofline_step": r["roofline_step"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--indenter", default="sphere", choices=["sphere", "letter"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="oracle time budget of the headline CPU baseline (the other legs take fractions of it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other rows (autograd, MLP, dual mesh, mortar, features, patch test)")
    ap.add_argument("--workload", default=None, choices=["batched_256_envs", "large_indent"],
                    help="measure only this workload's step (for per-workload kernel profiles)")
    ap.add_argument("--autotune-cache", default=None,
                    help="JSON file of autotuned cell sizes to reuse (default: tune every run)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--ingest-counters", nargs=5, default=None,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV", "WORKLOAD"),
                    help="CPU only: record the workload's per-kernel HBM traffic from rocprofv3 --pmc CSVs")
    args = ap.parse_args()

    if args.ingest_counters:
        ingest_counters(*args.ingest_counters)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = 64 * 1024 * 1024
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))
        return

    from gen import workloads

    dev = torch.device("cuda", 0)
    w = workloads.large_indent(indenter=args.indenter)
    if args.workload == "large_indent":
        r = measure(w.name, [w], workloads.concat([w]), args.steps, args.warmup, dev, args.autotune_cache)
        print(json.dumps(_workload_line(r, w.name)))
        return
    B = workloads.batched()
    bt = measure("batched_256_envs", B.envs, B, args.steps, args.warmup, dev, args.autotune_cache)
    if args.workload == "batched_256_envs":
        print(json.dumps(_workload_line(bt, "batched_256_envs")))
        return
    head = _workload_line(bt, "batched_256_envs")
    rules = sorted({e.rule_n for e in B.envs})
    out = {
        "metric": METRIC,
        "value": bt["value"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bt["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched_256_envs", "n_env": len(B.envs), "samples": int(bt["samples"]),
                   "slave_tris": int(B.ts.shape[0]), "master_tris": int(B.tm.shape[0]),
                   "pads": "32x32..128x128 quads", "rules": "/".join(f"{n}x{n}" for n in rules),
                   "indenter_tris": "980..40500", "dhat": B.envs[0].dhat, "kappa": B.envs[0].kappa},
        "ccd_pairs_per_s": head["ccd_pairs_per_s"],
        "active_samples_per_s": head["active_samples_per_s"],
        "counts": head["counts"],
        "counts_source": head["counts_source"],
        "gpu_counts": head["gpu_counts"],
        "stage_ms": head["stage_ms"],
        "autotune_ms": head["autotune_ms"],
        "tuning": head["tuning"],
        "roofline": head["roofline"],
        "roofline_step": head["roofline_step"],
    }
    single = measure(w.name, [w], workloads.concat([w]), args.steps, args.warmup, dev, args.autotune_cache)
    out["large_indent"] = _workload_line(single, w.name)
    if not args.no_extras:
        out["autograd"] = measure_autograd(w, dev)
        out["mlp"] = measure_mlp(dev)
        out["dualmesh"] = measure_dualmesh(dev)
        mo = measure(w.name + "/mortar", [w], workloads.concat([w]), max(10, args.steps // 5), 3, dev, mortar=True)
        out["mortar"] = {"workload": w.name + " with clipped mortar face samples", "ms_per_step": mo["ms"],
                         "slave_samples_per_s": mo["value"], "clipped_active_samples": mo["gpu_counts"]["active"],
                         "pairs": mo["gpu_counts"]["pairs"], "stage_ms": mo["stages"]}
        fe = measure(w.name + "/features", [w], workloads.concat([w]), max(10, args.steps // 5), 3, dev,
                     mortar=True, features=(w.kappa * 1e-3, w.kappa * 1e-7, 0.1))
        out["features"] = {"workload": w.name + " with clipped face, edge and point samples (kappa_edge = "
                                       "1e-3 kappa, kappa_point = 1e-7 kappa, delta_e = 0.1)",
                           "ms_per_step": fe["ms"], "slave_samples_per_s": fe["value"],
                           "active_samples": fe["gpu_counts"]["active"], "pairs": fe["gpu_counts"]["pairs"],
                           "stage_ms": fe["stages"]}
        out["patch_test"] = measure_patch(dev)
        out["newton_iters_learned_vs_plain"] = measure_warmstart()
    if not args.no_cpu_baseline:
        nt = oracle_threads()
        cb = cpu_baseline(B.envs, args.cpu_seconds, nt)
        cb["cpu_model"] = cpu_model()
        cb["build"] = "gcc -O3 -march=native -fopenmp"
        cb["single_thread"] = cpu_baseline(B.envs, args.cpu_seconds / 2, 1)
        cb["large_indent"] = {"threads": cpu_baseline([w], args.cpu_seconds / 2, nt),
                              "single_thread": cpu_baseline([w], args.cpu_seconds / 2, 1)}
        if not args.no_extras:
            cb["patch_test"] = cpu_patch()
        out["cpu_baseline"] = cb
    print(json.dumps(out))


if __name__ == "__main__":
    main()
