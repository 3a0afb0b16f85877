#!/usr/bin/env python3
"""Throughput of the GMCP hot path on one MI355X.

One step = one pass of the whole path over the resident input: broad phase,
assembly (selection, barrier, energy, gradient, BSR Hessian) and the step
bound (linearised gap + additive CCD).  Headline workload: the single large
indentation - 128x128 noisy gel pad (32768 triangles, 4x4 samples each =
524288 samples) under a 40500-triangle perturbed geodesic sphere, float32.
The step is captured once into a HIP graph and replayed; the broad-phase
cell size is chosen by the autotuner first.

Prints one JSON line: samples/s over the timed steps (inputs already in
HBM), per-kernel HIP-event times, the roofline of the dominant kernel, the
same figures for the 256-environment batch, and the FP64 oracle's
throughput on the host cores (a reported baseline, not the target).
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
# kernels that one profiled stage brackets exactly (candidates for the roofline)
KERNEL_STAGES = {"query": "k_query_f32", "cand_move": "k_cand_move", "narrow": "k_narrow_f32",
                 "rows_count": "k_rows<float, 0, false>", "rows_fill": "k_rows<float, 1, false>",
                 "rows_count_heavy": "k_rows<float, 0, true>", "rows_fill_heavy": "k_rows<float, 1, true>",
                 "ccd_linear": "k_ccd_linear<float>", "ccd_accd": "k_ccd_accd<float>"}


def src_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2605_24339_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def kernel_bytes(stage: str, sz: dict) -> int:
    """Algorithmic bytes of one launch: each input the kernel's function
    needs, read once, and each output it produces, written once (float32)."""
    Vs, Vm, Ts, Tm = sz["Vs"], sz["Vm"], sz["Ts"], sz["Tm"]
    na, npair, nc, nnzb, ntile = sz["n_active"], sz["n_pairs"], sz["n_cand"], sz["nnzb"], sz["n_tiles"]
    V = Vs + Vm
    if stage == "narrow":
        # slave x / triangles / areas, candidate CSR, master triangles + x;
        # records 64 B per active sample, per-triangle normal+sums+counters
        # 64 B, pairs 80 B, tile energies 8 B
        return 12 * Vs + 16 * Ts + 4 * (Ts + 1) + 4 * nc + 12 * Tm + 12 * Vm + 64 * na + 64 * Ts + 80 * npair + 8 * ntile
    if stage == "query":
        # slave positions / triangles, master boxes; out: per-triangle counts
        # and scratch offsets, sorted scratch lists
        return 12 * Vs + 12 * Ts + 48 * Tm + 8 * Ts + 4 * nc
    if stage == "cand_move":
        return 12 * Ts + 8 * nc
    if stage in ("rows_count", "rows_fill"):
        # light rows: active slave triangles' sums and normals, their pairs,
        # slave adjacency; out: counts, or blocks + row gradients
        rl, nl = sz["rows_light"], sz["nnzb_light"]
        ta = min(Ts, npair)
        inp = 48 * ta + 80 * npair + 12 * Ts + 4 * (Vs + 1) + 8 * rl
        return inp + (4 * rl if stage == "rows_count" else 40 * nl + 12 * rl)
    if stage in ("rows_count_heavy", "rows_fill_heavy"):
        # heavy rows: per-master-triangle blocks, bucket keys and the pairs'
        # slave triangles, master adjacency; out: counts, or blocks + gradients
        rh, nh = sz["rows_heavy"], sz["nnzb_heavy"]
        tma = min(Tm, npair)
        inp = 180 * tma + 8 * npair + 12 * npair + 4 * (Tm + 1) + 12 * Tm + 4 * (Vm + 1) + 8 * rh
        return inp + (4 * rh if stage == "rows_count_heavy" else 40 * nh + 12 * rh)
    if stage == "ccd_linear":
        # records, slave normals and triangles, slave / master displacements, master triangles
        return 64 * na + 24 * Ts + 12 * Vs + 12 * Tm + 12 * Vm
    if stage == "ccd_accd":
        return 24 * Vs + 12 * Ts + 24 * Vm + 12 * Tm + 48 * Tm
    return 0


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

    cells, table = autotune.tune(make, envs, (xs, xm, dxs, dxm), cache=tune_cache if not mortar else None,
                                 scales=autotune.SCALES if not mortar else (0.0,))
    ctx = make(cells)
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
    sz = dict(Vs=batch.xs.shape[0], Vm=batch.xm.shape[0], Ts=batch.ts.shape[0], Tm=batch.tm.shape[0],
              n_active=int(st.n_active), n_pairs=int(st.n_pairs), n_cand=int(st.n_candidates),
              nnzb=int(st.nnzb), n_tiles=sum((w.ts.shape[0] * w.rule_n ** 2 + 63) // 64 for w in envs),
              **ctx.row_classes())
    kern = {k: v for k, v in stages.items() if k in KERNEL_STAGES}
    dom = max(kern, key=kern.get)
    byts = kernel_bytes(dom, sz)
    achieved = byts / (kern[dom] * 1e-3) / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        with open(tf) as fh:
            rec = json.load(fh).get(f"{name}/{dom}")
        if rec and rec.get("src_hash") == src_hash():
            traffic = rec.get("bytes_per_launch")
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": KERNEL_STAGES[dom],
            "stage": dom, "algorithmic_bytes": int(byts), "avg_ms": round(kern[dom], 5)}
    ccd_ms = stages.get("ccd_linear", 0) + stages.get("ccd_grid", 0) + stages.get("ccd_accd", 0)
    return dict(ms=ms, value=Ns / (ms * 1e-3), samples=Ns, stages={k: round(v, 5) for k, v in stages.items()},
                roofline=roof, sizes=sz, n_swept=int(st.n_swept), ccd_ms=ccd_ms, autotune=table,
                cells=cells[:4])


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
    flops = 3 * 2 * batch * (PAD * 128 + 2 * 128 * 128 + 128 * PAD)
    Mg, Ng, Kg = 1 << 18, 128, 128
    A = torch.randn(Mg, Kg, generator=g).to(dev)
    B = torch.randn(Kg, Ng, generator=g).to(dev)
    gms = _event_ms(lambda: gemm_bf16(A, B), reps)
    tf = 2 * Mg * Ng * Kg / (gms * 1e-3) / 1e12
    return {"train_rows_per_s": batch / (ms * 1e-3), "train_step_ms": ms, "batch": batch,
            "train_tflops": flops / (ms * 1e-3) / 1e12,
            "gemm": {"M": Mg, "N": Ng, "K": Kg, "ms": gms, "tflops": tf, "mfma_peak_tflops": 2500.0,
                     "gbs": 4 * (Mg * Kg + Kg * Ng + Mg * Ng) / (gms * 1e-3) / 1e9, "hbm_peak_gbs": HBM_PEAK_GBS,
                     "note": "float32 operands converted to bf16 on load, float32 out: HBM-bound at K = 128"}}


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


def cpu_baseline(w, budget_s: float) -> dict:
    import oracle
    from gen import workloads
    P = workloads.to_problem(w)
    threads = len(os.sched_getaffinity(0))
    reps, t0 = 0, time.perf_counter()
    while True:
        nr = oracle.narrow(P)
        oracle.assemble(P, nr.M, project=False)
        oracle.ccd_step(P, nr.M, w.dxs, w.dxm)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": P.Ns * reps / dt, "unit": "samples/s",
            "cores": int(os.environ.get("OMP_NUM_THREADS", threads)), "kind": "oracle",
            "sample": f"{reps} full passes (narrow phase + assembly with BSR + step bound) over all "
                      f"{P.Ns} samples of the same workload, FP64, OpenMP, {dt:.1f} s"}


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


def ingest_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, workload, stage, kernel):
    """HBM traffic of one kernel from two counter runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch), each scaled by what the same counter
    reads for a plain device copy of known size; stored in
    profiles/traffic.json under the current source hash."""
    copy_bytes = 4 * 64 * 1024 * 1024
    cf = _counter_means(copy_fetch_csv, "FETCH_SIZE")
    cw = _counter_means(copy_write_csv, "WRITE_SIZE")
    ck = max(cf, key=cf.get)                    # the copy kernel is the largest dispatch
    f_scale = copy_bytes / (cf[ck] * 1024.0)
    w_scale = copy_bytes / (cw[ck] * 1024.0)
    f = _counter_means(fetch_csv, "FETCH_SIZE")[kernel] * 1024.0 * f_scale
    w = _counter_means(write_csv, "WRITE_SIZE")[kernel] * 1024.0 * w_scale
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    known = {}
    if os.path.exists(tf):
        with open(tf) as fh:
            known = json.load(fh)
    known[f"{workload}/{stage}"] = {"kernel": kernel, "src_hash": src_hash(), "fetch_bytes": f, "write_bytes": w,
                                    "bytes_per_launch": f + w, "copy_kernel": ck,
                                    "fetch_scale": f_scale, "write_scale": w_scale}
    with open(tf, "w") as fh:
        json.dump(known, fh, indent=1)
    print(json.dumps(known[f"{workload}/{stage}"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--indenter", default="sphere", choices=["sphere", "letter"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the autograd and MLP measurements")
    ap.add_argument("--batched-only", action="store_true",
                    help="measure only the 256-environment batch (for per-workload kernel profiles)")
    ap.add_argument("--autotune-cache", default=None,
                    help="JSON file of autotuned cell sizes to reuse (default: tune every run)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--ingest-counters", nargs=7, default=None,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV", "WORKLOAD", "STAGE",
                             "KERNEL"),
                    help="CPU only: record the kernel's HBM traffic from rocprofv3 --pmc CSVs")
    args = ap.parse_args()

    if args.ingest_counters:
        ingest_counters(*args.ingest_counters)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path; run with --gpus 1",
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
    if args.batched_only:
        B = workloads.batched()
        bt = measure("batched_256", B.envs, B, args.steps, args.warmup, dev, args.autotune_cache)
        print(json.dumps({"workload": "batched_256_envs", "samples": bt["samples"], "value": bt["value"],
                          "unit": "samples/s", "ms_per_step": bt["ms"], "stage_ms": bt["stages"],
                          "roofline": bt["roofline"], "autotune_ms": bt["autotune"]}))
        return
    w = workloads.large_indent(indenter=args.indenter)
    single = measure(w.name, [w], workloads.concat([w]), args.steps, args.warmup, dev, args.autotune_cache)
    out = {
        "metric": METRIC,
        "value": single["value"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": single["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "slave_tris": int(w.ts.shape[0]), "samples": int(w.n_samples),
                   "master_tris": int(w.tm.shape[0]), "rule": f"{w.rule_n}x{w.rule_n}", "dhat": w.dhat,
                   "kappa": w.kappa},
        "ccd_pairs_per_s": (single["sizes"]["n_active"] + single["n_swept"]) / (single["ccd_ms"] * 1e-3),
        "active_samples": single["sizes"]["n_active"],
        "swept_pairs": single["n_swept"],
        "nnzb": single["sizes"]["nnzb"],
        "stage_ms": single["stages"],
        "autotune_ms": single["autotune"],
        "roofline": single["roofline"],
    }
    if not args.no_batched:
        B = workloads.batched()
        bt = measure("batched_256", B.envs, B, max(5, args.steps // 10), 2, dev, args.autotune_cache)
        out["batched"] = {"workload": "batched_256_envs", "samples": bt["samples"], "value": bt["value"],
                          "unit": "samples/s", "ms_per_step": bt["ms"], "stage_ms": bt["stages"],
                          "ccd_pairs_per_s": (bt["sizes"]["n_active"] + bt["n_swept"]) / (bt["ccd_ms"] * 1e-3),
                          "roofline": bt["roofline"], "autotune_ms": bt["autotune"]}
    if not args.no_extras:
        out["autograd"] = measure_autograd(w, dev)
        out["mlp"] = measure_mlp(dev)
        out["dualmesh"] = measure_dualmesh(dev)
        mo = measure(w.name + "/mortar", [w], workloads.concat([w]), max(10, args.steps // 5), 3, dev, mortar=True)
        out["mortar"] = {"workload": w.name + " with clipped mortar face samples", "ms_per_step": mo["ms"],
                         "slave_samples_per_s": mo["value"], "clipped_active_samples": mo["sizes"]["n_active"],
                         "pairs": mo["sizes"]["n_pairs"], "stage_ms": mo["stages"]}
        fe = measure(w.name + "/features", [w], workloads.concat([w]), max(10, args.steps // 5), 3, dev,
                     mortar=True, features=(w.kappa * 1e-3, w.kappa * 1e-7, 0.1))
        out["features"] = {"workload": w.name + " with clipped face, edge and point samples (kappa_edge = "
                                       "1e-3 kappa, kappa_point = 1e-7 kappa, delta_e = 0.1)",
                           "ms_per_step": fe["ms"], "slave_samples_per_s": fe["value"],
                           "active_samples": fe["sizes"]["n_active"], "pairs": fe["sizes"]["n_pairs"],
                           "stage_ms": fe["stages"]}
        out["patch_test"] = measure_patch(dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        if not args.no_extras:
            out["cpu_baseline"]["patch_test"] = cpu_patch()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
