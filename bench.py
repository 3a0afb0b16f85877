#!/usr/bin/env python3
"""Throughput of the GMCP hot path on one MI355X.

One step = one pass of the whole path over the resident input: broad phase,
assembly (selection, barrier, energy, gradient, BSR Hessian) and the step
bound (linearised gap + additive CCD).  Workload: the single large
indentation - 128x128 noisy gel pad (32768 triangles, 4x4 samples each =
524288 samples) under a 40500-triangle perturbed geodesic sphere, float32.

Prints one JSON line: samples/s over the timed steps (inputs already in
HBM), per-stage HIP-event times, the roofline of the dominant stage and the
FP64 oracle's throughput on the host cores (a reported baseline).
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


def src_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2605_24339_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def stage_bytes(stage: str, w, st, ctx) -> float | None:
    """Algorithmic bytes of one launch of a stage: every input the stage's
    function needs read once, every output it produces written once."""
    Vs, Vm, Ts, Tm = w.xs.shape[0], w.xm.shape[0], w.ts.shape[0], w.tm.shape[0]
    na, npair, nc = int(st.n_active), int(st.n_pairs), int(st.n_candidates)
    if stage == "narrow":
        # slave positions/triangles/areas, candidate lists, master triangles and
        # positions; selected-sample records (48 B), per-triangle normal+sums
        # (48 B) and counters (16 B), pair sums (80 B), tile energies
        return (12 * Vs + 12 * Ts + 4 * Ts + 4 * (Ts + 1) + 4 * nc + 12 * Tm + 12 * Vm
                + 48 * na + 48 * Ts + 16 * Ts + 80 * npair + 8 * ctx.n_tiles_est)
    if stage == "bsr_rows":
        nnzb = int(st.nnzb)
        return (4 * 3 * Ts + 48 * Ts + 80 * npair + 4 * 3 * Tm + 4 * (Vs + Vm + 2)
                + 40 * nnzb + 4 * (Vs + Vm + 1))
    if stage == "cand_query":
        return 12 * Vs + 12 * Ts + 48 * Tm + 4 * (Ts + 1) + 4 * nc
    if stage == "ccd_accd":
        return 24 * Vs + 12 * Ts + 24 * Vm + 12 * Tm + 48 * Tm
    if stage == "grid_build":
        return 12 * Vs + 12 * Ts + 12 * Vm + 12 * Tm + 48 * Tm
    if stage == "grad_rows":
        return 48 * Ts + 80 * npair + 12 * (Vs + Vm)
    return None


def cpu_baseline(w, budget_s: float) -> dict:
    import numpy as np
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
    ns = P.Ns * reps
    return {"value": ns / dt, "unit": "samples/s", "cores": int(os.environ.get("OMP_NUM_THREADS", threads)),
            "kind": "oracle",
            "sample": f"{reps} full passes (narrow + assembly with BSR + step bound) of the whole "
                      f"{P.Ns}-sample workload, FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--indenter", default="sphere", choices=["sphere", "letter"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding paragraph of the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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
    from paper_2605_24339_amd import Context

    w = workloads.large_indent(indenter=args.indenter)
    dev = torch.device("cuda", 0)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    xs, xm, dxs, dxm = t(w.xs), t(w.xm), t(w.dxs), t(w.dxm)
    ctx = Context.single(w.ts, w.tm, w.xs.shape[0], w.xm.shape[0], rule_n=w.rule_n, kappa=w.kappa,
                         dhat=w.dhat, delta_T=w.delta_T, dtype=torch.float32, device=dev)
    ctx.build_samples(xs)
    # first pass settles the capacities (checked), then unchecked steps
    ctx.step(xs, xm, dxs, dxm, check=True)
    for _ in range(max(0, args.warmup - 1)):
        ctx.step(xs, xm, dxs, dxm)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.step(xs, xm, dxs, dxm)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = e0.elapsed_time(e1) / args.steps
    st = ctx.status()
    if st.code != 0:
        raise SystemExit(f"status {st.code} after the timed steps")
    n_swept = int(st.n_swept)
    n_active = int(st.n_active)

    # per-stage times over a second timed pass (events on the library's stream)
    ctx.profile(True)
    for _ in range(args.steps):
        ctx.step(xs, xm, dxs, dxm)
    prof = ctx.profile_read()
    ctx.profile(False)
    st2 = ctx.status()
    stages = {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1] > 0}
    ctx.n_tiles_est = (w.ts.shape[0] + 3) // 4
    dom = max(stages, key=stages.get)
    dom_ms = stages[dom]
    byts = stage_bytes(dom, w, st2, ctx)
    roof = None
    if byts is not None:
        achieved = byts / (dom_ms * 1e-3) / 1e9
        traffic = None
        tf = os.path.join(ROOT, "profiles", "traffic.json")
        if os.path.exists(tf):
            with open(tf) as fh:
                rec = json.load(fh)
            ent = rec.get(dom)
            if ent and ent.get("src_hash") == src_hash() and ent.get("workload") == w.name:
                traffic = ent.get("bytes_per_launch")
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": dom,
                "algorithmic_bytes": int(byts), "avg_ms": round(dom_ms, 5)}

    Ns = w.n_samples
    out = {
        "metric": METRIC,
        "value": Ns / (ms * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "slave_tris": int(w.ts.shape[0]), "samples": int(Ns),
                   "master_tris": int(w.tm.shape[0]), "rule": f"{w.rule_n}x{w.rule_n}", "dhat": w.dhat,
                   "kappa": w.kappa},
        "ccd_pairs_per_s": (n_active + n_swept) / ((stages.get("ccd_linear", 0) + stages.get("ccd_grid", 0)
                                                    + stages.get("ccd_accd", 0)) * 1e-3 + 1e-30),
        "active_samples": n_active,
        "swept_pairs": n_swept,
        "nnzb": int(st2.nnzb),
        "stage_ms": {k: round(v, 5) for k, v in stages.items()},
        "wall_s_timed": round(wall, 4),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
