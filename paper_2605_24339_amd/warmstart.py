"""Learned warm start study: a gel block pressed against a sphere, implicit
Euler steps solved by Newton (GMCP contact + linear tets), with the Newton
start either plain (x_t + dt v_t) or learned (plus the MLP's predicted
correction); both pass the same contact step-bound filter and both are run
to the same residual, so the converged solution judges the prediction.

Scene of trajectory j (seed 5000 + j): 64 x 64 x 8 cubes of 0.3125 mm
(20 x 20 x 2.5 mm, 196608 tets, 38025 vertices), E = 0.3 MPa, nu = 0.45,
density 1000 kg/m^3, dt = 1 ms, bottom face prescribed; a rigid sphere
(icosphere subdivision 3) of radius U[2, 6] mm above the top face (lateral
offset within 3 mm, initial gap U[0.05, 0.2] mm).  The relative
indentation is driven through the prescribed bottom face, which moves
toward the sphere at U[2, 6] mm/s with a lateral drift of at most 4 mm/s
(at most 0.6 mm of travel in 100 steps on a 2.5 mm block).  The tactile
surface (slave) is the top face, 2 x 2 samples per triangle, dhat = 1 mm,
kappa = 2.5e6 (a contact pressure of about 3e4 Pa, 10 % strain of the gel,
is reached at a gap of dhat / 10).

The network's inputs are standardised and its outputs scaled by the
targets' RMS (fitted on the training rows).  With the safeguard (default)
the learned and the plain start are both filtered and the one with the
lower incremental potential starts Newton (two energy-only evaluations,
counted separately from assemblies).

    python -m paper_2605_24339_amd.warmstart --train 20 --test 5 --steps 100
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from gen import meshes

from . import Context
from .fem import Fem
from .mlp import MLP, features, targets
from .newton import ImplicitSolver

E_Y, NU, RHO, DT = 3e5, 0.45, 1000.0, 1e-3
KAPPA = 2.5e6


class Scene:
    def __init__(self, seed, n=64, nz=8, h=3.125e-4, device="cuda"):
        rng = np.random.default_rng(seed)
        self.h = h
        X, tets, top, bottom = meshes.tet_block(n, n, nz, h)
        self.X, self.tets, self.top, self.bottom = X, tets, top, bottom
        R = rng.uniform(2e-3, 6e-3)
        xm, tm = meshes.icosphere(3, R)
        c = np.array([n * h / 2 + rng.uniform(-3e-3, 3e-3) * n / 64,
                      n * h / 2 + rng.uniform(-3e-3, 3e-3) * n / 64,
                      nz * h + R + rng.uniform(5e-5, 2e-4)])
        self.xm = xm + c
        self.tm = tm
        v = np.zeros(3)
        v[2] = rng.uniform(2e-3, 6e-3)
        lat = rng.normal(size=2)
        v[:2] = lat / np.linalg.norm(lat) * rng.uniform(0, 4e-3)
        self.plate_v = v
        self.center = X.mean(0)
        self.L = float(np.ptp(X, axis=0).max())
        self.device = device

    def make_solver(self, tol=1e-6):
        dev = self.device
        fem = Fem(self.X, self.tets, E_Y, NU, RHO, DT, self.bottom, device=dev)
        ctx = Context.single(self.top, self.tm, self.X.shape[0], self.xm.shape[0], rule_n=2, kappa=KAPPA, dhat=1e-3,
                             dtype=torch.float64, kinematic=True, device=dev)
        ctx.build_samples(torch.tensor(self.X, device=dev))
        return ImplicitSolver(fem, ctx, E_Y * self.h * self.h, tol=tol)


class Scaler:
    """Standardisation of the network's inputs (mean / std of the nine
    features) and outputs (per-component RMS of the targets), fitted on the
    training rows, so that the bf16 network works with O(1) values."""

    def __init__(self, X, T):
        self.mu = X[:, :9].mean(0)
        self.sd = X[:, :9].std(0).clamp_min(1e-12)
        self.ts = T[:, :3].pow(2).mean(0).sqrt().clamp_min(1e-12)

    def x(self, X):
        out = torch.zeros_like(X)
        out[:, :9] = (X[:, :9] - self.mu) / self.sd
        return out

    def t(self, T):
        out = torch.zeros_like(T)
        out[:, :3] = T[:, :3] / self.ts
        return out

    def y(self, Y):
        return Y[:, :3] * self.ts


def run_trajectory(scene: Scene, steps: int, net: MLP | None = None, keep=True, log=None, scaler=None,
                   safeguard=True):
    """Simulate; returns per-step records (positions kept on the device)."""
    dev = scene.device
    solver = scene.make_solver()
    x = torch.tensor(scene.X, device=dev)
    v = torch.zeros_like(x)
    d_prev = torch.zeros_like(x)
    xm = torch.tensor(scene.xm, device=dev)
    plate = torch.tensor(scene.X, device=dev)
    pv = torch.tensor(scene.plate_v, device=dev)
    center = torch.tensor(scene.center, device=dev)
    recs = []
    for s in range(steps):
        plate = plate + DT * pv
        x_start = None
        feat = None
        if net is not None or keep:
            feat = features(x, v, d_prev, center, scene.L, scene.h, DT)
        t0 = time.perf_counter()
        if net is not None:
            y, _ = net.forward(scaler.x(feat).contiguous())
            pred = scaler.y(y).double() * scene.h
            if torch.isfinite(pred).all():
                x_start = x + DT * v + pred
        xn, st = solver.solve_step(x, v, xm, plate, x_start=x_start, safeguard=safeguard)
        if net is not None and (not st.converged or st.start_alpha < 1e-3):
            xn, st = solver.solve_step(x, v, xm, plate)     # fall back to the plain start
            st.fallback = True
        el = time.perf_counter() - t0
        d = xn - (x + DT * v)
        start_err = float((st.x0 - xn).abs().max().item()) / scene.h
        rec = dict(step=s, newton=st.newton_iters, assemblies=st.assemblies, energy_evals=st.energy_evals,
                   cg=st.cg_iters, residual=st.residual, converged=st.converged, start_alpha=st.start_alpha,
                   start_err=start_err, seconds=el, fallback=getattr(st, "fallback", False),
                   used_learned=st.used_start, n_active=int(solver.contact.status().n_active))
        if keep:
            rec["feat"] = feat
            rec["target"] = targets(xn, x, v, DT, scene.h)
        recs.append(rec)
        if log and (s % 20 == 0 or s == steps - 1):
            log(f"step {s}: newton {st.newton_iters} asm {st.assemblies} cg {st.cg_iters} r {st.residual:.2e} "
                f"{el * 1e3:.1f} ms")
        v = (xn - x) / DT
        d_prev = d
        x = xn
    return recs


def summarize(recs):
    a = lambda k: np.array([r[k] for r in recs], dtype=float)
    out = {}
    for k in ("newton", "assemblies", "energy_evals", "cg", "start_err"):
        v = a(k)
        out[k] = {"mean": float(v.mean()), "median": float(np.median(v)), "p90": float(np.percentile(v, 90))}
    out["all_converged"] = bool(all(r["converged"] for r in recs))
    out["max_residual"] = float(max(r["residual"] for r in recs))
    out["fallbacks"] = int(sum(r["fallback"] for r in recs))
    used = [r["used_learned"] for r in recs if r.get("used_learned") is not None]
    out["learned_start_chosen"] = (sum(used) / len(used)) if used else None
    contact = [r for r in recs if r.get("n_active", 0) > 0]
    out["contact_steps"] = len(contact)
    if contact:
        out["newton_in_contact"] = float(np.mean([r["newton"] for r in contact]))
        out["assemblies_in_contact"] = float(np.mean([r["assemblies"] for r in contact]))
    out["seconds_per_step"] = float(a("seconds").mean())
    return out


def init_params(seed=0, device="cuda"):
    """He-style initial parameters in the library's layout (zero padding)."""
    g = torch.Generator().manual_seed(seed)
    r = lambda *s: torch.randn(*s, generator=g, dtype=torch.float64)
    W1 = torch.zeros(16, 128, dtype=torch.float64)
    W1[:9] = r(9, 128) * np.sqrt(2.0 / 9)
    W4 = torch.zeros(128, 16, dtype=torch.float64)
    W4[:, :3] = r(128, 3) * np.sqrt(1.0 / 128) * 0.1
    parts = [W1, torch.zeros(128), r(128, 128) * np.sqrt(2.0 / 128), torch.zeros(128),
             r(128, 128) * np.sqrt(2.0 / 128), torch.zeros(128), W4, torch.zeros(16)]
    return torch.cat([p.reshape(-1).double() for p in parts]).float().to(device)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20)
    ap.add_argument("--test", type=int, default=5)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--nz", type=int, default=8)
    ap.add_argument("--out", default=None)
    ap.add_argument("--no-safeguard", action="store_true",
                    help="always start from the network's prediction (no energy comparison with the plain start)")
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)
    dev = "cuda"
    t0 = time.perf_counter()
    feats, targs, plain_train = [], [], []
    for j in range(args.train):
        sc = Scene(5000 + j, args.n, args.nz, device=dev)
        recs = run_trajectory(sc, args.steps, None, keep=True, log=log)
        log(f"train trajectory {j}: {summarize(recs)['newton']}")
        for r in recs:
            feats.append(r.pop("feat"))
            targs.append(r.pop("target"))
        plain_train += recs
    X = torch.cat(feats)
    T = torch.cat(targs)
    del feats, targs
    gen_s = time.perf_counter() - t0
    scaler = Scaler(X, T)
    net = MLP(init_params(0, dev))
    t1 = time.perf_counter()
    hist = net.train(scaler.x(X), scaler.t(T), epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    # held-out evaluation
    plain, learned = [], []
    for j in range(args.test):
        sc = Scene(5000 + args.train + j, args.n, args.nz, device=dev)
        p = run_trajectory(sc, args.steps, None, keep=False, log=log)
        l = run_trajectory(sc, args.steps, net, keep=False, log=log, scaler=scaler, safeguard=not args.no_safeguard)
        log(f"test trajectory {j}: plain {summarize(p)['newton']} learned {summarize(l)['newton']}")
        plain += p
        learned += l
    report = {
        "workload": f"gel block {args.n}x{args.n}x{args.nz} tets vs sphere, dt=1e-3, residual 1e-6",
        "train_trajectories": args.train, "test_trajectories": args.test, "steps": args.steps,
        "training_rows": int(X.shape[0]), "epochs": args.epochs, "train_seconds": train_s,
        "generation_seconds": gen_s, "loss_history": hist,
        "plain_train": summarize(plain_train), "plain_test": summarize(plain), "learned_test": summarize(learned),
        "safeguard": not args.no_safeguard,
        "per_step_test": [{"plain_newton": p["newton"], "learned_newton": l["newton"], "n_active": p["n_active"],
                           "learned_chosen": l["used_learned"]} for p, l in zip(plain, learned)],
    }
    pa, la = report["plain_test"]["assemblies"]["mean"], report["learned_test"]["assemblies"]["mean"]
    report["assemblies_ratio_learned_over_plain"] = la / pa if pa else None
    print(json.dumps(report))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(report, fh, indent=1)


if __name__ == "__main__":
    main()
