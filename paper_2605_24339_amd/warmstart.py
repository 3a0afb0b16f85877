"""Learned warm start study: a gel block tapped by a rigid sphere, implicit
Euler steps solved by Newton (GMCP contact + linear tets), with the Newton
start either plain (x_t + dt v_t) or learned (plus the MLP's predicted
correction); both pass the same contact step-bound filter and both are run
to the same residual, so the converged solution judges the prediction.

Scene of trajectory j (seed 5000 + j): 64 x 64 x 8 cubes of 0.3125 mm
(20 x 20 x 2.5 mm, 196608 tets, 38025 vertices), E = 0.3 MPa, nu = 0.45,
density 1000 kg/m^3, dt = 1 ms, bottom face prescribed; a rigid sphere
(icosphere subdivision 3) of radius U[2, 6] mm (lateral offset within
3 mm) starting U[0.2, 1] mm above the top face.  The sphere taps the gel:
it approaches at U[0.01, 0.1] m/s, presses U[0.2, 0.6] mm past first
contact, withdraws at the same speed to its starting height and repeats,
with a lateral drift of at most 0.02 m/s.  The motion is applied to the
prescribed bottom face instead (the same relative motion; at these rates
the gel's inertia is four orders of magnitude below its stiffness, so the
response is quasi-static and the frame does not matter), which keeps the
contact context's master mesh fixed between steps.  The tactile surface
(slave) is the top face, 2 x 2 samples per triangle, dhat = 1 mm,
kappa = 2.5e6: a contact pressure of about 3e4 Pa (10 % strain of the gel)
balances the barrier at a gap of about 0.1 mm, above the sag of the
sphere's facets (25 to 70 um); at kappa = 1e5 the same pressure needs gaps
of a few um, below the facets' sag, and the indenter's vertices then press
between the slave samples where no sample resists them, which stalls
Newton against the step bound.

The network sees each vertex's position in the indenter's frame (lateral
offset from the sphere's axis in radii and the log of the distance to its
surface in cells), its velocity relative to the prescribed motion of the
coming step (x dt / cell) and its previous correction (/ cell); inputs are
standardised and outputs scaled by the targets' RMS (fitted on the
training rows).  With the safeguard (default) the learned and the plain
start are both filtered and the one with the lower incremental potential
starts Newton (two energy-only evaluations, counted separately from
assemblies).

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
from .mlp import MLP, PAD, targets
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
        g0 = rng.uniform(2e-4, 1e-3)
        c = np.array([n * h / 2 + rng.uniform(-3e-3, 3e-3) * n / 64,
                      n * h / 2 + rng.uniform(-3e-3, 3e-3) * n / 64, 0.0])
        xm = xm + c
        xm = meshes.place_above(xm, X[top.ravel()], g0)    # lowest sphere vertex g0 above the top face
        self.xm, self.tm = xm, tm
        self.R = R
        self.c = xm.mean(0)                                 # sphere centre (the icosphere is centred)
        self.speed = rng.uniform(0.01, 0.1)
        self.depth = rng.uniform(2e-4, 6e-4)
        self.amp = g0 + self.depth                          # approach travel of one tap
        lat = rng.normal(size=2)
        self.drift = np.zeros(3)
        self.drift[:2] = lat / np.linalg.norm(lat) * rng.uniform(0.0, 0.02)
        self.center = X.mean(0)
        self.L = float(np.ptp(X, axis=0).max())
        self.device = device

    def plate_offset(self, step: int) -> np.ndarray:
        """Displacement of the prescribed bottom face at the end of step
        `step` (time (step + 1) dt): the sphere's tap motion seen from the
        gel (upward toward the sphere, then back), minus the drift."""
        t = (step + 1) * DT
        u = (self.speed * t) % (2.0 * self.amp)
        z = u if u <= self.amp else 2.0 * self.amp - u
        return np.array([0.0, 0.0, z]) - self.drift * t

    def make_solver(self, tol=1e-6):
        dev = self.device
        fem = Fem(self.X, self.tets, E_Y, NU, RHO, DT, self.bottom, device=dev)
        ctx = Context.single(self.top, self.tm, self.X.shape[0], self.xm.shape[0], rule_n=2, kappa=KAPPA, dhat=1e-3,
                             dtype=torch.float64, kinematic=True, device=dev)
        ctx.build_samples(torch.tensor(self.X, device=dev))
        return ImplicitSolver(fem, ctx, E_Y * self.h * self.h, tol=tol)


def features(scene: Scene, x_t, v_t, d_prev, v_next):
    """[V][16] network inputs (float32, zero padding): position in the
    indenter's frame - lateral offset from the sphere's axis / R and
    ln(distance to the sphere's surface / cell + 1e-3) -, velocity relative
    to the prescribed motion of the coming step x dt / cell, previous
    correction / cell."""
    h = scene.h
    c = torch.tensor(scene.c, dtype=x_t.dtype, device=x_t.device)
    r = x_t - c
    dist = (r.norm(dim=1) - scene.R).clamp_min(0.0)
    f = torch.zeros(x_t.shape[0], PAD, dtype=torch.float32, device=x_t.device)
    f[:, 0:2] = (r[:, 0:2] / scene.R).float()
    f[:, 2] = torch.log(dist / h + 1e-3).float()
    vn = torch.tensor(v_next, dtype=x_t.dtype, device=x_t.device)
    f[:, 3:6] = ((v_t - vn) * DT / h).float()
    f[:, 6:9] = (d_prev / h).float()
    return f


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
                   safeguard=True, newton_log=None):
    """Simulate; returns per-step records (features and targets kept on the
    device when keep).  newton_log receives the solver's per-iteration lines."""
    dev = scene.device
    solver = scene.make_solver()
    x = torch.tensor(scene.X, device=dev)
    v = torch.zeros_like(x)
    d_prev = torch.zeros_like(x)
    xm = torch.tensor(scene.xm, device=dev)
    X0 = torch.tensor(scene.X, device=dev)
    recs = []
    for s in range(steps):
        off = scene.plate_offset(s)
        plate = X0 + torch.tensor(off, device=dev)
        v_next = (off - (scene.plate_offset(s - 1) if s > 0 else np.zeros(3))) / DT
        x_start = None
        feat = None
        if net is not None or keep:
            feat = features(scene, x, v, d_prev, v_next)
        t0 = time.perf_counter()
        if net is not None:
            y = net.predict(scaler.x(feat).contiguous())
            pred = scaler.y(y).double() * scene.h
            if torch.isfinite(pred).all():
                x_start = x + DT * v + pred
        xn, st = solver.solve_step(x, v, xm, plate, x_start=x_start, safeguard=safeguard, log=newton_log)
        if net is not None and (not st.converged or st.start_alpha < 1e-3):
            xn, st = solver.solve_step(x, v, xm, plate, log=newton_log)     # fall back to the plain start
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
                f"active {rec['n_active']} {el * 1e3:.1f} ms")
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


def save_checkpoint(path: str, net: MLP, scaler: Scaler):
    """Network parameters and feature / target scaling (numeric arrays only)."""
    np.savez(path, params=net.p.detach().cpu().numpy(), mu=scaler.mu.cpu().numpy(), sd=scaler.sd.cpu().numpy(),
             ts=scaler.ts.cpu().numpy())


def load_checkpoint(path: str, device="cuda"):
    """(MLP, Scaler) from save_checkpoint's file; loads no executable content."""
    with np.load(path, allow_pickle=False) as z:
        net = MLP(torch.tensor(z["params"], dtype=torch.float32, device=device))
        sc = Scaler.__new__(Scaler)
        sc.mu = torch.tensor(z["mu"], dtype=torch.float32, device=device)
        sc.sd = torch.tensor(z["sd"], dtype=torch.float32, device=device)
        sc.ts = torch.tensor(z["ts"], dtype=torch.float32, device=device)
    return net, sc


def normalized_loss(net: MLP, scaler: Scaler, X, T, batch=65536) -> float:
    """Mean squared error of the scaled prediction over the rows, divided by
    the mean square of the scaled targets (1 = no better than zero)."""
    num = den = 0.0
    for i in range(0, X.shape[0], batch):
        xb = scaler.x(X[i:i + batch]).contiguous()
        tb = scaler.t(T[i:i + batch])
        y = net.predict(xb)
        num += float(((y[:, :3] - tb[:, :3]) ** 2).sum().item())
        den += float((tb[:, :3] ** 2).sum().item())
    return num / max(den, 1e-300)


def study(train: int, test: int, steps: int, epochs: int, batch: int, lr: float, lr_min: float | None, n: int, nz: int,
          safeguard: bool = True, seed0: int = 5000, log=None, save: str | None = None, net=None, scaler=None,
          heldout_seed0: int | None = None):
    """Generate training trajectories with the plain start (seeds seed0..),
    train the network on the GPU (unless one is given), and run the
    held-out trajectories (seeds heldout_seed0.., by default right after the
    training seeds) with both starts."""
    if heldout_seed0 is None:
        heldout_seed0 = seed0 + train
    dev = "cuda"
    t0 = time.perf_counter()
    feats, targs, plain_train = [], [], []
    for j in range(train):
        sc = Scene(seed0 + j, n, nz, device=dev)
        recs = run_trajectory(sc, steps, None, keep=True, log=log)
        if log:
            log(f"train trajectory {j}: {summarize(recs)['newton']}")
        for r in recs:
            feats.append(r.pop("feat"))
            targs.append(r.pop("target"))
        plain_train += recs
    gen_s = time.perf_counter() - t0
    hist, train_s, rows, train_loss = [], 0.0, 0, None
    if net is None:
        X = torch.cat(feats)
        T = torch.cat(targs)
        del feats, targs
        rows = int(X.shape[0])
        scaler = Scaler(X, T)
        net = MLP(init_params(0, dev))
        t1 = time.perf_counter()
        hist = net.train(scaler.x(X), scaler.t(T), epochs=epochs, batch=batch, lr=lr, log=log, lr_min=lr_min)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t1
        train_loss = normalized_loss(net, scaler, X, T)
        del X, T
        if save:
            save_checkpoint(save, net, scaler)
    plain, learned, vx, vt = [], [], [], []
    for j in range(test):
        sc = Scene(heldout_seed0 + j, n, nz, device=dev)
        p = run_trajectory(sc, steps, None, keep=True, log=log)
        for r in p:
            vx.append(r.pop("feat"))
            vt.append(r.pop("target"))
        l = run_trajectory(sc, steps, net, keep=False, log=log, scaler=scaler, safeguard=safeguard)
        if log:
            log(f"test trajectory {j}: plain {summarize(p)['newton']} learned {summarize(l)['newton']}")
        plain += p
        learned += l
    val_loss = normalized_loss(net, scaler, torch.cat(vx), torch.cat(vt)) if vx else None
    report = {
        "workload": f"gel block {n}x{n}x{nz} cubes of linear tets tapped by a sphere, dt=1e-3, residual 1e-6",
        "train_trajectories": train, "test_trajectories": test, "steps": steps, "training_rows": rows,
        "epochs": epochs, "lr": lr, "lr_min": lr_min, "train_seconds": train_s, "generation_seconds": gen_s,
        "loss_history": hist, "train_normalized_loss": train_loss, "heldout_normalized_loss": val_loss,
        "plain_train": summarize(plain_train) if plain_train else None, "plain_test": summarize(plain),
        "learned_test": summarize(learned), "safeguard": safeguard,
        "per_step_test": [{"plain_newton": p["newton"], "learned_newton": l["newton"], "n_active": p["n_active"],
                           "plain_err": p["start_err"], "learned_err": l["start_err"],
                           "learned_chosen": l["used_learned"]} for p, l in zip(plain, learned)],
    }
    pa, la = report["plain_test"]["assemblies"]["mean"], report["learned_test"]["assemblies"]["mean"]
    report["assemblies_ratio_learned_over_plain"] = la / pa if pa else None
    return report, net, scaler


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20)
    ap.add_argument("--test", type=int, default=5)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-min", type=float, default=2e-5)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--nz", type=int, default=8)
    ap.add_argument("--out", default=None)
    ap.add_argument("--save", default=None, help="write the trained network and its scaling here (.npz)")
    ap.add_argument("--load", default=None,
                    help="evaluate this trained network (trained on the first --train seeds) instead of training one")
    ap.add_argument("--no-safeguard", action="store_true",
                    help="always start from the network's prediction (no energy comparison with the plain start)")
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)
    net = scaler = None
    if args.load:
        net, scaler = load_checkpoint(args.load)
    # a loaded network was trained on the first args.train seeds: held-out seeds follow them
    report, _, _ = study(0 if args.load else args.train, args.test, args.steps, args.epochs, args.batch, args.lr,
                         args.lr_min, args.n, args.nz, not args.no_safeguard, log=log, save=args.save, net=net,
                         scaler=scaler, heldout_seed0=5000 + args.train)
    print(json.dumps({k: v for k, v in report.items() if k != "per_step_test"}))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(report, fh, indent=1)


if __name__ == "__main__":
    main()
