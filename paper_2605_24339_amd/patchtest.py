"""The contact patch test of Sec. 5 (Table 1): two linear-elastic blocks
pressed together across a non-matching interface must carry the uniform
stress sigma_zz = -p (every other component zero) in both blocks.

The upper block is the slave body (its bottom face carries the samples),
the lower block the master body; both deform (no kinematic master), the
upper block moves along z only (u_x = u_y = 0) and the lower block's bottom
face is held, with a uniform pressure on the upper block's top face
(synthetic meshes of cubes split into six tetrahedra: the paper's TetGen
meshes are not available).  Quasi-static: implicit steps with zero velocity
(a proximal term M / dt^2 that vanishes at rest) until the positions stop
moving, each solved by the GPU Newton solver (FEM + GMCP + PCG + CCD line
search).  The stress of every tetrahedron is recovered from the converged
displacements (linear elasticity, small strain) on the device.

    python -m paper_2605_24339_amd.patchtest --out patch.json
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from gen import workloads

from . import Context
from .fem import Fem
from .newton import ImplicitSolver

RHO, DT = 1.0, 1.0      # quasi-static: the proximal term only regularises each step


def tet_stress(X, tets, x, young, poisson):
    """Cauchy stress [n_tet, 3, 3] of linear tetrahedra at positions x (torch, float64)."""
    mu = young / (2 * (1 + poisson))
    lam = young * poisson / ((1 + poisson) * (1 - 2 * poisson))
    P = X[tets]
    Dm = torch.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], dim=2)
    inv = torch.linalg.inv(Dm)                         # rows: gradients of N_1..N_3
    g = torch.cat([-inv.sum(1, keepdim=True), inv], 1)  # [n, 4, 3]
    F = torch.einsum("nai,naj->nij", (x - X)[tets], g)
    eps = 0.5 * (F + F.transpose(1, 2))
    tr = eps.diagonal(dim1=1, dim2=2).sum(-1)
    return lam * tr[:, None, None] * torch.eye(3, dtype=x.dtype, device=x.device) + 2 * mu * eps


def solve(pt: workloads.PatchTest, kappa: float, mortar: bool = False, rule_n: int = 2, steps: int = 4,
          tol: float = 1e-10, device="cuda"):
    """Quasi-static solve; returns (x [V, 3] tensor, stats per step)."""
    dev = torch.device(device)
    fem = Fem(pt.X, pt.tets, pt.young, pt.poisson, RHO, DT, pt.fixed, device=dev)
    fem.constrain(pt.roller, 1 | 2)
    Vs, V = pt.Vs, pt.X.shape[0]
    ctx = Context.single(pt.ts, pt.tm, Vs, V - Vs, rule_n=rule_n, kappa=kappa, dhat=pt.dhat, dtype=torch.float64,
                         kinematic=False, device=dev, mortar=mortar)
    X = torch.tensor(pt.X, dtype=torch.float64, device=dev)
    ctx.build_samples(X[:Vs].contiguous())
    f = torch.tensor(pt.f_ext, dtype=torch.float64, device=dev)
    solver = ImplicitSolver(fem, ctx, pt.young * pt.h_top ** 2, tol=tol, max_newton=200, f_ext=f)
    x, v = X.clone(), torch.zeros_like(X)
    stats = []
    for _ in range(steps):
        xn, st = solver.solve_step(x, v, None, X)
        stats.append(st)
        moved = float((xn - x).abs().max().item())
        x = xn
        if moved <= 1e-12:
            break
    return x, stats


def errors(pt: workloads.PatchTest, x) -> dict:
    """Max relative sigma_zz error and max spurious stress (largest |sigma_ij|
    over the other components), per block and overall (Table 1's measures)."""
    X = torch.tensor(pt.X, dtype=torch.float64, device=x.device)
    T = torch.tensor(pt.tets, dtype=torch.long, device=x.device)
    s = tet_stress(X, T, x, pt.young, pt.poisson)
    zz = (s[:, 2, 2] + pt.pressure).abs() / pt.pressure
    other = s.clone()
    other[:, 2, 2] = 0.0
    spur = other.abs().flatten(1).amax(1)
    upper = (T < pt.Vs).all(1)
    gap = float((x[:pt.Vs][torch.tensor(pt.ts, dtype=torch.long, device=x.device)][..., 2].min()
                 - x[pt.Vs:][torch.tensor(pt.tm, dtype=torch.long, device=x.device)][..., 2].max()).item())
    return {"sigma_zz_max_rel_err": float(zz.max()), "sigma_spur": float(spur.max()),
            "upper": {"sigma_zz_max_rel_err": float(zz[upper].max()), "sigma_spur": float(spur[upper].max())},
            "lower": {"sigma_zz_max_rel_err": float(zz[~upper].max()), "sigma_spur": float(spur[~upper].max())},
            "gap": gap}


def run(n_top: int = 4, n_bot: int = 6, kappas=(1e4, 1e6, 1e8), device="cuda") -> dict:
    """Table 1's sweep for both face-sample kinds on one mesh pair."""
    pt = workloads.patch_test(n_top=n_top, n_bot=n_bot)
    out = {"mesh": {"upper": f"{n_top}x{n_top}x{n_top // 2} cubes", "lower": f"{n_bot}x{n_bot}x{n_bot // 2} cubes",
                    "vertices": int(pt.X.shape[0]), "tets": int(pt.tets.shape[0]),
                    "slave_tris": int(pt.ts.shape[0]), "master_tris": int(pt.tm.shape[0])},
           "pressure": pt.pressure, "young": pt.young, "poisson": pt.poisson, "dhat": pt.dhat, "gap0": pt.gap,
           "runs": []}
    for mortar in (False, True):
        for k in kappas:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = solve(pt, k, mortar=mortar, device=device)
            torch.cuda.synchronize()
            r = {"samples": "clipped mortar" if mortar else "whole triangle", "kappa": k,
                 "seconds": time.perf_counter() - t0, "steps": len(st),
                 "newton_iters": [s.newton_iters for s in st], "converged": all(s.converged for s in st)}
            r.update(errors(pt, x))
            out["runs"].append(r)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-top", type=int, default=4)
    ap.add_argument("--n-bot", type=int, default=6)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = run(a.n_top, a.n_bot)
    for r in res["runs"]:
        print(f"{r['samples']:>15} kappa {r['kappa']:.0e}: sigma_zz err {r['sigma_zz_max_rel_err']:.3e} "
              f"spur {r['sigma_spur']:.3e} newton {r['newton_iters']} {r['seconds']:.2f} s", flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps({k: v for k, v in res.items() if k != "runs"}))


if __name__ == "__main__":
    main()
