"""Autotuner for the broad-phase grid.

The one shape parameter that moves the whole step is the grid cell size of
each environment (cells too fine: many empty cells per support prism; too
coarse: many master triangles per cell).  For a workload signature the
tuner times full captured steps (HIP graph replays, events on the stream)
for cell sizes that are multiples of the environment's mean master-edge
length, keeps the fastest, and caches the choice in a JSON file keyed by
the signature (size buckets of pads, rules and indenters).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

SCALES = (0.0, 0.75, 1.0, 1.5, 2.0, 3.0)   # 0.0: the library's automatic size
DEFAULT_CACHE = os.environ.get("GMCP_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "gmcp_autotune.json"))


def mean_edge(x: np.ndarray, tri: np.ndarray) -> float:
    e = np.linalg.norm(x[tri[:, [1, 2, 0]]] - x[tri], axis=2)
    return float(e.mean()) if e.size else 0.0


def signature(envs) -> str:
    """Size buckets (powers of two) of the environments' meshes and rules."""
    b = lambda n: int(2 ** round(math.log2(max(n, 1))))
    keys = sorted({(b(w.ts.shape[0]), b(w.tm.shape[0]), w.rule_n) for w in envs})
    return f"n_env={b(len(envs))};" + ";".join(f"{a}/{c}/{r}" for a, c, r in keys)


def time_graph(g, reps: int = 20) -> float:
    """Median milliseconds of one graph replay."""
    s = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        g.replay()
        b.record(s)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def tune(make_ctx, envs, inputs, scales=SCALES, reps: int = 20, cache: str | None = DEFAULT_CACHE,
         verbose: bool = False):
    """Pick the cell-size scale for these environments.

    make_ctx(cells: list[float]) -> Context; inputs = (xs, xm, dxs, dxm)
    device tensors; envs: the workloads (for edge lengths and the
    signature).  Returns (cells, table) where table maps scale -> ms.
    """
    sig = signature(envs)
    edges = [mean_edge(w.xm, w.tm) for w in envs]
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            known = json.load(fh)
        if sig in known:
            s = known[sig]["scale"]
            return [s * e for e in edges] if s > 0 else [0.0] * len(envs), known[sig]["table"]
    table = {}
    for s in scales:
        cells = [s * e for e in edges] if s > 0 else [0.0] * len(envs)
        ctx = make_ctx(cells)
        ctx.build_samples(inputs[0])
        g = ctx.capture(*inputs)
        g.replay()
        torch.cuda.synchronize()
        table[str(s)] = time_graph(g, reps)
        if verbose:
            print(f"autotune scale {s}: {table[str(s)]:.4f} ms", flush=True)
        del g, ctx
        torch.cuda.empty_cache()
    best = float(min(table, key=table.get))
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        known = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                known = json.load(fh)
        known[sig] = {"scale": best, "table": table}
        with open(cache, "w") as fh:
            json.dump(known, fh, indent=1)
    cells = [best * e for e in edges] if best > 0 else [0.0] * len(envs)
    return cells, table
