"""Autotuner for the step's shapes: the broad-phase grid cell size and the
launch shapes of the list-walking kernels.

First the grid cell size of each environment (cells too fine: many empty
cells per support prism; too coarse: many master triangles per cell): full
captured steps (HIP graph replays, events on the stream) are timed for cell
sizes that are multiples of the environment's mean master-edge length, plus
the library's automatic size.  Then, on the context with the best cell
size, a coordinate search over the launch shapes (gmcp_tuning): the query's
grid, the light BSR row class bound (the rows processed with small LDS
tables, which sets how many waves fit per CU) and the grids of the light-
and heavy-row kernels, each field in turn over its candidates with the
others at their best so far, every candidate timed on a freshly captured
graph.  Results do not depend on these shapes (the row class bound only
moves rows between two tables of the same arithmetic), so only time
decides.  The choice is cached in a JSON file keyed by the workload
signature (size buckets of pads, rules and indenters).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

SCALES = (0.0, 0.75, 1.0, 1.5, 2.0, 3.0)   # 0.0: the library's automatic size
# candidate values per launch-shape field (0: the library's default)
SHAPES = {
    "light_row_bound": (64, 128, 256),
    "light_row_blocks": (8192, 16384, 65536, 262144),
    "heavy_row_blocks": (512, 2048, 8192),
    "query_blocks": (0, 1024, 1536),
}
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


def _time_ctx(ctx, inputs, reps) -> float:
    g = ctx.capture(*inputs)
    g.replay()
    torch.cuda.synchronize()
    t = time_graph(g, reps)
    del g
    return t


def tune(make_ctx, envs, inputs, scales=SCALES, reps: int = 20, cache: str | None = DEFAULT_CACHE,
         verbose: bool = False, shapes: dict | None = SHAPES):
    """Pick the cell-size scale, then the launch shapes, for these environments.

    make_ctx(cells: list[float]) -> Context; inputs = (xs, xm, dxs, dxm)
    device tensors; envs: the workloads (for edge lengths and the
    signature).  Returns (cells, tuning, table): tuning maps gmcp_tuning
    fields to their chosen values (0 = default; pass it to
    Context.set_tuning), table maps each tried setting to its milliseconds.
    """
    sig = signature(envs)
    edges = [mean_edge(w.xm, w.tm) for w in envs]
    cells_of = lambda s: [s * e for e in edges] if s > 0 else [0.0] * len(envs)
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            known = json.load(fh)
        if sig in known:
            k = known[sig]
            return cells_of(k["scale"]), k.get("tuning", {}), k["table"]
    table = {}
    for s in scales:
        ctx = make_ctx(cells_of(s))
        ctx.build_samples(inputs[0])
        table[f"scale={s}"] = _time_ctx(ctx, inputs, reps)
        if verbose:
            print(f"autotune scale {s}: {table[f'scale={s}']:.4f} ms", flush=True)
        del ctx
        torch.cuda.empty_cache()
    best = min(scales, key=lambda s: table[f"scale={s}"])
    tuning = {}
    if shapes:
        ctx = make_ctx(cells_of(best))
        ctx.build_samples(inputs[0])
        best_ms = table[f"scale={best}"]
        for field, cands in shapes.items():
            for v in cands:
                ctx.set_tuning(**{**tuning, field: v})
                ms = _time_ctx(ctx, inputs, reps)
                table[f"{field}={v}"] = ms
                if verbose:
                    print(f"autotune {field}={v}: {ms:.4f} ms", flush=True)
                if ms < best_ms:
                    best_ms, tuning[field] = ms, v
            ctx.set_tuning(**tuning)
        del ctx
        torch.cuda.empty_cache()
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        known = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                known = json.load(fh)
        known[sig] = {"scale": best, "tuning": tuning, "table": table}
        with open(cache, "w") as fh:
            json.dump(known, fh, indent=1)
    return cells_of(best), tuning, table
