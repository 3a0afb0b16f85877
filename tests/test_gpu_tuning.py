"""Launch shapes (gmcp_tuning) and the autotuner.

The shapes only move work between blocks and between the two BSR row
tables, so a step under odd shapes - a light-row bound of 32 (more rows in
the heavy table), grids of a few blocks walking long lists, a small query
grid - must reproduce the default step bit for bit; out-of-range shapes are
rejected; the autotuner returns shapes the library accepts and caches them.
"""
import json

import numpy as np
import pytest

from gen import workloads
from gpu_helpers import make_ctx, need_gpu, to_dev

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _step(ctx, xs, xm, dxs, dxm):
    ctx.build_samples(xs)
    A, alpha = ctx.step(xs, xm, dxs, dxm, check=True)
    nb = int(ctx.status().nnzb)
    return (A.energy.clone(), A.grad.clone(), ctx.row_ptr.clone(), ctx.col[:nb].clone(), ctx.val[:nb].clone(),
            alpha.clone())


@pytest.mark.parametrize("workload", ["small", "large"])
def test_shapes_do_not_change_results(workload):
    need_gpu()
    from paper_2605_24339_amd import GMCPError
    w = workloads.small_indent() if workload == "small" else workloads.large_indent(pad_n=64, rule_n=3)
    xs, xm, dxs, dxm = (to_dev(a, torch.float32) for a in (w.xs, w.xm, w.dxs, w.dxm))
    ctx = make_ctx(w, torch.float32)
    ref = _step(ctx, xs, xm, dxs, dxm)
    d = ctx.tuning()
    assert d["light_row_bound"] == 128 and d["light_row_blocks"] == 65536 and d["heavy_row_blocks"] == 2048
    for shapes in (dict(light_row_bound=32, light_row_blocks=7, heavy_row_blocks=3, query_blocks=5),
                   dict(light_row_bound=256, light_row_blocks=262144, heavy_row_blocks=8192, query_blocks=2048)):
        ctx.set_tuning(**shapes)
        assert {k: v for k, v in ctx.tuning().items() if k in shapes} == shapes
        got = _step(ctx, xs, xm, dxs, dxm)
        assert all(torch.equal(a, b) for a, b in zip(ref, got)), shapes
    for bad in (dict(light_row_bound=96), dict(query_blocks=4096), dict(heavy_row_blocks=-1)):
        with pytest.raises(GMCPError):
            ctx.set_tuning(**bad)
    assert ctx.tuning()["light_row_bound"] == 256      # a rejected call changes nothing


def test_autotuner_picks_valid_shapes_and_caches(tmp_path):
    need_gpu()
    from paper_2605_24339_amd import Context, autotune
    w = workloads.small_indent()
    inputs = tuple(to_dev(a, torch.float32) for a in (w.xs, w.xm, w.dxs, w.dxm))

    def make(cells):
        return Context.single(w.ts, w.tm, w.xs.shape[0], w.xm.shape[0], rule_n=w.rule_n, kappa=w.kappa,
                              dhat=w.dhat, delta_T=w.delta_T, cell=cells[0], dtype=torch.float32)

    cache = str(tmp_path / "tune.json")
    cells, tuning, table = autotune.tune(make, [w], inputs, reps=3, cache=cache)
    assert set(tuning) <= set(autotune.SHAPES)
    assert all(v in autotune.SHAPES[k] for k, v in tuning.items())
    assert len(table) == len(autotune.SCALES) + sum(len(v) for v in autotune.SHAPES.values())
    ctx = make(cells)
    ctx.set_tuning(**tuning)
    with open(cache) as fh:
        assert json.load(fh)[autotune.signature([w])]["tuning"] == tuning
    again = autotune.tune(make, [w], inputs, reps=3, cache=cache)
    assert again[0] == cells and again[1] == tuning
    assert np.isfinite(list(table.values())).all()
