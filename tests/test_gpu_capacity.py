"""Capacity growth: a context created with far too small grid-item,
candidate, active-sample and pair capacities reports each overflow, grows,
and then gives exactly what a context with the default capacities gives
(the same kernels on the same inputs: bitwise equal)."""
import numpy as np
import pytest

from gpu_helpers import need_gpu, run_gpu
from gen import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_growth_from_tiny_capacities():
    need_gpu()
    w = workloads.small_indent()
    ref = run_gpu(w, torch.float32)
    tiny = run_gpu(w, torch.float32, caps={"grid_items": 16, "candidates": 16, "active": 16, "pairs": 16})
    caps = tiny["ctx"].caps
    assert caps["grid_items"] > 16 and caps["candidates"] > 16 and caps["active"] > 16 and caps["pairs"] > 16
    assert tiny["status"].code == 0 and tiny["ccd_status"].code == 0
    for k in ("energy", "grad", "row_ptr", "col", "val", "M", "g", "c1", "c2", "p"):
        assert np.array_equal(ref[k], tiny[k]), k
    assert ref["alpha"] == tiny["alpha"]
