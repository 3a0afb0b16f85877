"""The oracle-defined unit counts stored for the benchmark
(tests/golden/unit_counts.json, written by make_unit_counts.py) are current:
written from the present generator and oracle sources, and the single
large indentation's counts recomputed here agree with them."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_unit_counts as muc  # noqa: E402


def test_stored_counts_are_current():
    with open(muc.OUT) as fh:
        stored = json.load(fh)
    assert stored["source_hash"] == muc.source_hash(), "rerun tests/golden/make_unit_counts.py"
    from gen import workloads
    got = muc.counts([workloads.large_indent()])
    assert got == stored["large_indent_128x128_sphere"]
    b = stored["batched_256_envs"]
    assert b["n_env"] == 256 and b["samples"] > 3e7 and 0 < b["active"] < b["samples"]
