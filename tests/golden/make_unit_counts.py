"""Oracle-defined unit counts of the benchmark workloads, written to
tests/golden/unit_counts.json.

    python tests/golden/make_unit_counts.py

For each workload: active samples (the oracle's selection: closest opposing
inside hit with 0 < g < dhat, Sec. 4.1 and Eq. (gap)), BSR blocks of the
assembled Hessian (Sec. 4.2, blocks touched by active samples, both
triangles stored), and swept (sample point, master triangle) pairs whose
boxes over the linear motion overlap (the step bound's additive CCD pairs,
Eq. (global_ccd)).  These fix the algorithmic bytes of a step and the
denominator of the CCD pair rate independently of the HIP path.  Calls only
the workload generators and the oracle.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
OUT = os.path.join(HERE, "unit_counts.json")


# the sources the counts depend on: the workload generators and the
# whole-triangle oracle (selection, assembly, swept pairs)
SOURCES = ("gen/meshes.py", "gen/workloads.py", "oracle/__init__.py", "oracle/gmcp_oracle.c", "oracle/rule.py")


def source_hash() -> str:
    """Hash of the generator and oracle sources the counts depend on."""
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def counts(envs) -> dict:
    import oracle
    from gen import workloads
    out = dict(n_env=len(envs), Vs=0, Vm=0, Ts=0, Tm=0, samples=0, active=0, nnzb=0, swept=0)
    for w in envs:
        P = workloads.to_problem(w)
        nr = oracle.narrow(P)
        A = oracle.assemble(P, nr.M, project=False)
        out["Vs"] += P.Vs
        out["Vm"] += P.Vm
        out["Ts"] += int(P.ts.shape[0])
        out["Tm"] += int(P.tm.shape[0])
        out["samples"] += P.Ns
        out["active"] += int((nr.M >= 0).sum())
        out["nnzb"] += int(A.row_ptr[-1])
        out["swept"] += oracle.swept_count(P, w.dxs, w.dxm)
        del A, nr
    return out


def main():
    from gen import workloads
    res = {"source_hash": source_hash()}
    t0 = time.time()
    res["large_indent_128x128_sphere"] = counts([workloads.large_indent()])
    res["large_indent_128x128_letter"] = counts([workloads.large_indent(seed=22, indenter="letter")])
    res["batched_256_envs"] = counts(workloads.batched().envs)
    res["seconds"] = round(time.time() - t0, 1)
    with open(OUT, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
