"""Build the FP64 oracle shared library (test infrastructure only).

    python -m oracle.build

Compiles oracle/gmcp_oracle.c with gcc (-O2 -fopenmp, portable code) into
oracle/liboracle.so next to this file.  build_native() compiles a copy
tuned for the machine it runs on (-O3 -march=native -fopenmp) into a
temporary directory, for timing the oracle on that machine's cores.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gmcp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
           "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_native(verbose: bool = False) -> str:
    """-O3 -march=native build for the CPU this runs on (never shipped:
    built where it is timed, since the target CPU may differ from the
    build machine's)."""
    import hashlib
    import tempfile
    with open(SRC, "rb") as fh:
        tag = hashlib.sha256(fh.read()).hexdigest()[:12]
    out = os.path.join(tempfile.gettempdir(), f"gmcp_oracle_native_{tag}_{os.getpid()}.so")
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
           "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
