"""Compile the C oracle into ``oracle/liboracle.so`` with gcc.

Test infrastructure only.  Flags: -O2 -ffp-contract=off (no fused
multiply-add, so the oracle rounds exactly as its source reads), no
-ffast-math, no OpenMP.

A second library, ``oracle/liboracle_omp.so``, is the complex128 part of the
same source built with -fopenmp -DOR_OMP (threaded row and element-wise
loops, per-thread sums): it is used only to time the oracle on all host
cores.
"""

from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")
SOURCES = ["krylov.c", "refine.c", "oracle.h"]
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-std=c11", "-Wall", "-Wextra", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    cc = os.environ.get("CC", "gcc")
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        units = [
            ("krylov.c", ["-DOR_REAL=double", "-DOR_PFX=z"], "krylov_z.o"),
            ("krylov.c", ["-DOR_REAL=float", "-DOR_PFX=c"], "krylov_c.o"),
            ("refine.c", [], "refine.o"),
        ]
        for src, defs, obj in units:
            out = os.path.join(tmp, obj)
            cmd = [cc, *CFLAGS, *defs, "-c", os.path.join(HERE, src), "-o", out]
            if verbose:
                print(" ".join(cmd))
            subprocess.run(cmd, check=True)
            objs.append(out)
        tmp_lib = LIB + ".tmp"
        subprocess.run([cc, "-shared", "-o", tmp_lib, *objs, "-lm"], check=True)
        os.replace(tmp_lib, LIB)
        out = os.path.join(tmp, "krylov_omp.o")
        cmd = [cc, *CFLAGS, "-fopenmp", "-DOR_OMP", "-DOR_REAL=double", "-DOR_PFX=z", "-c",
               os.path.join(HERE, "krylov.c"), "-o", out]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        tmp_lib = LIB_OMP + ".tmp"
        subprocess.run([cc, "-shared", "-fopenmp", "-o", tmp_lib, out, "-lm"], check=True)
        os.replace(tmp_lib, LIB_OMP)
    return LIB


def stale() -> bool:
    if not (os.path.exists(LIB) and os.path.exists(LIB_OMP)):
        return True
    t = min(os.path.getmtime(LIB), os.path.getmtime(LIB_OMP))
    return any(os.path.getmtime(os.path.join(HERE, s)) > t for s in SOURCES)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
