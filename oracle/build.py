"""Compiles ``oracle/matmul.c``, ``oracle/transpose.c`` and ``oracle/madd.c`` into
``oracle/_build/liboracle.so`` with gcc.

Test infrastructure only.  Flags keep IEEE semantics (no fast-math, no FMA
contraction) so the double sums are taken exactly in the written order.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "matmul.c"), os.path.join(HERE, "transpose.c"), os.path.join(HERE, "madd.c"),
           os.path.join(HERE, "jacobi.c"), os.path.join(HERE, "polydiv.c")]
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(s) for s in SOURCES):
        return LIB
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
           "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp] + SOURCES
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True), file=sys.stdout)
