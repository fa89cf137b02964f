"""Build the C++ oracle into ``oracle/liboracle.so`` (g++, OpenMP, FP64) and
its FP32 evaluation into ``oracle/liboracle32.so`` (the same source with
``ORACLE_REAL=float`` and single-precision literals, so every step rounds to
float32).

Compiled with ``-ffp-contract=off`` so the FP32 values that decide integers
(depth bits, projected centres) are evaluated with exactly the rounding the
source spells out.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB32 = os.path.join(HERE, "liboracle32.so")
SRC = os.path.join(HERE, "oracle.cpp")


def _compile(out: str, extra, verbose: bool) -> None:
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter", *extra, SRC, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    _compile(LIB, [], verbose)
    _compile(LIB32, ["-DORACLE_REAL=float", "-fsingle-precision-constant", "-Wdouble-promotion"], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
