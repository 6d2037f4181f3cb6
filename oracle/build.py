"""Build the FP64 oracle as shared libraries (plain C, gcc, no fast-math).

liboracle.so is the oracle the tests use: one host thread. liboracle_omp.so
is the same oracle.c built with -fopenmp, which runs the loops over k on all
host cores and gives bit-identical results; the benchmark times it as the
all-cores CPU baseline.

Test infrastructure: the product library never links or loads either.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

_COMMON = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]


def _compile(out: str, extra: list, verbose: bool) -> str:
    tmp = out + ".tmp"
    cmd = _COMMON + extra + ["-o", tmp, os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)  # a reader never sees a half-written library
    return out


def build(verbose: bool = False) -> str:
    _compile(LIB_OMP, ["-fopenmp"], verbose)
    return _compile(LIB, ["-Wno-unknown-pragmas"], verbose)


if __name__ == "__main__":
    print(build(verbose=True))
