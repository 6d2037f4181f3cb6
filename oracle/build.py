"""Build the FP64 oracle as a shared library (plain C, gcc, no fast-math).

Test infrastructure: the product library never links or loads the result.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [
        "gcc", "-O2", "-std=c99", "-fPIC", "-shared",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
        "-o", tmp, os.path.join(HERE, "oracle.c"), "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)  # a reader never sees a half-written library
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
