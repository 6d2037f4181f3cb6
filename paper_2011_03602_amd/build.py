"""Build libofl.so (HIP kernels + host runtime) for gfx950, in-tree.

Every source is compiled by hipcc as HIP for gfx950 with packed-FP32
instruction selection turned off; objects go to _build/ and the shared
library lands next to this file, where the Python binding loads it.
"""

from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build", "ofl")
LIB = os.path.join(HERE, "libofl.so")
ARCH = "gfx950"

SOURCES = ["kernels.hip", "gemm.hip", "grid.cpp", "cpu_nests.cpp", "batch.cpp", "tune.cpp", "blocks.cpp", "trace.cpp", "device.cpp"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def source_hash() -> str:
    """First 16 hex digits of a SHA-256 over the library's sources and its
    header: the build identity the tile tuners' measurement file is keyed on."""
    h = hashlib.sha256()
    names = sorted(n for n in os.listdir(CSRC) if n.endswith((".hip", ".cpp", ".hpp")))
    for path in [os.path.join(CSRC, n) for n in names] + [os.path.join(ROOT, "include", "ofl.h")]:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _compile(src: str, verbose: bool, defines=()) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), "-x", "hip", *COMMON, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"compiling {src} failed")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source and link libofl.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    defines = [f'-DOFL_SOURCE_HASH="{source_hash()}"']
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, defines), SOURCES))
    tmp = LIB + ".tmp"
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread",
           f"-L{rocm_lib}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{rocm_lib}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
