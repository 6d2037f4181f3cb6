"""Address and undefined-behaviour sanitizers over the library's host code.

The host sources are compiled with g++ (-fsanitize=address,undefined) with
stub launchers in place of the device kernels, linked to a C program that
drives every host path of the interface (tests/csrc/abi_check.c), and run.
Host code only: no GPU code is built with a sanitizer."""

import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_03602_amd", "csrc")
HOST_SOURCES = ["grid.cpp", "cpu_nests.cpp", "batch.cpp", "tune.cpp", "blocks.cpp"]
ROCM = "/opt/rocm"


@pytest.mark.skipif(not shutil.which("g++") or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
                    reason="needs g++ and the HIP headers")
def test_host_code_under_asan_and_ubsan():
    flags = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    inc = ["-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{ROOT}/include", f"-I{CSRC}"]
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for src in HOST_SOURCES + ["stubs"]:
            path = os.path.join(ROOT, "tests", "csrc", "kernel_stubs.cpp") if src == "stubs" else os.path.join(CSRC, src)
            obj = os.path.join(d, os.path.basename(path) + ".o")
            subprocess.run(["g++", "-std=c++17", *flags, *inc, "-c", path, "-o", obj], check=True)
            objs.append(obj)
        main_obj = os.path.join(d, "abi_check.o")
        subprocess.run(["gcc", "-std=c11", *flags, f"-I{ROOT}/include", "-c",
                        os.path.join(ROOT, "tests", "csrc", "abi_check.c"), "-o", main_obj], check=True)
        exe = os.path.join(d, "abi_check")
        subprocess.run(["g++", *flags, "-o", exe, main_obj, *objs, f"-L{ROCM}/lib", "-lamdhip64", "-lpthread",
                        f"-Wl,-rpath,{ROCM}/lib"], check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
                   HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
        res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert res.returncode == 0, res.stdout + res.stderr
        assert "all host paths ok" in res.stdout
