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


TESTS_CSRC = os.path.join(ROOT, "tests", "csrc")
FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
needs_toolchain = pytest.mark.skipif(
    not shutil.which("g++") or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
    reason="needs g++ and the HIP headers")


def _build(d, extra_sources, driver, libs):
    """Host sources + the given test sources + a C driver, all sanitized."""
    inc = ["-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{ROOT}/include", f"-I{CSRC}"]
    objs = []
    for path in [os.path.join(CSRC, s) for s in HOST_SOURCES] + [os.path.join(TESTS_CSRC, s) for s in extra_sources]:
        obj = os.path.join(d, os.path.basename(path) + ".o")
        subprocess.run(["g++", "-std=c++17", *FLAGS, *inc, "-c", path, "-o", obj], check=True)
        objs.append(obj)
    main_obj = os.path.join(d, driver + ".o")
    subprocess.run(["gcc", "-std=c11", *FLAGS, f"-I{ROOT}/include", "-c", os.path.join(TESTS_CSRC, driver + ".c"),
                    "-o", main_obj], check=True)
    exe = os.path.join(d, driver)
    subprocess.run(["g++", *FLAGS, "-o", exe, main_obj, *objs, *libs, "-lpthread"], check=True)
    return exe


@needs_toolchain
def test_host_code_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = _build(d, ["kernel_stubs.cpp"], "abi_check", [f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
                   HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
        res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert res.returncode == 0, res.stdout + res.stderr
        assert "all host paths ok" in res.stdout


@needs_toolchain
def test_device_errors_are_sticky_and_leak_nothing():
    """Every HIP call of a grid sequence, of a first GPU use and of a batch
    sequence fails in turn, on a stand-in HIP runtime (host memory, no kernels):
    OFL_EDEVICE once the device state exists and on every later call, a usable
    handle before it, and a clean destroy (LeakSanitizer on, and the stand-in
    counts what it handed out)."""
    with tempfile.TemporaryDirectory() as d:
        exe = _build(d, ["hip_stand_in.cpp", "launch_noop.cpp"], "fault_check", [])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
        res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert res.returncode == 0, res.stdout + res.stderr
        assert "device-error paths ok" in res.stdout
        print(res.stdout)
