"""Marker ranges: a rocprofv3 marker trace of a small offloaded run names the
phases of the offloaded program (transfers by array and direction, nests on
each device, graph launches, a batched run), the ranges the library pushes
with ROCTx. Runs the profiler on a child process."""

import glob
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

if not torch.cuda.is_available() or not shutil.which("rocprofv3"):
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="needs a GPU and rocprofv3")]

PROGRAM = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
import paper_2011_03602_amd as ofl
import synth
omega = np.float32(0.8)
g = ofl.Grid(synth.make_problem(40, 20, 12))
ofl.ofl_jacobi_run(g.handle, 4, omega)                      # all-GPU gene: uploads, nests, a graph
ofl.ofl_set_offload_mask(g.handle, 0b101, ofl.OFL_XFER_PER_ITER)
ofl.ofl_jacobi_run(g.handle, 1, omega)                      # residual on the CPU, per-iteration copies
h = ofl.Grid(synth.make_problem(33, 17, 9), row_align=4)
b = ofl.ofl_batch_create([h.handle])
ofl.ofl_batch_run(b, 2, omega, 1)
ofl.ofl_batch_destroy(b)
print("markers program done", flush=True)
"""


def test_marker_trace_names_the_offloaded_phases():
    with tempfile.TemporaryDirectory() as d:
        prog = os.path.join(d, "prog.py")
        with open(prog, "w") as f:
            f.write(PROGRAM.format(root=ROOT))
        out = os.path.join(d, "out")
        res = subprocess.run(["rocprofv3", "--marker-trace", "--kernel-trace", "--output-format", "csv", "-d", out,
                              "-o", "mk", "--", sys.executable, prog],
                             capture_output=True, text=True, timeout=180, cwd=d, env=dict(os.environ, TMPDIR=d))
        print(res.stdout[-2000:], res.stderr[-2000:], flush=True)
        assert res.returncode == 0 and "markers program done" in res.stdout
        files = glob.glob(os.path.join(out, "**", "*marker*.csv"), recursive=True)
        assert files, os.listdir(out)
        text = "".join(open(f).read() for f in files)
        for name in ("ofl:h2d p", "ofl:h2d a0", "ofl:d2h p", "ofl:gpu sweep", "ofl:gpu residual",
                     "ofl:gpu copy-back", "ofl:graph of iterations", "ofl:cpu residual",
                     "ofl:batch prepare", "ofl:batch graph of iterations"):
            assert name in text, name
