"""The C front end (a subset of C99): tokenizing, parsing and lowering into the
representation the common analysis reads; binding by what the nests compute;
plans through the library's planner; the all-CPU gene against the original C
program compiled with gcc. No GPU is touched."""

import os
import shutil

import numpy as np
import pytest

import paper_2011_03602_amd as ofl
import oracle
import synth
from helpers import OMEGA, TOL_GOSA_F32, TOL_P_F32, p_rel_err, rel_err
from paper_2011_03602_amd import cfront as cf
from paper_2011_03602_amd import frontend as fe

HERE = os.path.dirname(os.path.abspath(__file__))
RELAX_C = open(os.path.join(HERE, "programs", "relax.c")).read()
# the C program's names for the library's arrays
NAMES = {"a0": "east", "a1": "north", "a2": "top", "a3": "inv_diag", "b0": "cxy", "b1": "cyz", "b2": "cxz",
         "c0": "west", "c1": "south", "c2": "bottom", "bnd": "keep", "wrk1": "rhs", "p": "v"}

needs_gcc = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


def c_values(arrays, sweeps):
    vals = {NAMES[k]: np.ascontiguousarray(arrays[k], dtype=np.float32).copy() for k in NAMES}
    vals.update(sweeps=sweeps, relax=float(OMEGA))
    return vals


def test_parse_lower_and_bind():
    cp = cf.analyse(RELAX_C)
    assert cp.func == "solve" and list(cp.local_arrays) == ["tmp"] and cp.written == ["tmp", "v"]
    assert cp.program.binding == {**{v: k for k, v in NAMES.items()}, "tmp": "wrk2"}
    assert cp.program.symbols == {"omega": "relax", "gosa": "res"}
    assert cp.program.live_after == ["v"]
    fe.check_against_library(cp.program)


@pytest.mark.parametrize("mode", [ofl.OFL_XFER_HOISTED, ofl.OFL_XFER_PER_ITER])
@pytest.mark.parametrize("mask", range(8))
def test_plans_equal_the_library_plans(mask, mode):
    prog = cf.analyse(RELAX_C).program
    xs, names = prog.plan(mask, mode, 2)
    ids = fe.library_ids(prog)
    assert sorted((it, n, w, ids[names[a]], d) for it, n, w, a, d in xs) == sorted(ofl.ofl_plan(mask, mode, 2, True)[0])


@needs_gcc
def test_all_cpu_gene_matches_the_c_program(tmp_path):
    arrays = synth.make_problem(8, 7, 6, seed=3)
    want_vals = c_values(arrays, 3)
    cp = cf.analyse(RELAX_C)
    res_c = cf.run_c(cp, want_vals, str(tmp_path))
    vals = c_values(arrays, 3)
    res, v = cf.offload(cp, vals, gene=0)
    assert v is vals["v"]
    assert p_rel_err(v, want_vals["v"]) <= TOL_P_F32
    assert rel_err(res, res_c) <= TOL_GOSA_F32


@needs_gcc
def test_c_program_with_a_local_array_beyond_the_default_stack(tmp_path):
    # tmp is a 10 MB variable-length array: more than a default 8 MB main-thread stack
    arrays = synth.make_problem(160, 160, 100, seed=4)
    want_vals = c_values(arrays, 1)
    cp = cf.analyse(RELAX_C)
    res_c = cf.run_c(cp, want_vals, str(tmp_path))
    vals = c_values(arrays, 1)
    res, v = cf.offload(cp, vals, gene=0)
    assert p_rel_err(v, want_vals["v"]) <= TOL_P_F32
    # the C program sums its residual in FP32 over 2.5M points; the library sums in FP64
    _, g_ref = oracle.jacobi(arrays, 1, float(OMEGA))
    assert rel_err(res, g_ref) <= TOL_GOSA_F32
    assert rel_err(res_c, g_ref) <= 1e-2


@needs_gcc
def test_run_c_checks_shapes_and_reports_gcc_errors(tmp_path):
    arrays = synth.make_problem(8, 7, 6, seed=3)
    cp = cf.analyse(RELAX_C)
    vals = c_values(arrays, 1)
    vals["rhs"] = np.zeros((6, 7, 9), np.float32)
    with pytest.raises(fe.FrontendError, match="rhs has shape"):
        cf.run_c(cp, vals, str(tmp_path))
    broken = cf.translate(RELAX_C)
    broken.source = RELAX_C.replace("return res;", "return res")
    with pytest.raises(fe.FrontendError, match="gcc failed"):
        cf.run_c(broken, c_values(arrays, 1), str(tmp_path))
    assert list(tmp_path.iterdir()) == []  # the build folder is removed


def _variant(old, new):
    assert RELAX_C.count(old) == 1, old
    return RELAX_C.replace(old, new)


REJECTED = {
    "gauss-seidel": _variant("tmp[z][y][x] = v[z][y][x] + relax * d;", "v[z][y][x] = v[z][y][x] + relax * d;"),
    "sign": _variant("- v[z - 1][y][x + 1] + v[z - 1][y][x - 1]", "+ v[z - 1][y][x + 1] + v[z - 1][y][x - 1]"),
    "call": _variant("float r = (tmp[z][y][x] - v[z][y][x]) / relax;", "float r = fabsf(tmp[z][y][x]) / relax;"),
    "while": _variant("    return res;", "    while (res) res = 0.0f;\n    return res;"),
    "step": _variant("for (int it = 0; it < sweeps; ++it)", "for (int it = 0; it < sweeps; it += 2)"),
    "const written": _variant("const float rhs[nz][ny][nx]", "const float rhs[nz][ny][nx]").replace(
        "tmp[z][y][x] = v[z][y][x] + relax * d;", "tmp[z][y][x] = v[z][y][x] + relax * d;\n"
        "                    rhs[z][y][x] = d;"),
    "bad token": RELAX_C.replace("float res = 0.0f;", "float res = 0.0f; @"),
}


@pytest.mark.parametrize("name", sorted(REJECTED))
def test_programs_that_are_not_the_library_program_are_rejected(name):
    with pytest.raises(fe.FrontendError):
        cf.analyse(REJECTED[name])
