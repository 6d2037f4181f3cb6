"""The Python front end (a second source language on the same boundary):
loop and variable analysis, the offload screen, binding by what the nests
compute, plans through the library's planner, and runs of the all-CPU gene
against the program itself, interpreted. No GPU is touched."""

import os

import numpy as np
import pytest

import paper_2011_03602_amd as ofl
import synth
from helpers import OMEGA, TOL_GOSA_F32, TOL_P_F32, p_rel_err, rel_err
from paper_2011_03602_amd import frontend as fe

HERE = os.path.dirname(os.path.abspath(__file__))
RELAX = open(os.path.join(HERE, "programs", "relax.py")).read()
# the program's own names for the library's arrays
NAMES = {"a0": "e", "a1": "n_", "a2": "t", "a3": "diag", "b0": "xy", "b1": "yz", "b2": "xz", "c0": "w_",
         "c1": "s_", "c2": "b_", "bnd": "mask", "wrk1": "src", "p": "u", "wrk2": "nxt"}


def program_args(arrays, steps, dtype=np.float32):
    args = {NAMES[k]: np.array(v, dtype=dtype) for k, v in arrays.items()}
    args.update(steps=steps, w=float(OMEGA))
    return args


def test_analysis_binds_by_what_the_nests_compute():
    prog = fe.analyse(RELAX)
    assert prog.binding == {v: k for k, v in NAMES.items()}
    assert prog.symbols == {"omega": "w", "gosa": "err"}
    assert prog.live_after == ["u"] and prog.returns == ["err", "u"]
    assert [n.name for n in prog.nests] == ["S", "R", "C"]
    fe.check_against_library(prog)


def test_screen_and_loop_table():
    prog = fe.analyse(RELAX)
    assert prog.loop_table() == [(-1, -1, 0)] + [(n, lev, 1) for n in range(3) for lev in range(3)]
    it = prog.loops[prog.iter_loop]
    assert (it.var, it.parallel) == ("step", False) and "across trips of step" in it.reason


SCREEN_CASES = [
    # (source, [(var, parallel)])
    ("def f(a, b, n):\n    for i in range(1, n):\n        a[i] = a[i - 1] + b[i]\n", [("i", False)]),
    ("def f(a, b, n):\n    for i in range(n):\n        a[i] = b[i] * 2\n", [("i", True)]),
    ("def f(a, n):\n    s = 0.0\n    for i in range(n):\n        s += a[i]\n    return s\n", [("i", True)]),
    ("def f(a, n):\n    s = 1.0\n    for i in range(n):\n        s = s * a[i]\n    return s\n", [("i", False)]),
    ("def f(a, b, n):\n    for i in range(n):\n        t = b[i] + 1\n        a[i] = t * t\n", [("i", True)]),
    ("def f(a, n, m):\n    for j in range(m):\n        for i in range(n):\n            a[j, i] = a[j, i] + 1\n",
     [("j", True), ("i", True)]),
    ("def f(a, n, m):\n    for j in range(1, m):\n        for i in range(n):\n            a[j, i] = a[j - 1, i]\n",
     [("j", False), ("i", True)]),
]


@pytest.mark.parametrize("src,want", SCREEN_CASES)
def test_offload_screen(src, want):
    assert [(v, ok) for v, _, ok, _ in fe.screen(src)] == want


@pytest.mark.parametrize("mode", [ofl.OFL_XFER_HOISTED, ofl.OFL_XFER_PER_ITER])
@pytest.mark.parametrize("mask", range(8))
def test_plans_from_the_analysis_equal_the_library_plans(mask, mode):
    prog = fe.analyse(RELAX)
    xs, names = prog.plan(mask, mode, 3)
    lib_xs, _, _ = ofl.ofl_plan(mask, mode, 3, True)
    ids = fe.library_ids(prog)
    renamed = [(it, n, w, ids[names[a]], d) for it, n, w, a, d in xs]
    assert sorted(renamed) == sorted(lib_xs)


def test_all_cpu_gene_matches_the_program_run_as_python():
    arrays = synth.make_problem(7, 6, 5, seed=4)
    want = fe.run_python(RELAX, program_args(arrays, 3, np.float64))
    prog = fe.analyse(RELAX)
    args = program_args(arrays, 3)
    err, u = fe.offload(prog, args, gene=0)
    assert u is args["u"]                      # written back in place
    assert p_rel_err(u, want[1]) <= TOL_P_F32
    assert rel_err(err, want[0]) <= TOL_GOSA_F32


def _variant(old, new, count=1):
    assert RELAX.count(old) >= 1
    return RELAX.replace(old, new, count)


REJECTED = {
    "sign of a cross term": _variant("- u[z + 1, y, x - 1] + u[z - 1, y, x - 1]", "+ u[z + 1, y, x - 1] + u[z - 1, y, x - 1]"),
    "gauss-seidel": _variant("nxt[z, y, x] = u[z, y, x] + w * upd", "u[z, y, x] = u[z, y, x] + w * upd"),
    "bounds": _variant("for x in range(1, ni - 1):", "for x in range(0, ni):"),
    "residual restarts once": _variant("    for step in range(steps):\n        err = 0.0\n",
                                       "    err = 0.0\n    for step in range(steps):\n"),
    "stored shifted": _variant("nxt[z, y, x] = u[z, y, x]", "nxt[z, y, x + 1] = u[z, y, x]"),
    "missing term": _variant(" + t[z, y, x] * u[z + 1, y, x]", ""),
    "while": RELAX.replace("    return err, u", "    while False:\n        pass\n    return err, u"),
}


@pytest.mark.parametrize("name", sorted(REJECTED))
def test_programs_that_are_not_the_library_program_are_rejected(name):
    with pytest.raises(fe.FrontendError):
        fe.analyse(REJECTED[name])
