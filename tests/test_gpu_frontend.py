"""GPU runs of a Python program through the front end: the loop genes it
offloads give the program's own results (interpreted, small grid) and the
oracle's (larger grid), and the loop-gene search runs on the program's data."""

import os
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import OMEGA, TOL_GOSA_F32, TOL_P_F32, p_rel_err, rel_err
from paper_2011_03602_amd import frontend as fe

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, skipped there
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="needs a GPU")]

HERE = os.path.dirname(os.path.abspath(__file__))
RELAX = open(os.path.join(HERE, "programs", "relax.py")).read()
NAMES = {"a0": "e", "a1": "n_", "a2": "t", "a3": "diag", "b0": "xy", "b1": "yz", "b2": "xz", "c0": "w_",
         "c1": "s_", "c2": "b_", "bnd": "mask", "wrk1": "src", "p": "u", "wrk2": "nxt"}


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def program_args(arrays, steps, dtype=np.float32):
    args = {NAMES[k]: np.array(v, dtype=dtype) for k, v in arrays.items()}
    args.update(steps=steps, w=float(OMEGA))
    return args


# genes in program loop order: bits 0-2 the sweep's z, y, x loops, 3-5 the residual's, 6-8 the copy-back's
GENES = {"whole nests": 0b001_001_001, "planes": 0b010_010_010, "rows": 0b100_100_100,
         "mixed": 0b100_010_001, "sweep only, rows": 0b000_000_100, "residual and copy-back": 0b001_001_000}


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("gene", sorted(GENES), ids=str)
def test_offloaded_program_matches_its_python_run(gene, mode):
    say("front end, gene", gene, "mode", mode)
    arrays = synth.make_problem(9, 7, 6, seed=12)
    want = fe.run_python(RELAX, program_args(arrays, 3, np.float64))
    prog = fe.analyse(RELAX)
    args = program_args(arrays, 3)
    stats = []
    err, u = fe.offload(prog, args, GENES[gene], xfer_mode=mode, stats=stats)
    assert p_rel_err(u, want[1]) <= TOL_P_F32 and rel_err(err, want[0]) <= TOL_GOSA_F32
    g = GENES[gene]
    for n in range(3):
        assert stats[0].gpu_nests[n] == (3 if (g >> (3 * n)) & 7 else 0)


def test_offloaded_program_matches_the_oracle_on_a_larger_grid():
    say("front end vs oracle, 70x40x33 x10")
    arrays = synth.make_problem(70, 40, 33, seed=6)
    p_ref, g_ref = oracle.jacobi(arrays, 10, float(OMEGA))
    prog = fe.analyse(RELAX)
    args = program_args(arrays, 10)
    err, u = fe.offload(prog, args, GENES["whole nests"], torch_memory=True)
    assert p_rel_err(u, p_ref) <= TOL_P_F32 and rel_err(err, g_ref) <= TOL_GOSA_F32


def test_search_on_the_programs_data():
    say("front end loop-gene search")
    arrays = synth.make_problem(40, 30, 20, seed=9)
    prog = fe.analyse(RELAX)
    args = program_args(arrays, 3)
    import paper_2011_03602_amd as ofl

    r = fe.search(prog, args, ga=ofl.ga_params(population=6, generations=3, seed=5, repeats=1))
    assert r.gene_bits == 9 and r.best_ms > 0 and r.patterns >= 1
    err, u = fe.offload(prog, args, r.gene)
    p_ref, g_ref = oracle.jacobi(arrays, 3, float(OMEGA))
    assert p_rel_err(u, p_ref) <= TOL_P_F32 and rel_err(err, g_ref) <= TOL_GOSA_F32


def test_program_driver_on_the_gpu():
    say("program driver: blocks then loops")
    import paper_2011_03602_amd as ofl
    from paper_2011_03602_amd.offload import offload_program

    arrays = synth.make_problem(40, 30, 20, seed=2)
    rep = offload_program(RELAX, program_args(arrays, 3), ga=ofl.ga_params(population=6, generations=2, seed=1,
                                                                           repeats=1))
    assert rep["blocks"] is None and rep["loops"]["offloadable"]
    assert rep["loops"]["best_ms"] > 0 and rep["loops"]["gene"] < (1 << 9)
    mlp = open(os.path.join(HERE, "programs", "mlp.py")).read()
    rng = np.random.default_rng(0)
    a = {"x": rng.uniform(-1, 1, (256, 128)).astype(np.float32), "w1": rng.uniform(-1, 1, (128, 128)).astype(np.float32),
         "w2": rng.uniform(-1, 1, (128, 64)).astype(np.float32), "w3": rng.uniform(-1, 1, (64, 8)).astype(np.float32)}
    rep = offload_program(mlp, a, block_repeats=1)
    assert len(rep["blocks"]["found"]) == 3 and all(s == "ok" for _, _, s in rep["blocks"]["trials"])
    assert rep["loops"]["offloadable"] is False


def test_c_program_offloaded_matches_itself_and_the_oracle(tmp_path):
    say("C front end on the GPU")
    from paper_2011_03602_amd import cfront as cf

    src = open(os.path.join(HERE, "programs", "relax.c")).read()
    names = {"a0": "east", "a1": "north", "a2": "top", "a3": "inv_diag", "b0": "cxy", "b1": "cyz", "b2": "cxz",
             "c0": "west", "c1": "south", "c2": "bottom", "bnd": "keep", "wrk1": "rhs", "p": "v"}
    cp = cf.analyse(src)

    def values(arrays, sweeps):
        vals = {names[k]: np.ascontiguousarray(arrays[k], dtype=np.float32).copy() for k in names}
        vals.update(sweeps=sweeps, relax=float(OMEGA))
        return vals

    small = synth.make_problem(12, 9, 8, seed=21)
    ref_vals = values(small, 3)
    res_c = cf.run_c(cp, ref_vals, str(tmp_path))
    for gene in (0b001_001_001, 0b010_100_001, 0b100_010_010):
        vals = values(small, 3)
        res, v = cf.offload(cp, vals, gene)
        assert p_rel_err(v, ref_vals["v"]) <= TOL_P_F32 and rel_err(res, res_c) <= TOL_GOSA_F32
    big = synth.make_problem(70, 40, 33, seed=22)
    p_ref, g_ref = oracle.jacobi(big, 6, float(OMEGA))
    res, v = cf.offload(cp, values(big, 6), 0b001_001_001)
    assert p_rel_err(v, p_ref) <= TOL_P_F32 and rel_err(res, g_ref) <= TOL_GOSA_F32
