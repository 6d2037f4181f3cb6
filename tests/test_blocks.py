"""Function-block offload of Python programs, host side: blocks found by the
called routine's name, the rewrite that routes them through a dispatcher, and
the trial procedure (each block alone, then combinations of the faster ones),
with stand-in routines so that no GPU is needed."""

import os
import time

import numpy as np
import pytest

from paper_2011_03602_amd import blocks as fb
from paper_2011_03602_amd.frontend import FrontendError

HERE = os.path.dirname(os.path.abspath(__file__))
MLP = open(os.path.join(HERE, "programs", "mlp.py")).read()


def args(n=24, seed=0):
    rng = np.random.default_rng(seed)
    return {"x": rng.standard_normal((n, 16)), "w1": rng.standard_normal((16, 32)),
            "w2": rng.standard_normal((32, 8)), "w3": rng.standard_normal((8, 4))}


def test_blocks_found_by_called_name():
    prog = fb.analyse_blocks(MLP)
    assert [(b.name, b.routine) for b in prog.blocks] == [
        ("numpy.matmul", "gemm_f32"), ("operator @", "gemm_f32"), ("numpy.dot", "gemm_f32")]
    assert [b.line for b in prog.blocks] == [8, 9, 10]


def test_host_gene_is_the_program():
    a = args()
    ns = {}
    exec(MLP, ns)
    want = ns["mlp"](**a)
    got = fb.compile_blocks(fb.analyse_blocks(MLP), 0)(**a)
    assert np.array_equal(got, want)


def test_each_block_routes_through_its_routine():
    calls = []

    def fake(a, b):
        calls.append((a.shape, b.shape))
        return np.matmul(a, b)

    prog = fb.analyse_blocks(MLP)
    fn = fb.compile_blocks(prog, 0b101, {"gemm_f32": fake})
    fn(**args())
    assert calls == [((24, 16), (16, 32)), ((24, 8), (8, 4))]


def test_unknown_calls_are_no_blocks_and_bad_arity_is_refused():
    src = "import numpy as np\n\ndef f(a, b):\n    return np.add(a, b)\n"
    assert fb.analyse_blocks(src).blocks == []
    with pytest.raises(FrontendError):
        fb.analyse_blocks("import numpy as np\n\ndef f(a, b):\n    return np.matmul(a, b, out=None)\n")


def _slow_host(delay):
    def run(a, b):
        time.sleep(delay)
        return np.matmul(a, b)
    return run


def test_trials_keep_the_faster_blocks_and_their_combination():
    prog = fb.analyse_blocks(MLP)
    hosts = {name: _slow_host(0.03) for name in fb.HOST_ROUTINES}
    # block 0 and 2 run faster "offloaded", block 1's offloaded form is slower
    def routine(a, b):
        if a.shape[1] == 32:   # block 1: h @ w2
            time.sleep(0.06)
        return np.matmul(a, b)

    res = fb.trial_blocks(prog, args(), repeats=1, host_routines=hosts, gpu_routines={"gemm_f32": routine})
    genes = [t.gene for t in res["trials"]]
    assert genes == [0b000, 0b001, 0b010, 0b100, 0b101]   # alone each, then the pair that sped up
    assert res["faster_alone"] == [0, 2]
    assert res["best"].gene == 0b101 and res["best"].status == "ok"


def test_trials_score_wrong_and_unbuildable_blocks_as_infinite():
    prog = fb.analyse_blocks(MLP)

    def wrong(a, b):
        return np.matmul(a, b) + 1.0

    def unbuildable(a, b):
        raise fb.BlockNotBuildable("no")

    res = fb.trial_blocks(prog, args(), repeats=1, gpu_routines={"gemm_f32": wrong})
    assert all(t.status == "wrong" for t in res["trials"] if t.gene) and res["best"].gene == 0
    res = fb.trial_blocks(prog, args(), repeats=1, gpu_routines={"gemm_f32": unbuildable})
    assert all(t.status == "not buildable" for t in res["trials"] if t.gene) and res["best"].gene == 0


def test_program_driver_tries_blocks_then_loops():
    from paper_2011_03602_amd.offload import offload_program

    rep = offload_program(MLP, args(), block_repeats=1, gpu_routines={"gemm_f32": np.matmul})
    assert len(rep["blocks"]["found"]) == 3 and rep["blocks"]["best_gene"] in range(8)
    assert rep["loops"]["offloadable"] is False and "iteration loop" in rep["loops"]["reason"]
    relax = open(os.path.join(HERE, "programs", "relax.py")).read()
    rep = offload_program(relax, {}, search_loops=False)
    assert rep["blocks"] is None
    assert rep["loops"]["offloadable"] and rep["loops"]["gene_bits"] == 9
    assert rep["loops"]["binding"]["u"] == "p"
