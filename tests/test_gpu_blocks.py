"""Function-block offload on the GPU: the matrix-product blocks of a Python
program replaced by the library's MFMA routine give the program's results
(within the FP32 accumulation bound), and the trials pick a pattern."""

import os
import sys

import numpy as np
import pytest

import oracle
from paper_2011_03602_amd import blocks as fb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, skipped there
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="needs a GPU")]

HERE = os.path.dirname(os.path.abspath(__file__))
MLP = open(os.path.join(HERE, "programs", "mlp.py")).read()


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def mlp_args(n, d, seed=0):
    rng = np.random.default_rng(seed)
    return {"x": rng.uniform(-1, 1, (n, d)).astype(np.float32),
            "w1": rng.uniform(-1, 1, (d, d)).astype(np.float32) / np.sqrt(d),
            "w2": rng.uniform(-1, 1, (d, d)).astype(np.float32) / np.sqrt(d),
            "w3": rng.uniform(-1, 1, (d, 10)).astype(np.float32) / np.sqrt(d)}


@pytest.mark.parametrize("gene", range(8))
def test_every_block_pattern_matches_the_oracle(gene):
    say("blocks gene", gene)
    a = mlp_args(300, 200)
    prog = fb.analyse_blocks(MLP)
    out = fb.compile_blocks(prog, gene)(**a)
    h = np.maximum(oracle.gemm(a["x"], a["w1"]), 0.0)
    h = np.maximum(oracle.gemm(h, a["w2"]), 0.0)
    want = oracle.gemm(h, a["w3"])
    assert np.max(np.abs(out - want)) <= 1e-5 * np.max(np.abs(want)) * 10


def test_trials_pick_a_correct_pattern():
    say("block trials")
    prog = fb.analyse_blocks(MLP)
    res = fb.trial_blocks(prog, mlp_args(2048, 1024), repeats=2)
    assert res["best"].status == "ok"
    assert {t.gene for t in res["trials"]} >= {0, 1, 2, 4}
    assert all(t.status == "ok" for t in res["trials"])
