"""Seeded random grids x random tiles x random fusion on the GPU.

A tile's occupancy caps the sweep's resident work-groups per CU by an LDS
reservation the kernel never touches, so it changes only timing.

Every point of the sweep is computed by the same fused multiply-adds in the
same order at every tile, vector width and fusion setting, so p must be
bitwise equal to the run with the default tile, and the residual equal up to
its summation order; both runs are checked against the FP64 oracle (on the
decoded inputs for bfloat16 storage) at the FP32 bars. Shapes run from one
interior point per axis to several i-tiles with ragged ends.
"""

import sys

import numpy as np
import pytest

import oracle
import paper_2011_03602_amd as ofl
import synth
from helpers import OMEGA, TOL_GOSA_F32, TOL_P_F32, boundary_equal, p_rel_err, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, skipped there
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="needs a GPU")]

CASES = 32


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def case(seed):
    rng = np.random.default_rng(20110360 + seed)
    I = int(rng.choice([3, 4, 5, int(rng.integers(6, 70)), int(rng.integers(70, 300)), int(rng.integers(300, 700))]))
    J = int(rng.integers(3, 30))
    K = int(rng.integers(3, 30))
    fmt = int(rng.choice([ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET, ofl.OFL_COEF_BF16]))
    vec = int(rng.choice([1, 2, 4, 8]))
    flags = int(rng.integers(0, 32))
    if vec == 8:
        flags &= ~ofl.OFL_TILE_MARCH_J
    tile = dict(vec=vec, rows=int(rng.integers(1, 9)), kchunk=int(rng.choice([1, 2, 3, 5, 8, 64])), flags=flags)
    fusion = int(rng.choice([0, ofl.OFL_FUSE_RESIDUAL, ofl.OFL_FUSE_COPYBACK_SWAP,
                             ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP]))
    iters = int(rng.integers(1, 6))
    # drawn last, so the cases above keep their earlier draws
    tile["occupancy"] = int(rng.choice([0, 0, 1, 2, 3, 4, 8, 16]))
    return (I, J, K), fmt, tile, fusion, iters


def decoded(a, fmt):
    out = dict(a)
    for name in ofl.COEF_NAMES:
        if fmt == ofl.OFL_COEF_BF16:
            out[name] = oracle.bf16_rne(a[name])
        elif fmt == ofl.OFL_COEF_BF16_OFFSET:
            out[name] = oracle.offset_bf16_decode(a[name], oracle.offset_bias(a[name]))
    return out


def run(a, fmt, iters, tile=None, fusion=0):
    g = ofl.Grid(a, coef_format=fmt)
    if tile is not None:
        ofl.ofl_set_tile(g.handle, ofl.tile(**tile))
    if fusion:
        ofl.ofl_set_fusion(g.handle, fusion)
    gosa = ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
    p = g.p.copy()
    g.close()
    return p, gosa


@pytest.mark.parametrize("seed", range(CASES))
def test_random_tile_equals_default_tile_and_oracle(seed):
    shape, fmt, tile, fusion, iters = case(seed)
    say("random case", seed, shape, "fmt", fmt, "tile", tile, "fusion", fusion, "iters", iters)
    a = synth.make_problem(*shape, seed=1000 + seed)
    p, gosa = run(a, fmt, iters, tile, fusion)
    p_ref, gosa_ref = run(a, fmt, iters)
    assert np.array_equal(p, p_ref)
    assert gosa == pytest.approx(gosa_ref, rel=1e-12, abs=1e-300)
    po, go = oracle.jacobi(decoded(a, fmt), iters, float(OMEGA))
    assert p_rel_err(p, po) <= TOL_P_F32
    if go != 0.0:
        assert rel_err(gosa, go) <= TOL_GOSA_F32
    assert boundary_equal(p, a["p"])


@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET])
def test_occupancy_caps_leave_results_bitwise_unchanged(fmt):
    """Every cap from one work-group per CU (half of a CU's LDS reserved per
    work-group) to 16, plain and fused: p and the residual (summed in a fixed
    order either way) bitwise equal to the uncapped run."""
    a = synth.make_problem(300, 40, 30, seed=77)
    base = dict(vec=4, rows=4, kchunk=2, flags=ofl.OFL_TILE_NT_LOADS | ofl.OFL_TILE_NT_STORES)
    for fusion in (0, ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP):
        p0, g0 = run(a, fmt, 4, dict(base, occupancy=0), fusion)
        for occ in (1, 2, 3, 4, 5, 8, 16):
            say("occupancy", occ, "fmt", fmt, "fusion", fusion)
            p, g = run(a, fmt, 4, dict(base, occupancy=occ), fusion)
            assert np.array_equal(p, p0) and g == g0, occ
