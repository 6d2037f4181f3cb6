"""The entry point that allocates nothing, ofl_jacobi_run_static, against the
allocating ofl_jacobi_run on the same grid, tile and fusion, through the C
interface.

Both run the fused iteration with the same kernels and the same fixed-order
residual sum; only where the sweep's per-wave partials live differs (the
library's static device array against a buffer it allocates). So p must be
bitwise equal and the residual exactly equal, and both must meet the FP32 bars
against the FP64 oracle. The static entry point is called twice in a row, the
second time on a smaller grid, whose sweep reuses a prefix of the partials the
first call left behind; and twice on one grid, which must equal one allocating
run of the summed length. A sweep that needs more partials than the array
holds is refused with EINVAL before any work.
"""

import sys

import numpy as np
import pytest

import oracle
import paper_2011_03602_amd as ofl
import synth
from helpers import OMEGA, TOL_BF16, TOL_GOSA_F32, TOL_P_F32, boundary_equal, p_rel_err, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, skipped there
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="needs a GPU")]

FUSE_ALL = ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP
# first call, then a smaller one; both span several tiles with ragged tails
SHAPES = [((150, 97, 70), 7), ((41, 23, 19), 5)]


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def run(a, fmt, fusion, iters_list, static):
    g = ofl.Grid(a, coef_format=fmt, torch_memory=True)
    ofl.ofl_set_fusion(g.handle, fusion)
    ofl.ofl_set_offload_mask(g.handle, ofl.OFL_MASK_ALL_GPU, ofl.OFL_XFER_HOISTED)
    ofl.ofl_data_enter(g.handle)
    fn = ofl.ofl_jacobi_run_static if static else ofl.ofl_jacobi_run
    gosa = [fn(g.handle, n, OMEGA) for n in iters_list]
    ofl.ofl_data_exit(g.handle)
    s = ofl.ofl_get_stats(g.handle)
    assert list(s.gpu_nests) == [sum(iters_list)] * 3
    p = g.p.copy()
    g.close()
    return p, gosa[-1]


@pytest.mark.parametrize("fusion", [ofl.OFL_FUSE_RESIDUAL, FUSE_ALL], ids=["fuse_r", "fuse_all"])
@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET], ids=["f32", "bf16_offset"])
def test_static_matches_allocating_on_two_calls(fmt, fusion):
    for shape, iters in SHAPES:
        say("static vs allocating", shape, "x", iters, "format", fmt, "fusion", fusion)
        a = synth.make_problem(*shape)
        p_ref, g_ref = run(a, fmt, fusion, [iters], static=False)
        p, g = run(a, fmt, fusion, [iters], static=True)
        assert np.array_equal(p, p_ref), shape
        assert g == g_ref, (shape, g, g_ref)
        p_o, g_o = oracle.jacobi(a, iters, float(OMEGA))
        tol_p, tol_g = (TOL_P_F32, TOL_GOSA_F32) if fmt == ofl.OFL_COEF_F32 else (TOL_BF16, TOL_BF16)
        assert p_rel_err(p, p_o) <= tol_p and rel_err(g, g_o) <= tol_g, shape
        assert boundary_equal(p, a["p"])


def test_static_calls_in_a_row_equal_one_run():
    a = synth.make_problem(97, 61, 45)
    say("static 3 + 4 iterations vs allocating 7")
    p_ref, g_ref = run(a, ofl.OFL_COEF_F32, FUSE_ALL, [7], static=False)
    p, g = run(a, ofl.OFL_COEF_F32, FUSE_ALL, [3, 4], static=True)
    assert np.array_equal(p, p_ref) and g == g_ref


def test_static_refuses_without_a_data_region():
    a = synth.make_problem(33, 20, 12)
    g = ofl.Grid(a, torch_memory=True)
    ofl.ofl_set_fusion(g.handle, ofl.OFL_FUSE_RESIDUAL)
    ofl.ofl_set_offload_mask(g.handle, ofl.OFL_MASK_ALL_GPU, ofl.OFL_XFER_HOISTED)
    ofl.ofl_jacobi_run(g.handle, 1, OMEGA)  # device state exists, no region
    p_before = g.p.copy()
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_jacobi_run_static(g.handle, 2, OMEGA)
    assert e.value.code == ofl.OFL_ESTATE
    assert np.array_equal(g.p, p_before)
    g.close()


def test_static_refuses_a_sweep_beyond_the_scratch():
    # 66x515x514 with one-point, one-row, one-plane tiles: 2 x 513 x 512 = 525,312
    # waves, two buffers of one partial each: more than the 2^19 the array holds
    shape = (66, 515, 514)
    say("static scratch limit", shape)
    a = {n: np.full(shape[::-1], 0.01, np.float32) for n in ofl.ARRAY_NAMES}
    g = ofl.Grid(a, torch_memory=True)
    ofl.ofl_set_tile(g.handle, ofl.tile(vec=1, rows=1, kchunk=1))
    ofl.ofl_set_fusion(g.handle, ofl.OFL_FUSE_RESIDUAL)
    ofl.ofl_set_offload_mask(g.handle, ofl.OFL_MASK_ALL_GPU, ofl.OFL_XFER_HOISTED)
    ofl.ofl_data_enter(g.handle)
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_jacobi_run_static(g.handle, 1, OMEGA)
    assert e.value.code == ofl.OFL_EINVAL and "static scratch" in ofl.ofl_last_error()
    assert ofl.ofl_get_stats(g.handle).gpu_nests[0] == 0
    ofl.ofl_data_exit(g.handle)
    g.close()
