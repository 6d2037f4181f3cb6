"""GPU parity at the workload's own configurations, each against one FP64
oracle run shared by every form it checks (the result-match rule of Sec.
4.2.2: a pattern whose results differ from the original program's is not
kept):

* 129x129x257, 200 iterations: every offload gene x both transfer placements;
* 257x257x513, 100 iterations: FP32 with the FP64 and the compensated-FP32
  residual, the bfloat16-offset and plain bfloat16 storage with both residual
  sums, and the fused forms, in the benchmark's launch configuration (PyTorch
  arena and stream, inside a data region, the default tile);
* 64 uneven grids in the benchmark's batch configuration (compact rows,
  packed where it pays, the default batch tile), plain and fused, FP32 and
  bfloat16-offset: every grid for 10 iterations, and a fixed subset of eight
  grids for the benchmark's full 100.

Bars (relative, max-norm over the interior for p): FP32 p <= 1e-5 and residual
<= 1e-4 against the oracle on the same FP32 inputs; bfloat16 storage and
batched bfloat16 <= 1e-3 against the oracle on the FP32 inputs, and the FP32
bars against the oracle on the decoded bfloat16 inputs (which isolates the
arithmetic from the storage rounding). Plain bfloat16 misses the 1e-3 bar on
the FP32 inputs (about 2e-2, the reason the benchmark reports the offset
form); it is held to the FP32 bars on its decoded inputs.
"""

import sys

import numpy as np
import pytest

import oracle
import paper_2011_03602_amd as ofl
import synth
from helpers import OMEGA, TOL_BF16, TOL_GOSA_F32, TOL_P_F32, boundary_equal, p_rel_err, rel_err

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

if not torch.cuda.is_available():  # collected on CPU hosts, skipped there
    pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.skip(reason="needs a GPU")]

FUSE_ALL = ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def check(a, p, gosa, ref, tol_p, tol_g, what):
    pe, ge = p_rel_err(p, ref[0]), rel_err(gosa, ref[1])
    say(f"  {what}: p rel {pe:.2e} (bar {tol_p:g}), gosa rel {ge:.2e} (bar {tol_g:g})")
    assert pe <= tol_p, f"{what}: p rel err {pe:.3e}"
    assert ge <= tol_g, f"{what}: gosa rel err {ge:.3e}"
    assert boundary_equal(p, a["p"]), what


def decoded(a, fmt):
    """The inputs a reader of the bfloat16 storage sees (coefficients decoded, p as given)."""
    out = dict(a)
    for name in ofl.COEF_NAMES:
        if fmt == ofl.OFL_COEF_BF16:
            out[name] = oracle.bf16_rne(a[name])
        else:
            out[name] = oracle.offset_bf16_decode(a[name], oracle.offset_bias(a[name]))
    return out


# ------------------------------------------- 129x129x257, every gene x placement

MID = (129, 129, 257)
MID_ITERS = 200


@pytest.fixture(scope="module")
def mid():
    say("129x129x257: inputs and the oracle's 200 iterations")
    a = synth.make_problem(*MID)
    return a, oracle.jacobi(a, MID_ITERS, float(OMEGA))


@pytest.mark.parametrize("mode", [ofl.OFL_XFER_PER_ITER, ofl.OFL_XFER_HOISTED], ids=["per_iter", "hoisted"])
@pytest.mark.parametrize("mask", range(8), ids=lambda m: f"gene{m:03b}")
def test_129x129x257_every_gene_and_placement(mid, mask, mode):
    say("129x129x257 x200, gene", format(mask, "03b"), "placement", mode)
    a, ref = mid
    g = ofl.Grid(a, torch_memory=True, pinned=True)
    ofl.ofl_set_offload_mask(g.handle, mask, mode)
    gosa = ofl.ofl_jacobi_run(g.handle, MID_ITERS, OMEGA)
    check(a, g.p, gosa, ref, TOL_P_F32, TOL_GOSA_F32, f"gene {mask:03b} mode {mode}")
    s = ofl.ofl_get_stats(g.handle)
    xs, _, _ = ofl.ofl_plan(mask, mode, MID_ITERS, True)
    assert s.h2d_count == sum(1 for x in xs if x[4] == 0)
    assert s.d2h_count == sum(1 for x in xs if x[4] == 1)
    for nest in range(3):
        on_gpu = (mask >> nest) & 1
        assert s.gpu_nests[nest] == (MID_ITERS if on_gpu else 0)
        assert s.cpu_nests[nest] == (0 if on_gpu else MID_ITERS)
    g.close()


# ------------------------------------------------- 257x257x513, 100 iterations

HEAD = (257, 257, 513)
HEAD_ITERS = 100


@pytest.fixture(scope="module")
def head():
    say("257x257x513: generating inputs")
    return synth.make_problem(*HEAD)


@pytest.fixture(scope="module")
def head_ref(head):
    say("257x257x513: the oracle's 100 iterations on the FP32 inputs")
    return oracle.jacobi(head, HEAD_ITERS, float(OMEGA))


@pytest.fixture(scope="module")
def head_ref_offset(head):
    say("257x257x513: the oracle's 100 iterations on the decoded offset-bfloat16 inputs")
    return oracle.jacobi(decoded(head, ofl.OFL_COEF_BF16_OFFSET), HEAD_ITERS, float(OMEGA))


@pytest.fixture(scope="module")
def head_ref_plain(head):
    say("257x257x513: the oracle's 100 iterations on the decoded plain-bfloat16 inputs")
    return oracle.jacobi(decoded(head, ofl.OFL_COEF_BF16), HEAD_ITERS, float(OMEGA))


def run_head(a, fmt, sum_mode=ofl.OFL_SUM_F64, fusion=0):
    """100 iterations as the benchmark runs them: PyTorch arena and stream,
    every nest on the GPU with hoisted transfers, inside a data region, the
    default tile."""
    g = ofl.Grid(a, coef_format=fmt, sum_mode=sum_mode, torch_memory=True)
    if fusion:
        ofl.ofl_set_fusion(g.handle, fusion)
    ofl.ofl_set_offload_mask(g.handle, ofl.OFL_MASK_ALL_GPU, ofl.OFL_XFER_HOISTED)
    ofl.ofl_data_enter(g.handle)
    gosa = ofl.ofl_jacobi_run(g.handle, HEAD_ITERS, OMEGA)
    ofl.ofl_data_exit(g.handle)
    p = g.p.copy()
    s = ofl.ofl_get_stats(g.handle)
    assert list(s.gpu_nests) == [HEAD_ITERS] * 3 and (s.h2d_count, s.d2h_count) == (13, 1)
    g.close()
    return p, gosa


@pytest.mark.parametrize("sum_mode", [ofl.OFL_SUM_F64, ofl.OFL_SUM_KAHAN_F32], ids=["f64_sum", "kahan_sum"])
def test_257x257x513_fp32_100_iterations(head, head_ref, sum_mode):
    say("257x257x513 x100 FP32, residual sum", sum_mode)
    p, gosa = run_head(head, ofl.OFL_COEF_F32, sum_mode)
    check(head, p, gosa, head_ref, TOL_P_F32, TOL_GOSA_F32, "FP32")


def test_257x257x513_fused_fp32_100_iterations(head, head_ref):
    say("257x257x513 x100 FP32 fused")
    p, gosa = run_head(head, ofl.OFL_COEF_F32, fusion=FUSE_ALL)
    check(head, p, gosa, head_ref, TOL_P_F32, TOL_GOSA_F32, "FP32 fused")


@pytest.mark.parametrize("sum_mode", [ofl.OFL_SUM_F64, ofl.OFL_SUM_KAHAN_F32], ids=["f64_sum", "kahan_sum"])
def test_257x257x513_bf16_offset_100_iterations(head, head_ref, head_ref_offset, sum_mode):
    say("257x257x513 x100 bfloat16-offset, residual sum", sum_mode)
    p, gosa = run_head(head, ofl.OFL_COEF_BF16_OFFSET, sum_mode)
    check(head, p, gosa, head_ref, TOL_BF16, TOL_BF16, "bf16-offset vs FP32-input oracle")
    check(head, p, gosa, head_ref_offset, TOL_P_F32, TOL_GOSA_F32, "bf16-offset vs decoded-input oracle")


def test_257x257x513_fused_bf16_offset_100_iterations(head, head_ref, head_ref_offset):
    say("257x257x513 x100 bfloat16-offset fused")
    p, gosa = run_head(head, ofl.OFL_COEF_BF16_OFFSET, fusion=FUSE_ALL)
    check(head, p, gosa, head_ref, TOL_BF16, TOL_BF16, "bf16-offset fused vs FP32-input oracle")
    check(head, p, gosa, head_ref_offset, TOL_P_F32, TOL_GOSA_F32, "bf16-offset fused vs decoded-input oracle")


@pytest.mark.parametrize("sum_mode", [ofl.OFL_SUM_F64, ofl.OFL_SUM_KAHAN_F32], ids=["f64_sum", "kahan_sum"])
def test_257x257x513_bf16_plain_100_iterations(head, head_ref, head_ref_plain, sum_mode):
    say("257x257x513 x100 plain bfloat16, residual sum", sum_mode)
    p, gosa = run_head(head, ofl.OFL_COEF_BF16, sum_mode)
    check(head, p, gosa, head_ref_plain, TOL_P_F32, TOL_GOSA_F32, "bf16-plain vs decoded-input oracle")
    # on the FP32 inputs plain storage is worse than 1e-3 (about 2e-2): recorded, not gated
    say(f"  bf16-plain vs FP32-input oracle: p rel {p_rel_err(p, head_ref[0]):.2e}, "
        f"gosa rel {rel_err(gosa, head_ref[1]):.2e} (reported only)")


# ------------------------------------------------ 64 uneven grids, batched

N_GRIDS = 64
BATCH_ITERS_ALL = 10
BATCH_ITERS_FULL = 100
# eight grids for the full 100 iterations: the two largest, the two smallest
# and four in between (by interior size), fixed by the seeded sizes
FULL_SUBSET = 8


@pytest.fixture(scope="module")
def batch():
    say("64 uneven grids: generating")
    probs = synth.make_batch(N_GRIDS)
    say("64 uneven grids: the oracle's 10 iterations on every grid")
    refs10 = [oracle.jacobi(a, BATCH_ITERS_ALL, float(OMEGA)) for _, a in probs]
    order = sorted(range(N_GRIDS), key=lambda t: synth.interior_points(*probs[t][0]))
    pick = sorted(set(order[:2] + order[-2:] + [order[int(q * (N_GRIDS - 1))] for q in (0.2, 0.4, 0.6, 0.8)]))
    assert len(pick) == FULL_SUBSET
    say("64 uneven grids: the oracle's 100 iterations on grids", pick)
    refs100 = {t: oracle.jacobi(probs[t][1], BATCH_ITERS_FULL, float(OMEGA)) for t in pick}
    return probs, refs10, refs100


def run_batch(probs, fmt, fusion, iters):
    """The benchmark's batch configuration: compact rows (4-element row
    alignment, packed rows where they pay), the default batch tile, one graph
    launch per run, inside the grids' data regions."""
    grids = [ofl.Grid(a, coef_format=fmt, row_align=4) for _, a in probs]
    for g in grids:
        ofl.ofl_data_enter(g.handle)
    b = ofl.ofl_batch_create([g.handle for g in grids])
    ofl.ofl_batch_set_fusion(b, fusion)
    gosa = ofl.ofl_batch_run(b, iters, OMEGA, len(grids))
    ofl.ofl_batch_destroy(b)
    out = []
    for g in grids:
        ofl.ofl_data_exit(g.handle)
        out.append(g.p.copy())
        g.close()
    return out, gosa


@pytest.mark.parametrize("fusion", [0, FUSE_ALL], ids=["plain", "fused"])
@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET], ids=["f32", "bf16_offset"])
def test_batch64_every_grid_10_iterations(batch, fmt, fusion):
    probs, refs10, _ = batch
    say("64 uneven grids x10, format", fmt, "fusion", fusion)
    ps, gosa = run_batch(probs, fmt, fusion, BATCH_ITERS_ALL)
    tol_p, tol_g = (TOL_P_F32, TOL_GOSA_F32) if fmt == ofl.OFL_COEF_F32 else (TOL_BF16, TOL_BF16)
    worst_p = worst_g = 0.0
    for (shape, a), p, x, ref in zip(probs, ps, gosa, refs10):
        pe, ge = p_rel_err(p, ref[0]), rel_err(x, ref[1])
        worst_p, worst_g = max(worst_p, pe), max(worst_g, ge)
        assert pe <= tol_p and ge <= tol_g, (shape, pe, ge)
        assert boundary_equal(p, a["p"]), shape
    say(f"  worst over 64 grids: p rel {worst_p:.2e}, gosa rel {worst_g:.2e}")


@pytest.mark.parametrize("fusion", [0, FUSE_ALL], ids=["plain", "fused"])
@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET], ids=["f32", "bf16_offset"])
def test_batch64_100_iterations_on_a_subset(batch, fmt, fusion):
    probs, _, refs100 = batch
    say("64 uneven grids x100, format", fmt, "fusion", fusion, "checked on grids", sorted(refs100))
    ps, gosa = run_batch(probs, fmt, fusion, BATCH_ITERS_FULL)
    tol_p, tol_g = (TOL_P_F32, TOL_GOSA_F32) if fmt == ofl.OFL_COEF_F32 else (TOL_BF16, TOL_BF16)
    for t, ref in refs100.items():
        shape, a = probs[t]
        check(a, ps[t], gosa[t], ref, tol_p, tol_g, f"grid {t} {shape}")
    for (_, a), p, x in zip(probs, ps, gosa):
        assert np.isfinite(x) and boundary_equal(p, a["p"])
