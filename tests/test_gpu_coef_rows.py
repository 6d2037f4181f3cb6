"""GPU parity of the coefficient arrays' own row pitch.

With 128-byte rows, the twelve coefficient arrays keep i = 0 .. I-2 of each
row (i = I-1 is a boundary column no nest reads), in rows of I-1 rounded up to
128 bytes, while p and wrk2 keep I rounded up to 32 elements. Where I-1 is a
multiple of 32 (FP32) or 64 (bfloat16) elements the coefficient rows are
shorter than p's, and a sweep lane whose vector would start past them reads
the row's last vector instead. Compact rows (row_align 32 here) keep one pitch
for every array, so the same grid laid out both ways must give bitwise the same
p and residual at every vector width and format, whole nests and nests split
into regions alike (the regions upload coefficient sub-boxes row by row).
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

FMTS = [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET, ofl.OFL_COEF_BF16]
FMT_IDS = ["f32", "bf16_offset", "bf16"]
# I-1 a multiple of 32: FP32 coefficient rows shorter than p's; a multiple of
# 64: bfloat16 ones too (33 keeps the bfloat16 rows at p's 64 elements)
WIDTHS = [33, 65, 97, 129, 257, 513]


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def decoded(a, fmt):
    out = dict(a)
    for name in ofl.COEF_NAMES:
        if fmt == ofl.OFL_COEF_BF16:
            out[name] = oracle.bf16_rne(a[name])
        elif fmt == ofl.OFL_COEF_BF16_OFFSET:
            out[name] = oracle.offset_bf16_decode(a[name], oracle.offset_bias(a[name]))
    return out


def run(a, fmt, row_align, iters, tile=None, regions=None):
    g = ofl.Grid(a, coef_format=fmt, row_align=row_align)
    if tile is not None:
        ofl.ofl_set_tile(g.handle, tile)
    if regions is not None:
        mask, levels, mode = regions
        ofl.ofl_set_regions(g.handle, mask, levels, mode)
    gosa = ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
    p = g.p.copy()
    g.close()
    return p, gosa


@pytest.mark.parametrize("fmt", FMTS, ids=FMT_IDS)
@pytest.mark.parametrize("I", WIDTHS)
def test_own_coefficient_rows_equal_one_shared_pitch(I, fmt):
    a = synth.make_problem(I, 9, 7, seed=I)
    for vec in (1, 2, 4, 8):
        say("coefficient rows I", I, "fmt", fmt, "vec", vec)
        t = ofl.tile(vec=vec, rows=2, kchunk=3, flags=ofl.OFL_TILE_NT_LOADS)
        p0, g0 = run(a, fmt, 0, 3, t)
        p1, g1 = run(a, fmt, 32, 3, t)
        assert np.array_equal(p0, p1) and g0 == g1, vec
    p_ref, g_ref = oracle.jacobi(decoded(a, fmt), 3, float(OMEGA))
    assert p_rel_err(p0, p_ref) <= TOL_P_F32 and rel_err(g0, g_ref) <= TOL_GOSA_F32
    assert boundary_equal(p0, a["p"])


@pytest.mark.parametrize("fmt", FMTS[:2], ids=FMT_IDS[:2])
@pytest.mark.parametrize("I", [65, 257])
@pytest.mark.parametrize("mode", [ofl.OFL_XFER_HOISTED, ofl.OFL_XFER_PER_ITER])
@pytest.mark.parametrize("levels", [[1, 1, 1], [2, 0, 2], [2, 2, 2]], ids=["jjj", "kik", "iii"])
def test_own_coefficient_rows_in_regions(I, fmt, mode, levels):
    """Regions per plane or per row: per iteration each region uploads the
    coefficient rows it reads, at the coefficient arrays' own pitch."""
    say("coefficient rows in regions I", I, "fmt", fmt, "mode", mode, "levels", levels)
    a = synth.make_problem(I, 8, 6, seed=3 * I)
    p_whole, g_whole = run(a, fmt, 32, 3)
    p, g = run(a, fmt, 0, 3, regions=(ofl.OFL_MASK_ALL_GPU, levels, mode))
    assert np.array_equal(p, p_whole)
    assert rel_err(g, g_whole) <= 1e-12
    assert boundary_equal(p, a["p"])
