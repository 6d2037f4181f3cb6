"""GPU parity of the sweep at 8 points per lane (tile.vec = 8): each wave owns
two rows of 256 points, one per half-wave, so every coefficient load is one
16-byte vector per lane in the bfloat16 formats (two in FP32).

Every point is computed with the same arithmetic in the same order as at 4
points per lane, and the residual and copy-back run their 4-point kernels, so
p and the residual must be bitwise equal to the vec-4 run on the same grid;
each run is also checked against the FP64 oracle (FP32 bars, and 1e-3 for the
bfloat16-offset storage against the oracle on the FP32 inputs). Shapes cover
several i-tiles with ragged ends, an odd count of interior rows (the last
wave's second half-wave then has no row and must store nothing), chunk and
row-block tails, and the degenerate grids with one interior point per axis.
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

FMTS = [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET, ofl.OFL_COEF_BF16]
FMT_IDS = ["f32", "bf16_offset", "bf16"]
FUSE_ALL = ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def run(a, iters, tile, fmt=ofl.OFL_COEF_F32, fusion=0, row_align=0):
    g = ofl.Grid(a, coef_format=fmt, row_align=row_align)
    ofl.ofl_set_tile(g.handle, tile)
    if fusion:
        ofl.ofl_set_fusion(g.handle, fusion)
    gosa = ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
    p = g.p.copy()
    g.close()
    return p, gosa


def decoded(a, fmt):
    out = dict(a)
    for name in ofl.COEF_NAMES:
        if fmt == ofl.OFL_COEF_BF16:
            out[name] = oracle.bf16_rne(a[name])
        elif fmt == ofl.OFL_COEF_BF16_OFFSET:
            out[name] = oracle.offset_bf16_decode(a[name], oracle.offset_bias(a[name]))
    return out


def check_oracle(a, fmt, p, gosa, iters):
    """FP32 bars against the oracle on the inputs the kernel reads (decoded
    bfloat16 for the stored formats), and 1e-3 on the FP32 inputs for the
    offset format."""
    p_ref, g_ref = oracle.jacobi(decoded(a, fmt), iters, float(OMEGA))
    assert p_rel_err(p, p_ref) <= TOL_P_F32 and rel_err(gosa, g_ref) <= TOL_GOSA_F32
    if fmt == ofl.OFL_COEF_BF16_OFFSET:
        p32, g32 = oracle.jacobi(a, iters, float(OMEGA))
        assert p_rel_err(p, p32) <= TOL_BF16 and rel_err(gosa, g32) <= TOL_BF16
    assert boundary_equal(p, a["p"])


VEC8_TILES = [
    dict(rows=1, kchunk=1, flags=0),
    dict(rows=2, kchunk=2, flags=ofl.OFL_TILE_NT_LOADS),
    dict(rows=3, kchunk=5, flags=ofl.OFL_TILE_NT_LOADS | ofl.OFL_TILE_NT_STORES),
    dict(rows=4, kchunk=2, flags=3),
    dict(rows=4, kchunk=64, flags=ofl.OFL_TILE_PREFETCH),
    dict(rows=8, kchunk=3, flags=7),
    dict(rows=4, kchunk=4, flags=ofl.OFL_TILE_XCD_REMAP | 3),
    dict(rows=5, kchunk=1024, flags=1),
]


@pytest.fixture(scope="module")
def wide():
    # 600 points along i: three i-tiles of 256 with a ragged last one; 17
    # interior rows: the last wave of a row block has one row
    return synth.make_problem(600, 19, 23, seed=8)


@pytest.mark.parametrize("fmt", FMTS, ids=FMT_IDS)
@pytest.mark.parametrize("t", VEC8_TILES, ids=lambda t: f"r{t['rows']}k{t['kchunk']}f{t['flags']}")
def test_vec8_tiles_equal_vec4_and_oracle(wide, t, fmt):
    say("600x19x23 x4 vec 8 tile", t, "format", fmt)
    a = wide
    p8, g8 = run(a, 4, ofl.tile(vec=8, **t), fmt)
    p4, g4 = run(a, 4, ofl.tile(vec=4, **t), fmt)
    assert np.array_equal(p8, p4) and g8 == g4
    check_oracle(a, fmt, p8, g8, 4)


@pytest.mark.parametrize("dims", [(3, 3, 3), (3, 5, 4), (4, 3, 3), (5, 3, 7), (258, 3, 3), (259, 4, 5), (257, 6, 3),
                                  (513, 3, 4), (66, 5, 4), (9, 8, 6)])
@pytest.mark.parametrize("fmt", FMTS, ids=FMT_IDS)
def test_vec8_edge_shapes(dims, fmt):
    say("edge", dims, "vec 8 format", fmt)
    a = synth.make_problem(*dims, seed=sum(dims) + 1)
    for rows, kchunk in ((1, 1), (2, 2), (3, 5)):
        p8, g8 = run(a, 3, ofl.tile(vec=8, rows=rows, kchunk=kchunk, flags=1), fmt)
        p4, g4 = run(a, 3, ofl.tile(vec=4, rows=rows, kchunk=kchunk, flags=1), fmt)
        assert np.array_equal(p8, p4) and g8 == g4, (rows, kchunk)
        check_oracle(a, fmt, p8, g8, 3)


@pytest.mark.parametrize("fmt", FMTS[:2], ids=FMT_IDS[:2])
@pytest.mark.parametrize("fusion", [ofl.OFL_FUSE_RESIDUAL, ofl.OFL_FUSE_COPYBACK_SWAP, FUSE_ALL],
                         ids=["fuse_r", "swap", "fuse_all"])
def test_vec8_fused_forms(wide, fmt, fusion):
    say("vec 8 fused", fusion, "format", fmt)
    a = wide
    t = ofl.tile(vec=8, rows=4, kchunk=2, flags=3)
    p_plain, g_plain = run(a, 5, t, fmt)
    p, g = run(a, 5, t, fmt, fusion=fusion)
    assert np.array_equal(p, p_plain)
    assert g == pytest.approx(g_plain, rel=1e-12)  # fused partials are summed in another order
    check_oracle(a, fmt, p, g, 5)


# A k-chunk of 257x66x19 at vec 8 with 4 waves per work-group holds 1 i-tile x
# 8 row blocks of 8 rows, so the launch takes the XCD band order: it must equal
# the XCD-contiguous order bitwise.
@pytest.mark.parametrize("fmt", FMTS[:2], ids=FMT_IDS[:2])
def test_vec8_band_order_equals_remap_order(fmt):
    a = synth.make_problem(257, 66, 19, seed=66)
    base = dict(vec=8, rows=4, kchunk=4)
    p0, g0 = run(a, 5, ofl.tile(**base, flags=1), fmt)
    p1, g1 = run(a, 5, ofl.tile(**base, flags=1 | ofl.OFL_TILE_XCD_REMAP), fmt)
    assert np.array_equal(p0, p1) and g0 == g1
    check_oracle(a, fmt, p0, g0, 5)


@pytest.mark.parametrize("row_align", [8, 16])
def test_vec8_compact_rows(row_align):
    a = synth.make_problem(45, 29, 23, seed=31)
    t = ofl.tile(vec=8, rows=2, kchunk=3, flags=1)
    p_ref, g_ref = run(a, 4, t)
    p, g = run(a, 4, t, row_align=row_align)
    assert np.array_equal(p, p_ref) and g == g_ref
    check_oracle(a, ofl.OFL_COEF_F32, p, g, 4)


def test_vec8_static_entry_point():
    a = synth.make_problem(300, 40, 30, seed=3)
    t = ofl.tile(vec=8, rows=4, kchunk=2, flags=3)
    out = []
    for static in (False, True):
        g = ofl.Grid(a, coef_format=ofl.OFL_COEF_BF16_OFFSET, torch_memory=True)
        ofl.ofl_set_tile(g.handle, t)
        ofl.ofl_set_fusion(g.handle, FUSE_ALL)
        ofl.ofl_data_enter(g.handle)
        fn = ofl.ofl_jacobi_run_static if static else ofl.ofl_jacobi_run
        x = fn(g.handle, 5, OMEGA)
        ofl.ofl_data_exit(g.handle)
        out.append((g.p.copy(), x))
        g.close()
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


@pytest.mark.parametrize("fmt", FMTS, ids=FMT_IDS)
def test_vec8_257x257x513_in_the_benchmark_configuration(fmt):
    """Full size, two iterations, PyTorch arena and stream inside a data region,
    the default tile with 8 points per lane."""
    say("257x257x513 x2 vec 8 format", fmt)
    a = synth.make_problem(257, 257, 513)
    g = ofl.Grid(a, coef_format=fmt, torch_memory=True)
    t = ofl.ofl_get_tile(g.handle)
    ofl.ofl_set_tile(g.handle, ofl.tile(vec=8, rows=t.rows, kchunk=t.kchunk, flags=t.flags))
    ofl.ofl_data_enter(g.handle)
    x = ofl.ofl_jacobi_run(g.handle, 2, OMEGA)
    ofl.ofl_data_exit(g.handle)
    p = g.p.copy()
    g.close()
    check_oracle(a, fmt, p, x, 2)


def test_vec8_refused_for_batches():
    a = synth.make_problem(40, 20, 10)
    g = ofl.Grid(a)
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_batch_create([g.handle], ofl.tile(vec=8, rows=2, kchunk=2))
    assert e.value.code == ofl.OFL_ENOTSUP
    g.close()
