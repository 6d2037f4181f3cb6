"""GPU parity: the HIP path (through the C interface) against the FP64 oracle
on the same seeded inputs, element by element over the interior.

Bars: FP32 p max-norm relative error <= 1e-5 and residual relative error <=
1e-4; bfloat16-offset storage and batched forms <= 1e-3 against the oracle
on the FP32 inputs. The boundary layer must come back bitwise unchanged.
"""

import sys

import numpy as np
import pytest

import oracle
import paper_2011_03602_amd as ofl
import synth
from helpers import (OMEGA, TOL_BF16, TOL_GOSA_F32, TOL_P_F32, boundary_equal, p_rel_err, rel_err)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, skipped there
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="needs a GPU")]


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def run_gpu(arrays, iters, mask=ofl.OFL_MASK_ALL_GPU, mode=ofl.OFL_XFER_HOISTED, tile=None, fmt=ofl.OFL_COEF_F32,
            sum_mode=ofl.OFL_SUM_F64, torch_memory=False):
    g = ofl.Grid(arrays, coef_format=fmt, sum_mode=sum_mode, torch_memory=torch_memory)
    ofl.ofl_set_offload_mask(g.handle, mask, mode)
    if tile is not None:
        ofl.ofl_set_tile(g.handle, tile)
    gosa = ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
    return g, gosa


def check_against_oracle(arrays, g, gosa, iters, tol_p=TOL_P_F32, tol_g=TOL_GOSA_F32, ref=None):
    p_ref, g_ref = ref if ref is not None else oracle.jacobi(arrays, iters, float(OMEGA))
    pe, ge = p_rel_err(g.p, p_ref), rel_err(gosa, g_ref)
    assert pe <= tol_p, f"p rel err {pe:.3e}"
    assert ge <= tol_g, f"gosa rel err {ge:.3e}"
    assert boundary_equal(g.p, arrays["p"])
    return pe, ge


# ------------------------------------------------------------ small config


@pytest.mark.parametrize("mask", [ofl.OFL_MASK_ALL_CPU, ofl.OFL_MASK_ALL_GPU])
def test_33x33x65_50_iterations(mask):
    say("33x33x65 x50, mask", mask)
    a = synth.make_problem(33, 33, 65)
    g, gosa = run_gpu(a, 50, mask=mask)
    check_against_oracle(a, g, gosa, 50)
    s = ofl.ofl_get_stats(g.handle)
    if mask == ofl.OFL_MASK_ALL_GPU:
        assert list(s.gpu_nests) == [50] * 3 and list(s.cpu_nests) == [0] * 3
        assert s.h2d_count == 13 and s.d2h_count == 1
    g.close()


@pytest.fixture(scope="module")
def ragged():
    a = synth.make_problem(70, 37, 29, seed=77)
    return a, oracle.jacobi(a, 12, float(OMEGA))


@pytest.mark.parametrize("mode", [ofl.OFL_XFER_PER_ITER, ofl.OFL_XFER_HOISTED])
@pytest.mark.parametrize("mask", range(8))
def test_every_mask_and_placement(ragged, mask, mode):
    say("70x37x29 x12 mask", mask, "mode", mode)
    a, ref = ragged
    g, gosa = run_gpu(a, 12, mask=mask, mode=mode)
    check_against_oracle(a, g, gosa, 12, ref=ref)
    s = ofl.ofl_get_stats(g.handle)
    xs, _, _ = ofl.ofl_plan(mask, mode, 12, True)
    assert s.h2d_count == len([x for x in xs if x[4] == 0])
    assert s.d2h_count == len([x for x in xs if x[4] == 1])
    for nest in range(3):
        on_gpu = (mask >> nest) & 1
        assert s.gpu_nests[nest] == (12 if on_gpu else 0)
        assert s.cpu_nests[nest] == (0 if on_gpu else 12)
    g.close()


TILES = [
    ofl.tile(vec=1, rows=1, kchunk=1),
    ofl.tile(vec=1, rows=3, kchunk=5, flags=ofl.OFL_TILE_NT_LOADS),
    ofl.tile(vec=2, rows=8, kchunk=64, flags=ofl.OFL_TILE_PREFETCH),
    ofl.tile(vec=2, rows=2, kchunk=7, flags=ofl.OFL_TILE_NT_STORES),
    ofl.tile(vec=4, rows=4, kchunk=32, flags=0),
    ofl.tile(vec=4, rows=5, kchunk=3, flags=7),
    ofl.tile(vec=4, rows=8, kchunk=1024, flags=ofl.OFL_TILE_PREFETCH | ofl.OFL_TILE_NT_LOADS),
    ofl.tile(vec=4, rows=4, kchunk=4, flags=ofl.OFL_TILE_MARCH_J | ofl.OFL_TILE_NT_LOADS),
    ofl.tile(vec=2, rows=3, kchunk=5, flags=ofl.OFL_TILE_MARCH_J | ofl.OFL_TILE_PREFETCH),
    ofl.tile(vec=1, rows=8, kchunk=1, flags=ofl.OFL_TILE_MARCH_J | 7),
    ofl.tile(vec=4, rows=1, kchunk=64, flags=ofl.OFL_TILE_MARCH_J | ofl.OFL_TILE_NT_STORES),
    ofl.tile(vec=4, rows=4, kchunk=8, flags=ofl.OFL_TILE_XCD_REMAP | 3),
    ofl.tile(vec=2, rows=2, kchunk=3, flags=ofl.OFL_TILE_XCD_REMAP | ofl.OFL_TILE_MARCH_J),
]


@pytest.fixture(scope="module")
def wide():
    # 300 points along i: two or more i-tiles at every vector width, ragged ends
    a = synth.make_problem(300, 19, 23, seed=5)
    return a, oracle.jacobi(a, 4, float(OMEGA))


@pytest.mark.parametrize("t", TILES, ids=lambda t: f"v{t.vec}r{t.rows}k{t.kchunk}f{t.flags}")
def test_tiles(wide, t):
    say("300x19x23 x4 tile", t.as_dict())
    a, ref = wide
    g, gosa = run_gpu(a, 4, tile=t)
    check_against_oracle(a, g, gosa, 4, ref=ref)
    g.close()


# Shapes whose k-chunks hold a multiple of 8 tiles (i-tiles x row blocks), where
# the sweep hands each XCD one band of every k-chunk: the result must not
# depend on the order, so it is compared bitwise with the XCD-contiguous order
# and with the oracle. The third marches along j; the last has a ragged last
# row block (29 rows in blocks of 4).
@pytest.mark.parametrize("dims,vec,rows,kchunk,march", [
    ((300, 34, 21), 1, 4, 3, 0),                       # 5 i-tiles x 8 row blocks
    ((257, 66, 19), 4, 8, 4, 0),                       # 1 x 8
    ((130, 20, 34), 2, 2, 5, ofl.OFL_TILE_MARCH_J),    # 2 x 16 plane blocks
    ((300, 31, 21), 1, 4, 2, 0),                       # 5 x 8, last block one row
])
@pytest.mark.parametrize("fused", [False, True])
def test_sweep_band_order(dims, vec, rows, kchunk, march, fused):
    say("band order", dims, vec, rows, kchunk, march, "fused", fused)
    a = synth.make_problem(*dims, seed=dims[1])
    out = []
    for order in (0, ofl.OFL_TILE_XCD_REMAP):
        g = ofl.Grid(a)
        ofl.ofl_set_tile(g.handle, ofl.tile(vec=vec, rows=rows, kchunk=kchunk,
                                            flags=march | ofl.OFL_TILE_NT_LOADS | order))
        if fused:
            ofl.ofl_set_fusion(g.handle, ofl.OFL_FUSE_RESIDUAL)
        out.append((g, ofl.ofl_jacobi_run(g.handle, 5, OMEGA)))
    (g0, r0), (g1, r1) = out
    assert np.array_equal(g0.p, g1.p)
    if fused:
        assert r0 == pytest.approx(r1, rel=1e-12)   # partials land in other slots
    else:
        assert r0 == r1
    check_against_oracle(a, g0, r0, 5)
    g0.close()
    g1.close()


@pytest.mark.parametrize("dims", [(3, 3, 3), (3, 5, 4), (4, 3, 3), (5, 3, 7), (258, 3, 3), (66, 4, 5), (65, 6, 3),
                                  (130, 3, 4), (257, 5, 4)])
@pytest.mark.parametrize("vec", [1, 2, 4])
@pytest.mark.parametrize("march_j", [0, ofl.OFL_TILE_MARCH_J])
def test_edge_shapes(dims, vec, march_j):
    say("edge", dims, "vec", vec, "march_j", march_j)
    a = synth.make_problem(*dims, seed=sum(dims))
    g, gosa = run_gpu(a, 3, tile=ofl.tile(vec=vec, rows=2, kchunk=2, flags=march_j))
    check_against_oracle(a, g, gosa, 3)
    g.close()


def test_zero_iterations_on_gpu():
    say("zero iterations")
    a = synth.make_problem(9, 8, 7)
    g, gosa = run_gpu(a, 0)
    assert np.isnan(gosa) and np.array_equal(g.p, a["p"])
    g.close()


# --------------------------------------------------------- full-size configs


def test_129x129x257_200_iterations():
    say("129x129x257 x200 mask 7 hoisted")
    a = synth.make_problem(129, 129, 257)
    g, gosa = run_gpu(a, 200)
    pe, ge = check_against_oracle(a, g, gosa, 200)
    say(f"  p rel {pe:.2e} gosa rel {ge:.2e}")
    g.close()


def test_full_batch_in_the_benchmark_configuration():
    """The 64 uneven grids as the benchmark runs them: compact rows (packed
    where that pays), the default batch tile, plain and fused; two iterations
    against the oracle on every grid."""
    say("64 uneven grids: generating")
    probs = synth.make_batch(64)
    say("64 uneven grids: oracle")
    refs = [oracle.jacobi(a, 2, float(OMEGA)) for _, a in probs]
    for fusion in (0, ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP):
        say("64 uneven grids: batch, fusion", fusion)
        grids = [ofl.Grid(a, row_align=4) for _, a in probs]
        b = ofl.ofl_batch_create([g.handle for g in grids])
        ofl.ofl_batch_set_fusion(b, fusion)
        gosa = ofl.ofl_batch_run(b, 2, OMEGA, len(grids))
        ofl.ofl_batch_destroy(b)
        for (_, a), g, x, ref in zip(probs, grids, gosa, refs):
            check_against_oracle(a, g, x, 2, ref=ref)
            g.close()


@pytest.fixture(scope="module")
def headline():
    say("generating 257x257x513")
    return synth.make_problem(257, 257, 513)


def test_257x257x513_first_iterations(headline):
    say("257x257x513 x2 full compare")
    a = headline
    g, gosa = run_gpu(a, 2)
    pe, ge = check_against_oracle(a, g, gosa, 2)
    say(f"  p rel {pe:.2e} gosa rel {ge:.2e}")
    g.close()


@pytest.mark.parametrize("form", ["bf16_offset", "fused_f32", "fused_bf16_offset"])
def test_257x257x513_variants_first_iterations(headline, form):
    """The benchmark's other single-grid forms at full size, in its launch
    configuration (default tile, PyTorch arena and stream, inside a data
    region): two iterations against the oracle on the FP32 inputs."""
    say("257x257x513 x2", form)
    a = headline
    fmt = ofl.OFL_COEF_BF16_OFFSET if "bf16" in form else ofl.OFL_COEF_F32
    g = ofl.Grid(a, coef_format=fmt, torch_memory=True)
    if form.startswith("fused"):
        ofl.ofl_set_fusion(g.handle, ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP)
    ofl.ofl_data_enter(g.handle)
    gosa = ofl.ofl_jacobi_run(g.handle, 2, OMEGA)
    ofl.ofl_data_exit(g.handle)
    tol = TOL_BF16 if fmt != ofl.OFL_COEF_F32 else TOL_P_F32
    tol_g = TOL_BF16 if fmt != ofl.OFL_COEF_F32 else TOL_GOSA_F32
    pe, ge = check_against_oracle(a, g, gosa, 2, tol_p=tol, tol_g=tol_g)
    say(f"  p rel {pe:.2e} gosa rel {ge:.2e}")
    g.close()


def test_257x257x513_100th_iteration(headline):
    """The 100-iteration run in the benchmark's configuration: after 99
    iterations inside a data region, fetch p; the 100th step must equal one
    oracle sweep applied to exactly that FP32 iterate."""
    say("257x257x513 x100 in a data region")
    a = headline
    g = ofl.Grid(a, torch_memory=True)
    ofl.ofl_set_offload_mask(g.handle, 7, ofl.OFL_XFER_HOISTED)
    ofl.ofl_data_enter(g.handle)
    ofl.ofl_jacobi_run(g.handle, 99, OMEGA)
    assert np.array_equal(g.p, a["p"])  # nothing came home inside the region
    ofl.ofl_update_host(g.handle)
    p99 = g.p.copy()
    gosa100 = ofl.ofl_jacobi_run(g.handle, 1, OMEGA)
    ofl.ofl_data_exit(g.handle)
    assert boundary_equal(g.p, a["p"])
    w_ref, g_ref = oracle.sweep(dict(a, p=p99), float(OMEGA))
    p_ref = p99.astype(np.float64)
    p_ref[1:-1, 1:-1, 1:-1] = w_ref[1:-1, 1:-1, 1:-1]
    pe, ge = p_rel_err(g.p, p_ref), rel_err(gosa100, g_ref)
    say(f"  step-100 p rel {pe:.2e} gosa rel {ge:.2e}")
    assert pe <= TOL_P_F32 and ge <= TOL_GOSA_F32
    g.close()


# ------------------------------------------------------ formats and residual


@pytest.fixture(scope="module")
def mid():
    a = synth.make_problem(129, 129, 65, seed=11)
    return a, oracle.jacobi(a, 50, float(OMEGA))


def test_bf16_offset_storage(mid):
    say("bf16-offset 129x129x65 x50")
    a, ref = mid
    g, gosa = run_gpu(a, 50, fmt=ofl.OFL_COEF_BF16_OFFSET)
    pe, ge = check_against_oracle(a, g, gosa, 50, tol_p=TOL_BF16, tol_g=TOL_BF16, ref=ref)
    say(f"  vs FP32-input oracle: p rel {pe:.2e} gosa rel {ge:.2e}")
    # the library's bias (its own encoder) must be the oracle's, which decodes the reference
    bias = ofl.ofl_grid_coef_bias(g.handle)
    dec = dict(a)
    for n, name in enumerate(ofl.COEF_NAMES):
        ref_bias = oracle.offset_bias(a[name])
        assert bias[n] == ref_bias, name
        dec[name] = oracle.offset_bf16_decode(a[name], ref_bias)
    pe2, ge2 = check_against_oracle(dec, g, gosa, 50)
    say(f"  vs decoded-input oracle: p rel {pe2:.2e} gosa rel {ge2:.2e}")
    g.close()


def test_bf16_plain_storage_matches_decoded_inputs(mid):
    say("bf16-plain 129x129x65 x50")
    a, _ = mid
    g, gosa = run_gpu(a, 50, fmt=ofl.OFL_COEF_BF16)
    dec = {k: (oracle.bf16_rne(v) if k in ofl.COEF_NAMES else v) for k, v in a.items()}
    check_against_oracle(dec, g, gosa, 50)
    g.close()


@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET])
def test_compensated_fp32_residual(mid, fmt):
    say("kahan residual fmt", fmt)
    a, ref = mid
    g, gosa = run_gpu(a, 50, fmt=fmt, sum_mode=ofl.OFL_SUM_KAHAN_F32)
    tol = TOL_GOSA_F32 if fmt == ofl.OFL_COEF_F32 else TOL_BF16
    assert rel_err(gosa, ref[1]) <= tol
    g.close()


def test_residual_entry_point_on_gpu():
    say("ofl_residual")
    a = synth.make_problem(67, 45, 37, seed=3)
    g = ofl.Grid(a)
    r = ofl.ofl_residual(g.handle)
    assert rel_err(r, oracle.residual(a)) <= TOL_GOSA_F32
    assert np.array_equal(g.p, a["p"])
    g.close()


def test_torch_memory_and_stream():
    say("torch arena + stream")
    a = synth.make_problem(40, 33, 21, seed=8)
    g, gosa = run_gpu(a, 10, torch_memory=True)
    check_against_oracle(a, g, gosa, 10)
    g.close()


@pytest.mark.parametrize("dims,row_align", [((96, 33, 65), 4), ((32, 33, 65), 32), ((45, 29, 23), 8)])
def test_torch_arena_sized_for_compact_rows(dims, row_align):
    """An arena of exactly ofl_grid_device_bytes(..., row_align) bytes holds a
    grid with compact rows (whose planes are padded to 64 elements, so it can
    need more than 128-byte rows)."""
    say("torch arena, compact rows", dims, row_align)
    a = synth.make_problem(*dims, seed=9)
    g = ofl.Grid(a, torch_memory=True, row_align=row_align)
    assert g.desc.dev_arena_bytes == ofl.ofl_grid_device_bytes(*dims, ofl.OFL_COEF_F32, row_align)
    gosa = ofl.ofl_jacobi_run(g.handle, 6, OMEGA)
    check_against_oracle(a, g, gosa, 6)
    g.close()


# ------------------------------------------------ determinism and semantics


def test_bitwise_deterministic():
    say("determinism")
    a = synth.make_problem(129, 67, 45, seed=12)
    g1, r1 = run_gpu(a, 20)
    g2, r2 = run_gpu(a, 20)
    assert np.array_equal(g1.p, g2.p) and r1 == r2
    g1.close()
    g2.close()


def test_split_runs_in_data_region_equal_one_run():
    say("split runs")
    a = synth.make_problem(80, 40, 30, seed=13)
    g1, r1 = run_gpu(a, 10)
    g2 = ofl.Grid(a)
    ofl.ofl_data_enter(g2.handle)
    ofl.ofl_jacobi_run(g2.handle, 4, OMEGA)
    r2 = ofl.ofl_jacobi_run(g2.handle, 6, OMEGA)
    ofl.ofl_data_exit(g2.handle)
    assert np.array_equal(g1.p, g2.p) and r1 == r2
    s = ofl.ofl_get_stats(g2.handle)
    assert s.h2d_count == 13 and s.d2h_count == 1
    g1.close()
    g2.close()


def test_profiling_counts_every_gpu_nest():
    say("profiling")
    a = synth.make_problem(65, 33, 33, seed=14)
    g = ofl.Grid(a)
    ofl.ofl_set_profiling(g.handle, True)
    ofl.ofl_jacobi_run(g.handle, 7, OMEGA)
    s = ofl.ofl_get_stats(g.handle)
    assert list(s.timed_nests) == [7, 7, 7]
    assert all(ms > 0 for ms in s.kernel_ms)
    g.close()


@pytest.mark.parametrize("setup", ["whole", "regions", "fused"])
def test_profiling_only_the_chosen_nests(setup):
    say("profiled nests", setup)
    a = synth.make_problem(65, 33, 33, seed=14)
    g = ofl.Grid(a)
    if setup == "regions":
        ofl.ofl_set_regions(g.handle, 7, [1, 2, 0])
    if setup == "fused":
        ofl.ofl_set_fusion(g.handle, ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP)
    ofl.ofl_set_profiling(g.handle, True)
    ofl.ofl_set_profiled_nests(g.handle, ofl.OFL_NEST_SWEEP | ofl.OFL_NEST_COPYBACK)
    ofl.ofl_jacobi_run(g.handle, 5, OMEGA)
    s = ofl.ofl_get_stats(g.handle)
    want_c = 0 if setup == "fused" else 5  # a fused copy-back is a buffer exchange: no kernel to time
    assert list(s.timed_nests) == [5, 0, want_c] and s.kernel_ms[0] > 0
    ofl.ofl_reset_stats(g.handle)
    ofl.ofl_set_profiled_nests(g.handle, ofl.OFL_MASK_ALL_GPU)
    ofl.ofl_jacobi_run(g.handle, 2, OMEGA)
    # fused: each iteration's residual sum but the last runs inside the next
    # sweep launch, so one residual reduction per run is timed on its own
    want = [2, 1, 0] if setup == "fused" else [2, 2, 2]
    assert list(ofl.ofl_get_stats(g.handle).timed_nests) == want
    g.close()


def test_device_copy_kernel():
    say("device copy")
    src = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    ofl.ofl_device_copy(dst.data_ptr(), src.data_ptr(), src.numel() * 4, None)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


@pytest.mark.parametrize("n32,n16", [(13, 0), (1, 12)])
def test_device_stream_kernel(n32, n16):
    """The sweep-pattern ceiling probe sums its sources exactly (small
    integers, so any order is exact); n ends on a partial work-group."""
    say("device stream", n32, n16)
    n = 256 * 37 + 12
    g = torch.Generator(device="cuda").manual_seed(n32)
    f = [torch.randint(-64, 64, (n,), device="cuda", generator=g).float() for _ in range(n32)]
    h = [torch.randint(-64, 64, (n,), device="cuda", generator=g).to(torch.bfloat16) for _ in range(n16)]
    dst = torch.full((n,), float("nan"), device="cuda")
    ofl.ofl_device_stream([x.data_ptr() for x in f], [x.data_ptr() for x in h], dst.data_ptr(), n)
    torch.cuda.synchronize()
    want = torch.stack(f).sum(0) + (torch.stack([x.float() for x in h]).sum(0) if h else 0)
    assert torch.equal(dst, want)
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_device_stream([x.data_ptr() for x in f[:2]], [], dst.data_ptr(), n)
    assert e.value.code == ofl.OFL_ENOTSUP


# ------------------------------------------------------------------ fusion


@pytest.mark.parametrize("fusion", [ofl.OFL_FUSE_RESIDUAL, ofl.OFL_FUSE_COPYBACK_SWAP,
                                    ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP])
@pytest.mark.parametrize("iters", [1, 6, 7])
@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET])
def test_fused_nests_equal_unfused(fusion, iters, fmt):
    say("fusion", fusion, "iters", iters, "fmt", fmt)
    a = synth.make_problem(131, 37, 45, seed=17)
    ref, r_ref = run_gpu(a, iters, fmt=fmt)
    g = ofl.Grid(a, coef_format=fmt)
    ofl.ofl_set_fusion(g.handle, fusion)
    r = ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
    assert np.array_equal(g.p, ref.p)          # same per-point arithmetic, exact exchange
    assert r == pytest.approx(r_ref, rel=1e-12)  # same terms, another summation order
    s = ofl.ofl_get_stats(g.handle)
    assert list(s.gpu_nests) == [iters] * 3 and list(s.cpu_nests) == [0] * 3
    if fmt == ofl.OFL_COEF_F32:
        check_against_oracle(a, g, r, iters)
    ref.close()
    g.close()


# The fused residual of each iteration but the last is summed by the first
# work-group of the next sweep, and the last one by a work-group of the same
# size running the same group sum: work-groups of 1, 3, 5 and 7 waves (not
# powers of two) and runs long enough to fold several sums.
@pytest.mark.parametrize("rows", [1, 3, 5, 7])
def test_fused_residual_sum_at_every_work_group_size(rows):
    say("fused residual sum, rows", rows)
    a = synth.make_problem(131, 37, 45, seed=19)
    t = ofl.tile(vec=4, rows=rows, kchunk=3, flags=1)
    ref, r_ref = run_gpu(a, 5, tile=t)
    g = ofl.Grid(a)
    ofl.ofl_set_tile(g.handle, t)
    ofl.ofl_set_fusion(g.handle, ofl.OFL_FUSE_RESIDUAL)
    r = ofl.ofl_jacobi_run(g.handle, 5, OMEGA)
    assert np.array_equal(g.p, ref.p)
    assert r == pytest.approx(r_ref, rel=1e-12)
    check_against_oracle(a, g, r, 5)
    ref.close()
    g.close()


def test_fused_batch_residual_sum_with_three_wave_work_groups():
    say("fused batch residual sum, rows 3")
    probs = _small_batch()
    tile = ofl.tile(vec=0, rows=3, kchunk=2, flags=1)
    ref = [ofl.Grid(a) for a in probs]
    rb = ofl.ofl_batch_create([g.handle for g in ref], tile)
    r_ref = ofl.ofl_batch_run(rb, 4, OMEGA, len(ref))
    grids = [ofl.Grid(a) for a in probs]
    b = ofl.ofl_batch_create([g.handle for g in grids], tile)
    ofl.ofl_batch_set_fusion(b, ofl.OFL_FUSE_RESIDUAL)
    r = ofl.ofl_batch_run(b, 4, OMEGA, len(grids))
    for a, g, gr, x, xr in zip(probs, grids, ref, r, r_ref):
        assert np.array_equal(g.p, gr.p)
        assert x == pytest.approx(xr, rel=1e-12)
        check_against_oracle(a, g, x, 4)
    ofl.ofl_batch_destroy(b)
    ofl.ofl_batch_destroy(rb)
    for g in grids + ref:
        g.close()


def test_fused_runs_hand_over_state_to_unfused_runs_and_cpu_nests():
    say("fusion state handover")
    a = synth.make_problem(70, 41, 33, seed=19)
    g = ofl.Grid(a)
    ofl.ofl_set_fusion(g.handle, ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP)
    ofl.ofl_data_enter(g.handle)
    ofl.ofl_jacobi_run(g.handle, 3, OMEGA)        # odd count: p lives in the other buffer
    ofl.ofl_set_fusion(g.handle, 0)
    ofl.ofl_jacobi_run(g.handle, 2, OMEGA)        # plain GPU nests continue from there
    ofl.ofl_data_exit(g.handle)
    ofl.ofl_set_offload_mask(g.handle, ofl.OFL_NEST_SWEEP, ofl.OFL_XFER_PER_ITER)
    ofl.ofl_jacobi_run(g.handle, 2, OMEGA)        # mixed gene, per-iteration transfers
    ofl.ofl_set_fusion(g.handle, ofl.OFL_FUSE_COPYBACK_SWAP)
    ofl.ofl_set_offload_mask(g.handle, ofl.OFL_MASK_ALL_GPU, ofl.OFL_XFER_HOISTED)
    r = ofl.ofl_jacobi_run(g.handle, 3, OMEGA)    # p re-uploaded: the boundary copy is redone
    check_against_oracle(a, g, r, 10)
    g.close()


def test_fused_residual_refused_for_a_compensated_batch():
    say("fused residual + compensated batch")
    grids = [ofl.Grid(a, sum_mode=ofl.OFL_SUM_KAHAN_F32) for a in _small_batch(2)]
    b = ofl.ofl_batch_create([g.handle for g in grids])
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_batch_set_fusion(b, ofl.OFL_FUSE_RESIDUAL)
    assert e.value.code == ofl.OFL_ENOTSUP
    ofl.ofl_batch_set_fusion(b, ofl.OFL_FUSE_COPYBACK_SWAP)
    gosa = ofl.ofl_batch_run(b, 3, OMEGA, len(grids))
    ofl.ofl_batch_destroy(b)
    for a, g, x in zip(_small_batch(2), grids, gosa):
        check_against_oracle(a, g, x, 3)
        g.close()


def test_fusion_rejected_inside_a_batch():
    say("fusion + batch")
    probs = _small_batch(2)
    grids = [ofl.Grid(a) for a in probs]
    b = ofl.ofl_batch_create([g.handle for g in grids])
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_set_fusion(grids[0].handle, ofl.OFL_FUSE_RESIDUAL)
    assert e.value.code == ofl.OFL_ESTATE
    ofl.ofl_batch_destroy(b)
    ofl.ofl_set_fusion(grids[0].handle, ofl.OFL_FUSE_RESIDUAL)
    with pytest.raises(ofl.OflError):
        ofl.ofl_batch_create([g.handle for g in grids])
    for g in grids:
        g.close()


# ------------------------------------------------------------------- batch


def _small_batch(n=6):
    sizes = [(37, 41, 67), (70, 33, 70), (130, 35, 66), (33, 33, 65), (161, 40, 80), (50, 90, 70)][:n]
    return [synth.make_problem(I, J, K, seed=synth.grid_seed(t)) for t, (I, J, K) in enumerate(sizes)]


@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET])
@pytest.mark.parametrize("occupancy", [0, 2])
@pytest.mark.parametrize("march_j", [0, ofl.OFL_TILE_MARCH_J])
def test_batch_matches_oracle_and_single_runs(fmt, occupancy, march_j):
    say("batch fmt", fmt, "occupancy", occupancy, "march_j", march_j)
    probs = _small_batch()
    tile = ofl.tile(vec=2, rows=4, kchunk=16, occupancy=occupancy, flags=march_j)
    grids = [ofl.Grid(a, coef_format=fmt) for a in probs]
    b = ofl.ofl_batch_create([g.handle for g in grids], tile)
    gosa = ofl.ofl_batch_run(b, 8, OMEGA, len(grids))
    tol = TOL_P_F32 if fmt == ofl.OFL_COEF_F32 else TOL_BF16
    tol_g = TOL_GOSA_F32 if fmt == ofl.OFL_COEF_F32 else TOL_BF16
    for a, g, r in zip(probs, grids, gosa):
        check_against_oracle(a, g, r, 8, tol_p=tol, tol_g=tol_g)
    # the same tile on one grid at a time: identical per-point arithmetic -> identical p
    for a, g in zip(probs, grids):
        single, _ = run_gpu(a, 8, tile=ofl.tile(vec=2, rows=4, kchunk=16, flags=march_j), fmt=fmt)
        assert np.array_equal(single.p, g.p)
        single.close()
    ofl.ofl_batch_destroy(b)
    for g in grids:
        g.close()


@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET])
def test_batch_per_grid_vector_width(fmt):
    say("batch vec=0 fmt", fmt)
    probs = _small_batch()
    grids = [ofl.Grid(a, coef_format=fmt) for a in probs]
    b = ofl.ofl_batch_create([g.handle for g in grids], ofl.tile(vec=0, rows=4, kchunk=4, flags=1))
    gosa = ofl.ofl_batch_run(b, 6, OMEGA, len(grids))
    tol = TOL_P_F32 if fmt == ofl.OFL_COEF_F32 else TOL_BF16
    tol_g = TOL_GOSA_F32 if fmt == ofl.OFL_COEF_F32 else TOL_BF16
    for a, g, r in zip(probs, grids, gosa):
        check_against_oracle(a, g, r, 6, tol_p=tol, tol_g=tol_g)
    ofl.ofl_batch_destroy(b)
    for g in grids:
        g.close()


def test_batch_default_tile_follows_format_and_fusion():
    """A batch without a tile of its own: each grid's width, one line per
    work-group, 2-plane chunks (FP32) or 4-plane ones (bfloat16), non-temporal
    loads and stores; unfused bfloat16 batches 4 points per lane and 2 lines.
    Fusion re-derives it until a tile is set; the unfused bfloat16 default is
    checked against the FP64 oracle at the bfloat16 bar."""
    say("batch default tiles")
    probs = _small_batch(3)
    fuse = ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP
    for fmt in (ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET):
        f32 = fmt == ofl.OFL_COEF_F32
        fused = dict(vec=0, rows=1, kchunk=2 if f32 else 4, flags=3, occupancy=0)
        plain = fused if f32 else dict(fused, vec=4, rows=2)
        grids = [ofl.Grid(a, coef_format=fmt) for a in probs]
        b = ofl.ofl_batch_create([g.handle for g in grids])
        assert ofl.ofl_batch_get_tile(b).as_dict() == plain
        if not f32:
            gosa = ofl.ofl_batch_run(b, 4, OMEGA, len(grids))
            for a, g, r in zip(probs, grids, gosa):
                check_against_oracle(a, g, r, 4, tol_p=TOL_BF16, tol_g=TOL_BF16)
        ofl.ofl_batch_set_fusion(b, fuse)
        assert ofl.ofl_batch_get_tile(b).as_dict() == fused
        ofl.ofl_batch_set_fusion(b, 0)
        assert ofl.ofl_batch_get_tile(b).as_dict() == plain
        mine = ofl.tile(vec=2, rows=3, kchunk=5, flags=1)
        ofl.ofl_batch_set_tile(b, mine)
        ofl.ofl_batch_set_fusion(b, fuse)
        assert ofl.ofl_batch_get_tile(b).as_dict() == mine.as_dict()
        ofl.ofl_batch_destroy(b)
        for g in grids:
            g.close()


@pytest.mark.parametrize("fusion", [ofl.OFL_FUSE_RESIDUAL, ofl.OFL_FUSE_COPYBACK_SWAP,
                                    ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP])
@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET])
def test_fused_batch_equals_unfused_batch(fusion, fmt):
    say("fused batch", fusion, "fmt", fmt)
    probs = _small_batch()
    tile = ofl.tile(vec=0, rows=4, kchunk=4, flags=1)
    ref = [ofl.Grid(a, coef_format=fmt) for a in probs]
    rb = ofl.ofl_batch_create([g.handle for g in ref], tile)
    r_ref = ofl.ofl_batch_run(rb, 5, OMEGA, len(ref))
    grids = [ofl.Grid(a, coef_format=fmt) for a in probs]
    b = ofl.ofl_batch_create([g.handle for g in grids], tile)
    ofl.ofl_batch_set_fusion(b, fusion)
    for g in grids:
        ofl.ofl_data_enter(g.handle)
    ofl.ofl_batch_run(b, 3, OMEGA, len(grids))        # odd: buffers end exchanged
    r = ofl.ofl_batch_run(b, 2, OMEGA, len(grids))    # replay continues from there
    for g in grids:
        ofl.ofl_data_exit(g.handle)
    for g, gr, x, xr in zip(grids, ref, r, r_ref):
        assert np.array_equal(g.p, gr.p)
        assert x == pytest.approx(xr, rel=1e-12)
    for a, g, x in zip(probs, grids, r):
        if fmt == ofl.OFL_COEF_F32:
            check_against_oracle(a, g, x, 5)
    ofl.ofl_batch_destroy(b)
    ofl.ofl_batch_destroy(rb)
    for g in grids + ref:
        g.close()


# Edge shapes for packed rows: the smallest grid, rows that fill whole
# segments exactly ((J-2) * pitch a multiple of 256), one row, and a grid
# whose rows are longer than a wave's segment.
_PACKED_SIZES = [(3, 3, 3), (34, 66, 9), (5, 3, 7), (33, 33, 65), (300, 7, 6), (97, 41, 12), (62, 130, 5)]


def _batch_run(probs, fmt, tile, row_align, iters, fusion=0):
    grids = [ofl.Grid(a, coef_format=fmt, row_align=ra) for a, ra in zip(probs, row_align)]
    b = ofl.ofl_batch_create([g.handle for g in grids], tile)
    if fusion:
        ofl.ofl_batch_set_fusion(b, fusion)
    gosa = ofl.ofl_batch_run(b, iters, OMEGA, len(grids))
    ofl.ofl_batch_destroy(b)
    return grids, gosa


@pytest.mark.parametrize("fusion", [0, ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP])
@pytest.mark.parametrize("vec,flags", [(0, ofl.OFL_TILE_NT_LOADS), (2, ofl.OFL_TILE_NT_LOADS),
                                       (0, ofl.OFL_TILE_NT_LOADS | ofl.OFL_TILE_NT_STORES)])
@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET])
def test_packed_row_batch_equals_row_batch(fmt, vec, flags, fusion):
    say("packed-row batch fmt", fmt, "vec", vec, "flags", flags, "fusion", fusion)
    probs = [synth.make_problem(I, J, K, seed=synth.grid_seed(40 + t)) for t, (I, J, K) in enumerate(_PACKED_SIZES)]
    tile = ofl.tile(vec=vec, rows=4, kchunk=4, flags=flags)
    ref, r_ref = _batch_run(probs, fmt, tile, [0] * len(probs), 5, fusion)
    # compact rows everywhere but one grid, so both forms share the launches
    aligns = [4, 4, 8, 4, 0, 16, 4]
    grids, r = _batch_run(probs, fmt, tile, aligns, 5, fusion)
    tol = TOL_P_F32 if fmt == ofl.OFL_COEF_F32 else TOL_BF16
    tol_g = TOL_GOSA_F32 if fmt == ofl.OFL_COEF_F32 else TOL_BF16
    for a, g, gr, x, xr in zip(probs, grids, ref, r, r_ref):
        assert np.array_equal(g.p, gr.p)
        assert x == pytest.approx(xr, rel=1e-12, abs=1e-300)
        check_against_oracle(a, g, x, 5, tol_p=tol, tol_g=tol_g)
    for g in grids + ref:
        g.close()


def test_batch_default_tile():
    say("batch default tile")
    grids = [ofl.Grid(a, row_align=4) for a in _small_batch(2)]
    b = ofl.ofl_batch_create([g.handle for g in grids])
    assert ofl.ofl_batch_get_tile(b).as_dict() == dict(
        vec=0, rows=1, kchunk=2, flags=ofl.OFL_TILE_NT_LOADS | ofl.OFL_TILE_NT_STORES, occupancy=0)
    ofl.ofl_batch_destroy(b)
    for g in grids:
        g.close()
    grids = [ofl.Grid(a, row_align=4, coef_format=ofl.OFL_COEF_BF16_OFFSET) for a in _small_batch(2)]
    b = ofl.ofl_batch_create([g.handle for g in grids])
    assert ofl.ofl_batch_get_tile(b).kchunk == 4
    ofl.ofl_batch_destroy(b)
    for g in grids:
        g.close()


@pytest.mark.parametrize("fusion", [0, ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP])
@pytest.mark.parametrize("rows,occupancy", [(1, 0), (4, 0), (2, 1)])
@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET])
def test_batch_band_order_equals_remap_order(fmt, rows, occupancy, fusion):
    """The batch hands each XCD runs of consecutive sweep items unless the
    tile asks for XCD-contiguous ranges: both orders must give bitwise the
    same p (and, unfused, the same residuals; fused, the same terms summed in
    other slots), on packed and row-per-wave grids, one work-group per item
    or a smaller grid walking the list."""
    say("batch band order fmt", fmt, "rows", rows, "occupancy", occupancy, "fusion", fusion)
    probs = _small_batch() + [synth.make_problem(40, 66, 30, seed=synth.grid_seed(77))]
    aligns = [4, 0, 4, 4, 0, 4, 4]
    base = dict(vec=0, rows=rows, kchunk=3, occupancy=occupancy)
    flags = ofl.OFL_TILE_NT_LOADS | ofl.OFL_TILE_NT_STORES
    band, r_band = _batch_run(probs, fmt, ofl.tile(flags=flags, **base), aligns, 5, fusion)
    remap, r_remap = _batch_run(probs, fmt, ofl.tile(flags=flags | ofl.OFL_TILE_XCD_REMAP, **base), aligns, 5, fusion)
    for a, g, gr, x, xr in zip(probs, band, remap, r_band, r_remap):
        assert np.array_equal(g.p, gr.p)
        assert x == (xr if fusion == 0 else pytest.approx(xr, rel=1e-12))
    if fmt == ofl.OFL_COEF_F32:
        for a, g, x in zip(probs[:2], band, r_band):
            check_against_oracle(a, g, x, 5)
    for g in band + remap:
        g.close()


@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET])
def test_packed_rows_on_random_shapes(fmt):
    """16 seeded random shapes (I 3..300, J 3..80, K 3..40) with random compact
    row alignments, as one packed batch, bitwise against the one-wave-per-row
    batch on 128-byte rows."""
    rng = np.random.default_rng(20110360)
    shapes = [(int(rng.integers(3, 301)), int(rng.integers(3, 81)), int(rng.integers(3, 41))) for _ in range(16)]
    aligns = [int(rng.choice([4, 8, 16])) for _ in shapes]
    say("packed rows, random shapes", shapes, aligns)
    probs = [synth.make_problem(I, J, K, seed=synth.grid_seed(100 + t)) for t, (I, J, K) in enumerate(shapes)]
    tile = ofl.tile(vec=0, rows=4, kchunk=4, flags=ofl.OFL_TILE_NT_LOADS | ofl.OFL_TILE_NT_STORES)
    ref, r_ref = _batch_run(probs, fmt, tile, [0] * len(probs), 3)
    grids, r = _batch_run(probs, fmt, tile, aligns, 3)
    for shape, g, gr, x, xr in zip(shapes, grids, ref, r, r_ref):
        assert np.array_equal(g.p, gr.p), shape
        assert x == pytest.approx(xr, rel=1e-12, abs=1e-300), shape
    for g in grids + ref:
        g.close()


@pytest.mark.parametrize("row_align", [4, 8, 16])
@pytest.mark.parametrize("tile", [dict(vec=1, rows=2, kchunk=3), dict(vec=4, rows=4, kchunk=4, flags=1),
                                  dict(vec=2, rows=4, kchunk=5, flags=ofl.OFL_TILE_MARCH_J)], ids=str)
def test_compact_rows_single_grid_bitwise(row_align, tile):
    say("compact rows, single grid, align", row_align, tile)
    a = synth.make_problem(45, 29, 23, seed=31)
    ref = ofl.Grid(a)
    g = ofl.Grid(a, row_align=row_align)
    for h in (ref.handle, g.handle):
        ofl.ofl_set_tile(h, ofl.tile(**tile))
    x_ref = ofl.ofl_jacobi_run(ref.handle, 4, OMEGA)
    x = ofl.ofl_jacobi_run(g.handle, 4, OMEGA)
    assert np.array_equal(g.p, ref.p) and x == x_ref
    check_against_oracle(a, g, x, 4)
    ref.close()
    g.close()


def test_batch_graph_replays_continue_the_iteration():
    say("batch graph replay")
    probs = _small_batch(4)
    grids = [ofl.Grid(a) for a in probs]
    b = ofl.ofl_batch_create([g.handle for g in grids], ofl.tile(vec=1, rows=2, kchunk=32))
    for g in grids:
        ofl.ofl_data_enter(g.handle)
    ofl.ofl_batch_run(b, 3, OMEGA, len(grids))   # captures the graph
    torch.cuda.synchronize()
    ofl.ofl_batch_run(b, 3, OMEGA, len(grids))   # replays it
    gosa = ofl.ofl_batch_run(b, 3, OMEGA, len(grids))  # and again
    for g in grids:
        ofl.ofl_data_exit(g.handle)
    for a, g, r in zip(probs, grids, gosa):
        check_against_oracle(a, g, r, 9)
    ofl.ofl_batch_destroy(b)
    for g in grids:
        g.close()


def test_residual_sums_only_fresh_partials():
    """The residual kernel's last block sums every block's partial. Iterations
    at omega 0.1 alternate with ofl_residual (omega 1, partials 100x larger),
    so a partial left over from the previous launch would be far off; every
    value must agree with the library's CPU nests on the same iterates."""
    say("residual partials, alternating scales")
    a = synth.make_problem(67, 45, 37, seed=5)
    gpu, cpu = ofl.Grid(a), ofl.Grid(a)
    ofl.ofl_set_offload_mask(cpu.handle, ofl.OFL_MASK_ALL_CPU, ofl.OFL_XFER_HOISTED)
    for step in range(6):
        om = np.float32(0.1 if step % 2 else 1.3)
        xg, xc = ofl.ofl_jacobi_run(gpu.handle, 1, om), ofl.ofl_jacobi_run(cpu.handle, 1, om)
        assert rel_err(xg, xc) <= TOL_GOSA_F32, step
        rg, rc = ofl.ofl_residual(gpu.handle), ofl.ofl_residual(cpu.handle)
        assert rel_err(rg, rc) <= TOL_GOSA_F32, step
        assert p_rel_err(gpu.p, cpu.p.astype(np.float64)) <= TOL_P_F32, step
    gpu.close()
    cpu.close()


@pytest.mark.parametrize("row_align", [0, 4])
def test_whole_row_copyback_keeps_the_boundary(row_align):
    """After a resident run's first iteration the device wrk2 carries p's
    boundary and the copy-back copies whole rows. Genes that move p or wrk2
    between the host and the device in between must not let a stale boundary
    through: every run is checked against the library's CPU nests, with the
    boundary of p bitwise unchanged."""
    say("whole-row copy-back, row_align", row_align)
    a = synth.make_problem(45, 29, 23, seed=77)
    gpu, cpu = ofl.Grid(a, row_align=row_align), ofl.Grid(a)
    ofl.ofl_set_offload_mask(cpu.handle, ofl.OFL_MASK_ALL_CPU, ofl.OFL_XFER_HOISTED)
    ofl.ofl_data_enter(gpu.handle)
    for mask, mode in [(7, 1), (3, 1), (7, 1), (5, 0), (7, 1), (6, 1), (7, 0), (7, 1)]:
        ofl.ofl_set_offload_mask(gpu.handle, mask, mode)
        xg, xc = ofl.ofl_jacobi_run(gpu.handle, 3, OMEGA), ofl.ofl_jacobi_run(cpu.handle, 3, OMEGA)
        ofl.ofl_update_host(gpu.handle)
        assert boundary_equal(gpu.p, a["p"]), (mask, mode)
        assert p_rel_err(gpu.p, cpu.p.astype(np.float64)) <= TOL_P_F32, (mask, mode)
        assert rel_err(xg, xc) <= TOL_GOSA_F32, (mask, mode)
    ofl.ofl_data_exit(gpu.handle)
    assert boundary_equal(gpu.p, a["p"])
    gpu.close()
    cpu.close()


# --------------------------------------------------------- graph replays


@pytest.mark.parametrize("region", [True, False])
@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET])
def test_graph_replays_equal_eager_runs(fmt, region):
    """Whole-nest, hoisted, all-GPU runs replay their steady-state iterations
    from captured graphs; with profiling on every nest is launched on its own.
    Every call of the graphed grid must equal the eager grid's, through
    replays of one graph, a second length, runs longer than one graph, single
    iterations, a new tile and a new omega, with host copies and
    synchronisations between the calls."""
    say("graph replays, fmt", fmt, "region", region)
    a = synth.make_problem(33, 33, 65, seed=71)
    eager = ofl.Grid(a, coef_format=fmt)
    graphed = ofl.Grid(a, coef_format=fmt)
    ofl.ofl_set_profiling(eager.handle, True)
    if region:
        for g in (eager, graphed):
            ofl.ofl_data_enter(g.handle)
    total = 0
    plan = [(7, OMEGA, None), (7, OMEGA, None), (3, OMEGA, None), (7, OMEGA, None), (300, OMEGA, None),
            (1, OMEGA, None), (7, OMEGA, dict(vec=1, rows=2, kchunk=5, flags=1)), (7, OMEGA, None),
            (5, np.float32(0.7), None), (7, OMEGA, None)]
    for iters, om, tile in plan:
        if tile:
            for g in (eager, graphed):
                ofl.ofl_set_tile(g.handle, ofl.tile(**tile))
        x_e = ofl.ofl_jacobi_run(eager.handle, iters, om)
        x_g = ofl.ofl_jacobi_run(graphed.handle, iters, om)
        if region:
            for g in (eager, graphed):
                ofl.ofl_update_host(g.handle)
        torch.cuda.synchronize()
        assert np.array_equal(graphed.p, eager.p), (iters, om, tile)
        assert x_g == x_e, (iters, om, tile)
        total += iters
    se, sg = ofl.ofl_get_stats(eager.handle), ofl.ofl_get_stats(graphed.handle)
    assert list(sg.gpu_nests) == list(se.gpu_nests) == [total] * 3
    assert list(sg.gpu_regions) == list(se.gpu_regions)
    if region:
        for g in (eager, graphed):
            ofl.ofl_data_exit(g.handle)
    assert np.array_equal(graphed.p, eager.p)
    eager.close()
    graphed.close()


def test_separate_handles_run_concurrently():
    """Separate handles may run at the same time from separate host threads on
    their own streams (graph capture is thread-local). Four grids, two of them
    with graph replay and two profiled (launched nest by nest), run
    concurrently and must equal the same runs made one after another."""
    import threading

    say("concurrent handles")
    probs = [synth.make_problem(40 + 7 * t, 33, 29 + t, seed=90 + t) for t in range(4)]

    def run(a, profiled, out, slot):
        g = ofl.Grid(a, torch_memory=True)
        ofl.ofl_set_profiling(g.handle, profiled)
        ofl.ofl_data_enter(g.handle)
        xs = [ofl.ofl_jacobi_run(g.handle, 9, OMEGA) for _ in range(3)]
        ofl.ofl_data_exit(g.handle)
        out[slot] = (g.p.copy(), xs)
        g.close()

    seq = [None] * 4
    for t, a in enumerate(probs):
        run(a, t % 2 == 1, seq, t)
    par = [None] * 4
    errors = []

    def guarded(t, a):
        try:
            run(a, t % 2 == 1, par, t)
        except Exception as e:  # reported below, in the test's own thread
            errors.append(e)

    threads = [threading.Thread(target=guarded, args=(t, a)) for t, a in enumerate(probs)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for (p_s, x_s), (p_p, x_p) in zip(seq, par):
        assert np.array_equal(p_s, p_p) and x_s == x_p


# -------------------------------------------------------------------- tuner


def test_grid_tuner_small_search():
    say("grid GA tuner")
    a = synth.make_problem(67, 45, 37, seed=21)
    g = ofl.Grid(a)
    res = ofl.ofl_grid_tune(g.handle, ofl.ga_params(population=4, generations=2, probe_iters=2, repeats=1))
    assert res.best_ms > 0 and res.evaluated >= 1
    assert np.array_equal(g.p, a["p"])  # tuning leaves the iterate alone
    t = ofl.ofl_get_tile(g.handle)
    assert t.as_dict() == res.best.as_dict()
    gosa = ofl.ofl_jacobi_run(g.handle, 5, OMEGA)
    check_against_oracle(a, g, gosa, 5)
    g.close()


def test_offload_gene_search():
    say("offload gene GA")
    a = synth.make_problem(66, 35, 40, seed=23)
    g = ofl.Grid(a)
    r = ofl.ofl_grid_search_offload(g.handle, 4, OMEGA, ofl.ga_params(population=6, generations=3, seed=9))
    assert 0 <= r.mask <= 7 and r.xfer_mode in (0, 1)
    assert r.best_ms > 0 and r.cpu_ms > 0 and r.evaluated >= 2
    assert np.array_equal(g.p, a["p"])             # the search leaves the iterate alone
    gosa = ofl.ofl_jacobi_run(g.handle, 4, OMEGA)   # the chosen gene is applied
    check_against_oracle(a, g, gosa, 4)
    g.close()


def test_batch_tuner_small_search():
    say("batch GA tuner")
    probs = _small_batch(3)
    grids = [ofl.Grid(a) for a in probs]
    b = ofl.ofl_batch_create([g.handle for g in grids])
    res = ofl.ofl_batch_tune(b, ofl.ga_params(population=4, generations=2, probe_iters=2, repeats=1))
    assert res.best_ms > 0
    for a, g in zip(probs, grids):
        assert np.array_equal(g.p, a["p"])
    gosa = ofl.ofl_batch_run(b, 4, OMEGA, len(grids))
    for a, g, r in zip(probs, grids, gosa):
        check_against_oracle(a, g, r, 4)
    ofl.ofl_batch_destroy(b)
    for g in grids:
        g.close()
