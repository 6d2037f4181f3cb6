"""CPU-only checks of the C interface: it loads, exports every declared entry
point, validates arguments, and its host logic (planner, CPU loop nests,
bfloat16 encoding) behaves as specified. No GPU is touched."""

import ctypes
import subprocess

import numpy as np
import pytest

import oracle
import paper_2011_03602_amd as ofl
import synth
from helpers import OMEGA, TOL_GOSA_F32, TOL_P_F32, boundary_equal, header_functions, p_rel_err, rel_err


def test_library_loads_and_exports_every_declared_symbol():
    lib = ofl.lib()
    names = header_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", ofl.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    assert set(names) <= exported
    assert ofl.ofl_version().startswith("ofl ")


def test_binding_covers_every_entry_point():
    names = header_functions()
    assert [n for n in names if not callable(getattr(ofl, n, None))] == []


def test_library_never_links_the_oracle():
    deps = subprocess.run(["ldd", ofl.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in deps
    syms = subprocess.run(["nm", "-D", ofl.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle_" not in syms


def _desc(arrays, **kw):
    K, J, I = arrays["p"].shape
    d = ofl.OflGridDesc()
    d.I, d.J, d.K = I, J, K
    d.p = arrays["p"].ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    d.wrk2 = arrays["wrk2"].ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    for n, name in enumerate(ofl.COEF_NAMES):
        d.coef[n] = arrays[name].ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    d.device = -1
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_create_validates_arguments():
    a = synth.make_problem(5, 4, 3)
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_grid_create(_desc(a, I=2))
    assert e.value.code == ofl.OFL_EINVAL
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_grid_create(_desc(a, coef_format=7))
    assert e.value.code == ofl.OFL_EINVAL
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_grid_create(_desc(a, sum_mode=3))
    assert e.value.code == ofl.OFL_EINVAL
    d = _desc(a)
    d.coef[5] = None
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_grid_create(d)
    assert e.value.code == ofl.OFL_EINVAL
    assert "coefficient" in ofl.ofl_last_error()
    with pytest.raises(ofl.OflError):
        ofl.ofl_grid_device_bytes(3, 3, 2)
    for bad in (1, 3, 6, 64, -4):
        with pytest.raises(ofl.OflError) as e:
            ofl.ofl_grid_create(_desc(a, row_align=bad))
        assert e.value.code == ofl.OFL_EINVAL and "row_align" in ofl.ofl_last_error()
    for good in (0, 4, 8, 16, 32):  # accepted; no device memory is taken at creation
        ofl.ofl_grid_destroy(ofl.ofl_grid_create(_desc(a, row_align=good)))


def test_device_bytes_follow_the_row_alignment():
    """A compact row alignment also pads each plane to 64 elements, so it can
    need more device memory than 128-byte rows: the arena size must follow
    desc.row_align. Pinned on two shapes where it does (FP32, 12 arrays of
    coefficients + p + wrk2 with their guards, staging, partials)."""
    assert ofl.ofl_grid_device_bytes(96, 33, 65, ofl.OFL_COEF_F32, 4) == 12_603_392
    assert ofl.ofl_grid_device_bytes(96, 33, 65, ofl.OFL_COEF_F32, 0) == 12_488_704
    assert ofl.ofl_grid_device_bytes(32, 33, 65, ofl.OFL_COEF_F32, 32) == 4_366_336
    assert ofl.ofl_grid_device_bytes(32, 33, 65, ofl.OFL_COEF_F32, 0) == 4_251_648
    # a lower bound from the layout's rules, for every alignment and format:
    # compact rows share one pitch; 128-byte rows give the coefficient arrays
    # rows that end before the boundary column i = I-1
    def up(x, a):
        return -(-x // a) * a

    for I, J, K in [(3, 3, 3), (33, 33, 65), (97, 41, 12), (161, 7, 9), (257, 5, 4)]:
        for fmt, eb in ((ofl.OFL_COEF_F32, 4), (ofl.OFL_COEF_BF16_OFFSET, 2)):
            for ra in (0, 4, 8, 16, 32):
                if ra:
                    plane = cplane = up(up(I, ra) * J, 64)
                else:
                    plane, cplane = up(I, 32) * J, up(I - 1, 128 // eb) * J
                need = 12 * (cplane * K + 2 * 1024) * eb + 2 * (plane * K + 2 * 1024) * 4 + I * J * K * 4
                assert ofl.ofl_grid_device_bytes(I, J, K, fmt, ra) >= need, (I, J, K, fmt, ra)
    # 257 points per row: 256-element coefficient rows, 288-element rows of p
    # and wrk2 (one layout for all arrays took 288 FP32 or 320 bfloat16
    # elements per row), each array with 1024 elements of guard on each side,
    # plus the staging buffer, partials and alignment
    for fmt, eb in ((ofl.OFL_COEF_F32, 4), (ofl.OFL_COEF_BF16_OFFSET, 2)):
        arrays = 12 * (256 * 257 * 513 + 2048) * eb + 2 * (288 * 257 * 513 + 2048) * 4
        extra = ofl.ofl_grid_device_bytes(257, 257, 513, fmt, 0) - arrays - 257 * 257 * 513 * 4
        assert 8 * 2048 <= extra < 8 * 2048 + 16 * 4096, (fmt, extra)
    for bad in (1, 3, 64, -4):
        with pytest.raises(ofl.OflError) as e:
            ofl.ofl_grid_device_bytes(33, 33, 65, ofl.OFL_COEF_F32, bad)
        assert e.value.code == ofl.OFL_EINVAL and "row_align" in ofl.ofl_last_error()


def test_library_bias_equals_the_oracle_bias():
    """The library's bfloat16-offset encoder (C++, at grid creation) and the
    oracle's offset_bias are two independent derivations of the bias: they
    must agree exactly on every array of a seeded problem, and on arrays that
    tell the mid-range from the mean and from zero."""
    a = synth.make_problem(19, 11, 9, seed=3)
    rng = np.random.default_rng(11)
    n = a["a0"].size
    e = 2.0 ** -20
    a["a1"] = (0.95 + 0.1 * rng.uniform(0, 1, n) ** 6).astype(np.float32).reshape(a["a1"].shape)
    a["wrk1"] = np.where(rng.uniform(0, 1, n) < 0.5, 0.5, -3.0).astype(np.float32).reshape(a["wrk1"].shape)
    b0 = np.full(n, 1 + e, np.float32)
    b0[-1] = 1.5 + e
    a["b0"] = b0.reshape(a["b0"].shape)
    g = ofl.Grid(a, coef_format=ofl.OFL_COEF_BF16_OFFSET)
    lib_bias = ofl.ofl_grid_coef_bias(g.handle)
    for k, name in enumerate(ofl.COEF_NAMES):
        assert lib_bias[k] == oracle.offset_bias(a[name]), name
    assert lib_bias[ofl.COEF_NAMES.index("b0")] == np.float32(1 + e + 0.25)
    assert lib_bias[ofl.COEF_NAMES.index("wrk1")] == 0.0
    g.close()


def test_fused_residual_refused_for_compensated_sums():
    """The fused residual sums in FP64 only: a grid that asks for the
    compensated FP32 sum cannot have it fused (a copy-back exchange alone is fine)."""
    g = ofl.Grid(synth.make_problem(6, 5, 4), sum_mode=ofl.OFL_SUM_KAHAN_F32)
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_set_fusion(g.handle, ofl.OFL_FUSE_RESIDUAL)
    assert e.value.code == ofl.OFL_ENOTSUP and "FP64" in ofl.ofl_last_error()
    ofl.ofl_set_fusion(g.handle, ofl.OFL_FUSE_COPYBACK_SWAP)
    g.close()


def test_run_validates_arguments():
    g = ofl.Grid(synth.make_problem(6, 5, 4))
    h = g.handle
    for bad in (lambda: ofl.ofl_set_offload_mask(h, 8), lambda: ofl.ofl_set_offload_mask(h, 1, 5),
                lambda: ofl.ofl_jacobi_run(h, -1, 0.8), lambda: ofl.ofl_jacobi_run(h, 1, 0.0),
                lambda: ofl.ofl_jacobi_run(h, 1, float("nan")),
                lambda: ofl.ofl_set_tile(h, ofl.tile(vec=3)), lambda: ofl.ofl_set_tile(h, ofl.tile(rows=9)),
                lambda: ofl.ofl_set_tile(h, ofl.tile(kchunk=0)), lambda: ofl.ofl_set_tile(h, ofl.tile(flags=32)),
                lambda: ofl.ofl_set_fusion(h, 4), lambda: ofl.ofl_set_profiled_nests(h, 8)):
        with pytest.raises(ofl.OflError) as e:
            bad()
        assert e.value.code == ofl.OFL_EINVAL
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_data_exit(h)
    assert e.value.code == ofl.OFL_ESTATE
    g.close()


def test_default_tile_follows_row_length_format_and_fusion():
    """A new grid's sweep tile: the vector width from the row length, 2-plane
    chunks, non-temporal loads, and non-temporal stores for FP32 coefficients
    or, for the bfloat16 formats, while the copy-back is a buffer exchange; for
    FP32 at 4 points per lane, at most 3 resident work-groups per CU and, unless
    the residual is fused, coefficients loaded a step ahead. A tile the caller
    sets stays, whatever the fusion."""
    nt, ns = ofl.OFL_TILE_NT_LOADS, ofl.OFL_TILE_NT_STORES
    f32, bf = ofl.OFL_COEF_F32, ofl.OFL_COEF_BF16_OFFSET
    swap = ofl.OFL_FUSE_COPYBACK_SWAP
    for I, fmt, fusion, vec, flags in [(300, f32, 0, 4, nt | ns), (100, f32, 0, 2, nt | ns), (40, f32, 0, 1, nt | ns),
                                       (300, bf, 0, 4, nt), (40, ofl.OFL_COEF_BF16, 0, 1, nt),
                                       (300, bf, swap, 4, nt | ns), (300, bf, ofl.OFL_FUSE_RESIDUAL, 4, nt),
                                       (300, f32, swap, 4, nt | ns), (300, f32, ofl.OFL_FUSE_RESIDUAL, 4, nt | ns)]:
        g = ofl.Grid(synth.make_problem(I, 5, 4), coef_format=fmt)
        ofl.ofl_set_fusion(g.handle, fusion)
        f32v4 = fmt == f32 and vec == 4
        if f32v4 and not fusion & ofl.OFL_FUSE_RESIDUAL:
            flags |= ofl.OFL_TILE_PREFETCH
        want = dict(vec=vec, rows=4, kchunk=2, flags=flags, occupancy=3 if f32v4 else 0)
        assert ofl.ofl_get_tile(g.handle).as_dict() == want, (I, fmt, fusion)
        ofl.ofl_set_fusion(g.handle, 0)
        pf = ofl.OFL_TILE_PREFETCH if f32v4 else 0
        assert ofl.ofl_get_tile(g.handle).flags == (nt | ns | pf if fmt == f32 else nt)
        g.close()
    g = ofl.Grid(synth.make_problem(300, 5, 4), coef_format=bf)
    mine = ofl.tile(vec=2, rows=3, kchunk=5, flags=nt)
    ofl.ofl_set_tile(g.handle, mine)
    ofl.ofl_set_fusion(g.handle, swap)
    assert ofl.ofl_get_tile(g.handle).as_dict() == mine.as_dict()
    g.close()


def test_zero_iterations_leave_p_alone():
    a = synth.make_problem(6, 5, 4)
    g = ofl.Grid(a)
    ofl.ofl_set_offload_mask(g.handle, 0)
    assert np.isnan(ofl.ofl_jacobi_run(g.handle, 0, OMEGA))
    assert np.array_equal(g.p, a["p"])
    g.close()


def test_gpu_mask_without_gpu_reports_device_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    g = ofl.Grid(synth.make_problem(6, 5, 4))
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_jacobi_run(g.handle, 1, OMEGA)
    assert e.value.code == ofl.OFL_EDEVICE
    # No silent CPU fallback happened and nothing moved.
    s = ofl.ofl_get_stats(g.handle)
    assert list(s.cpu_nests) == [0, 0, 0] and s.h2d_count == 0
    g.close()


# ----------------------------------------------------------------- planner

# Steady-state transfers per iteration (arrays), per mask (bit0 S, bit1 R,
# bit2 C; 1 = GPU): hoisted vs per-iteration placement.
STEADY = {0: (0, 0), 1: (2, 14), 2: (2, 2), 3: (2, 16), 4: (2, 3), 5: (2, 17), 6: (2, 5), 7: (0, 19)}


@pytest.mark.parametrize("mask", range(8))
def test_planner_steady_state_counts(mask):
    hoisted, per_iter = STEADY[mask]
    for mode, want in ((ofl.OFL_XFER_HOISTED, hoisted), (ofl.OFL_XFER_PER_ITER, per_iter)):
        xs, _, _ = ofl.ofl_plan(mask, mode, 4, True)
        for it in (1, 2):
            assert len([x for x in xs if x[0] == it]) == want, (mask, mode, it)


def test_planner_hoisted_all_gpu_moves_inputs_once():
    xs, hv, dv = ofl.ofl_plan(7, ofl.OFL_XFER_HOISTED, 100, True)
    h2d = [x for x in xs if x[4] == 0]
    d2h = [x for x in xs if x[4] == 1]
    assert sorted(x[3] for x in h2d) == list(range(13))      # 12 read-only arrays + p, once
    assert all(x[0] == 0 and x[1] == 0 and x[2] == 0 for x in h2d)
    assert [(x[0], x[3]) for x in d2h] == [(100, ofl.OFL_ARR_P)]  # p comes home after the loop
    assert hv[ofl.OFL_ARR_P] == 1 and dv[ofl.OFL_ARR_P] == 1


def test_planner_read_only_arrays_never_move_when_sweep_on_cpu():
    for mask in (0, 2, 4, 6):
        for mode in (0, 1):
            xs, _, _ = ofl.ofl_plan(mask, mode, 3, True)
            assert all(x[3] >= 12 for x in xs), (mask, mode)


def test_planner_exact_lists_for_mixed_masks():
    # mask 001 hoisted: S on GPU, R and C on CPU
    xs, _, _ = ofl.ofl_plan(1, ofl.OFL_XFER_HOISTED, 2, True)
    it1 = [x for x in xs if x[0] == 1]
    assert it1 == [(1, 0, 0, ofl.OFL_ARR_P, 0), (1, 1, 0, ofl.OFL_ARR_WRK2, 1)]
    # mask 100 per-iteration: C on GPU copies wrk2 and p in, p out
    xs, _, _ = ofl.ofl_plan(4, ofl.OFL_XFER_PER_ITER, 1, True)
    assert xs == [(0, 2, 0, ofl.OFL_ARR_WRK2, 0), (0, 2, 0, ofl.OFL_ARR_P, 0), (0, 2, 1, ofl.OFL_ARR_P, 1)]


def test_planner_state_roundtrip_and_no_stale_overwrite():
    # p newest on the device: a GPU nest in per-iteration mode must not upload the stale host copy
    hv = [1] * 14
    dv = [0] * 14
    hv[ofl.OFL_ARR_P] = 0
    dv[ofl.OFL_ARR_P] = 1
    for a in range(12):
        dv[a] = 1
    xs, hv2, dv2 = ofl.ofl_plan(7, ofl.OFL_XFER_PER_ITER, 1, False, hv, dv)
    assert (0, 0, 0, ofl.OFL_ARR_P, 0) not in xs
    with pytest.raises(ofl.OflError):
        ofl.ofl_plan(7, 1, 1, True, [0] * 14, [0] * 14)


@pytest.mark.parametrize("mask", range(8))
def test_planner_bytes_per_iteration_at_129x129x257(mask):
    n = 129 * 129 * 257
    hoisted, per_iter = STEADY[mask]
    for mode, want in ((1, hoisted), (0, per_iter)):
        xs, _, _ = ofl.ofl_plan(mask, mode, 3, True)
        assert 4 * n * len([x for x in xs if x[0] == 1]) == 4 * n * want


# --------------------------------------------------------- host loop nests


@pytest.mark.parametrize("dims,iters", [((33, 33, 65), 50), ((17, 9, 12), 7), ((3, 3, 3), 3), ((4, 7, 3), 2)])
def test_all_cpu_mask_matches_oracle(dims, iters):
    a = synth.make_problem(*dims)
    g = ofl.Grid(a)
    ofl.ofl_set_offload_mask(g.handle, ofl.OFL_MASK_ALL_CPU)
    gosa = ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
    p_ref, g_ref = oracle.jacobi(a, iters, float(OMEGA))
    assert p_rel_err(g.p, p_ref) <= TOL_P_F32
    assert rel_err(gosa, g_ref) <= TOL_GOSA_F32
    assert boundary_equal(g.p, a["p"])
    s = ofl.ofl_get_stats(g.handle)
    assert list(s.cpu_nests) == [iters] * 3 and list(s.gpu_nests) == [0, 0, 0]
    g.close()


def test_cpu_residual_entry_point():
    a = synth.make_problem(19, 11, 13)
    g = ofl.Grid(a)
    ofl.ofl_set_offload_mask(g.handle, 0)
    r = ofl.ofl_residual(g.handle)
    assert rel_err(r, oracle.residual(a)) <= TOL_GOSA_F32
    assert np.array_equal(g.p, a["p"])
    g.close()


@pytest.mark.parametrize("fmt", [ofl.OFL_COEF_BF16, ofl.OFL_COEF_BF16_OFFSET])
def test_bf16_bias_and_cpu_nests_match_oracle_on_decoded_inputs(fmt):
    a = synth.make_problem(21, 13, 17)
    g = ofl.Grid(a, coef_format=fmt)
    bias = ofl.ofl_grid_coef_bias(g.handle)
    dec = dict(a)
    for n, name in enumerate(ofl.COEF_NAMES):
        want = oracle.offset_bias(a[name]) if fmt == ofl.OFL_COEF_BF16_OFFSET else np.float32(0)
        assert bias[n].tobytes() == np.float32(want).tobytes(), name
        dec[name] = oracle.offset_bf16_decode(a[name], want)
    ofl.ofl_set_offload_mask(g.handle, 0)
    gosa = ofl.ofl_jacobi_run(g.handle, 10, OMEGA)
    p_ref, g_ref = oracle.jacobi(dec, 10, float(OMEGA))
    assert p_rel_err(g.p, p_ref) <= TOL_P_F32
    assert rel_err(gosa, g_ref) <= TOL_GOSA_F32
    g.close()


def test_split_cpu_runs_equal_one_run():
    a = synth.make_problem(15, 12, 10)
    g1 = ofl.Grid(a)
    g2 = ofl.Grid(a)
    for g in (g1, g2):
        ofl.ofl_set_offload_mask(g.handle, 0)
    r1 = ofl.ofl_jacobi_run(g1.handle, 6, OMEGA)
    ofl.ofl_jacobi_run(g2.handle, 3, OMEGA)
    r2 = ofl.ofl_jacobi_run(g2.handle, 3, OMEGA)
    assert np.array_equal(g1.p, g2.p) and r1 == r2


def test_gemm_argument_checks_need_no_gpu():
    for args in ((-1, 1, 1, 0, 1, 0, 1, 0, 1), (2, 2, 2, 0, 1, 0, 2, 0, 2), (2, 2, 2, 0, 2, 0, 1, 0, 2),
                 (2, 2, 2, 0, 2, 0, 2, 0, 1), (2, 2, 2, 0, 2, 0, 2, 0, 2), (2, 2, 0, 0, 0, 0, 2, 0, 2),
                 (65535 * 128 + 1, 1, 1, 8, 1, 8, 1, 8, 1)):
        with pytest.raises(ofl.OflError) as e:
            ofl.ofl_gemm_f32(*args, None)
        assert e.value.code == ofl.OFL_EINVAL, args
    ofl.ofl_gemm_f32(0, 4, 3, 0, 3, 0, 4, 0, 4, None)  # empty result: nothing read or written
    ofl.ofl_gemm_f32(5, 0, 3, 0, 3, 0, 0, 0, 0, None)


def test_static_run_refuses_a_grid_that_is_not_resident():
    """ofl_jacobi_run_static allocates nothing, so it needs the device state and
    an open data region; here neither exists and nothing runs."""
    g = ofl.Grid(synth.make_problem(6, 5, 4))
    p0 = g.p.copy()
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_jacobi_run_static(g.handle, 2, OMEGA)
    assert e.value.code == ofl.OFL_ESTATE and "data region" in ofl.ofl_last_error()
    for bad in ((-1, OMEGA), (1, 0.0), (1, float("inf"))):
        with pytest.raises(ofl.OflError) as e:
            ofl.ofl_jacobi_run_static(g.handle, *bad)
        assert e.value.code == ofl.OFL_EINVAL
    assert np.array_equal(g.p, p0)
    g.close()


def test_eight_point_tiles_are_checked_against_the_layout():
    """tile.vec 8 (two rows per wave, 16-byte bfloat16 loads) marches along k
    only, needs a row pitch that is a multiple of 8 elements, and is refused
    for batches; the checks run on the host, before any device work."""
    a = synth.make_problem(45, 9, 7)
    g = ofl.Grid(a)
    ofl.ofl_set_tile(g.handle, ofl.tile(vec=8, rows=4, kchunk=2, flags=3))
    assert ofl.ofl_get_tile(g.handle).vec == 8
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_set_tile(g.handle, ofl.tile(vec=8, rows=4, kchunk=2, flags=ofl.OFL_TILE_MARCH_J))
    assert e.value.code == ofl.OFL_EINVAL and "MARCH_J" in ofl.ofl_last_error()
    with pytest.raises(ofl.OflError):
        ofl.ofl_set_tile(g.handle, ofl.tile(vec=16))
    g.close()
    # compact rows: 45 points at a 4-element alignment give a 48-element pitch
    # (a multiple of 8), 43 points a 44-element one (not)
    for I, ok in ((45, True), (43, False)):
        g = ofl.Grid(synth.make_problem(I, 9, 7), row_align=4)
        if ok:
            ofl.ofl_set_tile(g.handle, ofl.tile(vec=8, rows=2, kchunk=2))
        else:
            with pytest.raises(ofl.OflError) as e:
                ofl.ofl_set_tile(g.handle, ofl.tile(vec=8, rows=2, kchunk=2))
            assert e.value.code == ofl.OFL_EINVAL and "pitch" in ofl.ofl_last_error()
        g.close()
    g = ofl.Grid(a)
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_batch_create([g.handle], ofl.tile(vec=8, rows=2, kchunk=2))
    assert e.value.code == ofl.OFL_ENOTSUP
    g.close()


def test_library_links_the_marker_api():
    """The nests, transfers and graph launches are marked with ROCTx ranges."""
    deps = subprocess.run(["ldd", ofl.LIB_PATH], capture_output=True, text=True).stdout
    assert "roctx" in deps
