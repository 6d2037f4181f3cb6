#!/usr/bin/env python3
"""Benchmark of the offloaded Jacobi hot path on one MI355X.

One step = one ofl_jacobi_run of 100 iterations (sweep, residual, copy-back,
every nest on the GPU, transfers hoisted) over the 257x257x513 FP32 grid, with
the inputs already resident in HBM (a data region is open before timing).
value = lattice updates per second of the whole iteration, in GLUP/s.

Also reported: the sweep kernel against the HBM roofline (HIP-event time of
every sweep launch inside the timed region, and the counter-measured bytes when
they were taken on the current kernel source) and against the practical
ceiling of its own streaming pattern (13 reads + 1 write per point without the
stencil), a 1:1 copy's rate, the bfloat16-offset, fused and batched forms of
the same metric (batches with the library's default batch tile, or GA-tuned
ones with --tune-batch), every form's error against the FP64 oracle over the
oracle's sample, and the FP64 oracle timed on that bounded sample (the first
50 iterations) on one host thread and on all host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-variants]
       [--skip-cpu-baseline] [--tune-batch] [--profile-only NAME]
       [--config headline|masks|precision|loops|blocks]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GLUP/s + HBM GB/s %peak, 257x257x513 Jacobi: FP32 vs BF16-coef, batched"
PEAK_HBM_GBS = 8000.0
OMEGA = np.float32(0.8)
ITERS = 100
SHAPE = (257, 257, 513)  # I, J, K
SWEEP_BYTES = {"f32": 56, "bf16": 32}  # algorithmic bytes per lattice update of the sweep
ITER_BYTES = {"f32": 72, "bf16": 48}   # sweep + residual + copy-back
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "sweep_f32_257x257x513_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2011_03602_amd", "csrc", "kernels.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def interior(I, J, K):
    return (I - 2) * (J - 2) * (K - 2)


def kernel_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(tile):
    """Counter-measured HBM bytes per sweep launch, if taken on the current
    kernel source with the tile the headline ran (else None)."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_hash() or rec.get("tile") != tile:
        return None
    return rec.get("hbm_bytes_per_launch")


def errors_against(p, gosa, p_ref, g_ref):
    """Relative errors of a result against the FP64 oracle: p as the max-norm
    over the interior (also the L2 norm), the residual as |d| / |ref|."""
    inner = (slice(1, -1),) * 3
    d = np.asarray(p, np.float64)[inner] - p_ref[inner]
    return {"p_max_rel_err": float(np.max(np.abs(d)) / np.max(np.abs(p_ref[inner]))),
            "p_l2_rel_err": float(np.linalg.norm(d) / np.linalg.norm(p_ref[inner])),
            "gosa_rel_err": float(abs(gosa - g_ref) / abs(g_ref))}


def single_error(ofl, arrays, fmt, fusion, iters, p_ref, g_ref):
    """One form on a fresh grid for ``iters`` iterations from the initial
    iterate, in the benchmark's configuration, against the oracle's result."""
    g = ofl.Grid(arrays, coef_format=fmt, torch_memory=True)
    if fusion:
        ofl.ofl_set_fusion(g.handle, fusion)
    ofl.ofl_set_offload_mask(g.handle, ofl.OFL_MASK_ALL_GPU, ofl.OFL_XFER_HOISTED)
    ofl.ofl_data_enter(g.handle)
    gosa = ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
    ofl.ofl_data_exit(g.handle)
    e = errors_against(g.p, gosa, p_ref, g_ref)
    g.close()
    e["iterations"] = iters
    return e


def run_single(ofl, arrays, fmt, steps, warmup, tile=None, profile=True, iters=ITERS, fusion=0):
    """Time `steps` runs of ITERS iterations on one grid; returns a result dict."""
    import torch

    g = ofl.Grid(arrays, coef_format=fmt, torch_memory=True)
    h = g.handle
    if tile is not None:
        ofl.ofl_set_tile(h, tile)
    if fusion:
        ofl.ofl_set_fusion(h, fusion)
    ofl.ofl_set_offload_mask(h, ofl.OFL_MASK_ALL_GPU, ofl.OFL_XFER_HOISTED)
    ofl.ofl_data_enter(h)  # inputs resident in HBM before timing
    for _ in range(warmup):
        ofl.ofl_jacobi_run(h, iters, OMEGA)
    ofl.ofl_reset_stats(h)
    # The sweep (the roofline kernel) is timed live by events around every one
    # of its launches in the timed region; the other nests are not bracketed
    # there (each bracket adds event records between kernels) but in one more
    # profiled step after it.
    ofl.ofl_set_profiled_nests(h, ofl.OFL_NEST_SWEEP)
    ofl.ofl_set_profiling(h, profile)
    # step boundaries: events on the grid's own stream (no host synchronisation between steps)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gosa = None
    marks[0].record(g.stream)
    for n in range(steps):
        gosa = ofl.ofl_jacobi_run(h, iters, OMEGA)
        marks[n + 1].record(g.stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step_ms = sorted(marks[n].elapsed_time(marks[n + 1]) for n in range(steps))
    st = ofl.ofl_get_stats(h)
    st_all = None
    if profile:
        ofl.ofl_reset_stats(h)
        ofl.ofl_set_profiled_nests(h, ofl.OFL_MASK_ALL_GPU)
        ofl.ofl_jacobi_run(h, iters, OMEGA)
        st_all = ofl.ofl_get_stats(h)
    ofl.ofl_set_profiling(h, False)
    tile_used = ofl.ofl_get_tile(h).as_dict()
    ofl.ofl_data_exit(h)
    g.close()
    I, J, K = SHAPE
    lups = interior(I, J, K) * iters * steps
    res = {
        "seconds": dt,
        "ms_per_step": 1e3 * dt / steps,
        "step_ms_median": step_ms[len(step_ms) // 2],
        "step_ms_min": step_ms[0],
        "glups": lups / dt / 1e9,
        "gosa": gosa,
        "tile": tile_used,
        "h2d_in_timed_region": int(st.h2d_count),
        "d2h_in_timed_region": int(st.d2h_count),
    }
    if profile:
        # sweep: every launch of the timed region; residual and copy-back: the extra step
        res["nest_ms_avg"] = [st.kernel_ms[0] / max(1, st.timed_nests[0])] + [
            st_all.kernel_ms[n] / max(1, st_all.timed_nests[n]) for n in (1, 2)]
        res["nest_launches"] = [int(st.timed_nests[0])] + [int(st_all.timed_nests[n]) for n in (1, 2)]
    return res


def end_to_end(ofl, arrays, reps=3):
    """The headline step with its transfers: ofl_jacobi_run of 100 iterations
    on a grid whose inputs start in (pinned) host memory and whose p comes back
    at the end, the hoisted placement's 13 uploads and 1 download. Reported
    beside the resident figure, never as `value`."""
    import torch

    res = []
    for _ in range(reps + 1):
        # a fresh grid: its device block comes from PyTorch's arena, and the
        # run takes its device state (block zeroed once), uploads the inputs,
        # iterates and brings p back before returning
        g = ofl.Grid(arrays, torch_memory=True, pinned=True)
        ofl.ofl_set_offload_mask(g.handle, ofl.OFL_MASK_ALL_GPU, ofl.OFL_XFER_HOISTED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ofl.ofl_jacobi_run(g.handle, ITERS, OMEGA)
        dt = time.perf_counter() - t0
        st = ofl.ofl_get_stats(g.handle)
        res.append((dt, int(st.h2d_count), int(st.d2h_count), (st.h2d_bytes + st.d2h_bytes) / 1e9))
        g.close()
    res = sorted(res[1:])
    dt, h2d, d2h, gb = res[len(res) // 2]
    I, J, K = SHAPE
    return {"glups": round(interior(I, J, K) * ITERS / dt / 1e9, 3), "ms_per_step": round(dt * 1e3, 3),
            "h2d": h2d, "d2h": d2h, "pcie_gb": round(gb, 3),
            "note": "one 100-iteration run on a fresh grid, from pinned host inputs to p back on the host: device "
                    "state, 13 uploads, the iterations and 1 download (median of 3)"}


def run_batch(ofl, probs, fmt, steps, warmup, tune, iters=ITERS, row_align=0, check=None):
    """The uneven grids in one batch: plain and fused graph runs against the
    same grids run one after another with single-grid calls. ``row_align``:
    the grids' device row alignment (4: packed rows in the batch). ``check``:
    (iterations, {grid index: oracle (p, gosa)}); each form's first run is
    that many iterations from the initial iterate, and its worst error on
    those grids against the oracle is reported."""
    import torch

    n_grids = len(probs)
    total_lups = sum(interior(*shape) for shape, _ in probs) * iters

    def setup():
        grids = [ofl.Grid(arr, coef_format=fmt, row_align=row_align) for _, arr in probs]
        for g in grids:
            ofl.ofl_data_enter(g.handle)
        return grids, ofl.ofl_batch_create([g.handle for g in grids])

    def teardown(grids, b):
        ofl.ofl_batch_destroy(b)
        for g in grids:
            ofl.ofl_data_exit(g.handle)
            g.close()

    def oracle_error(grids, b):
        if not check:
            return None
        n_it, refs = check
        gosa = ofl.ofl_batch_run(b, n_it, OMEGA, n_grids)
        worst = {"p_max_rel_err": 0.0, "gosa_rel_err": 0.0}
        for t, (p_ref, g_ref) in refs.items():
            ofl.ofl_update_host(grids[t].handle)
            e = errors_against(grids[t].p, gosa[t], p_ref, g_ref)
            worst = {k: max(worst[k], e[k]) for k in worst}
        worst.update(iterations=n_it, grids=sorted(refs))
        return worst

    def timed(b):
        for _ in range(warmup):
            ofl.ofl_batch_run(b, iters, OMEGA, n_grids)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ofl.ofl_batch_run(b, iters, OMEGA, n_grids)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    tuned = None
    errors = {}
    grids, b = setup()
    if tune:
        log("GA tile search for the batch")
        r = ofl.ofl_batch_tune(b, ofl.ga_params(population=10, generations=6, probe_iters=10, repeats=2))
        tuned = {"tile": r.best.as_dict(), "probe_ms": r.best_ms, "evaluated": r.evaluated, "rejected": r.rejected}
    errors["plain"] = oracle_error(grids, b)
    dt_batch = timed(b)
    tile_used = ofl.ofl_batch_get_tile(b).as_dict()
    ofl.ofl_batch_destroy(b)
    # baseline: the same grids one after another, plain single-grid runs
    for g in grids:
        ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in grids:
        ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    for g in grids:
        ofl.ofl_data_exit(g.handle)
        g.close()
    # the fused form on fresh grids, so that its check starts from the initial iterate
    grids, b = setup()
    if tuned:
        ofl.ofl_batch_set_tile(b, ofl.tile(**tuned["tile"]))
    ofl.ofl_batch_set_fusion(b, ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP)
    errors["fused"] = oracle_error(grids, b)
    dt_fused = timed(b)
    teardown(grids, b)
    return {
        "grids": n_grids,
        "lattice_updates": total_lups,
        "glups_batched": round(total_lups / dt_batch / 1e9, 3),
        "glups_batched_fused": round(total_lups / dt_fused / 1e9, 3),
        "glups_sequential": round(total_lups / dt_seq / 1e9, 3),
        "ms_batched": round(1e3 * dt_batch, 3),
        "ms_batched_fused": round(1e3 * dt_fused, 3),
        "ms_sequential": round(1e3 * dt_seq, 3),
        "tile": tile_used,
        "row_align": row_align,
        "tuner": tuned,
        "oracle_error": errors["plain"],
        "oracle_error_fused": errors["fused"],
    }


def run_small(ofl):
    """33x33x65, 50 iterations, genes 000 and 111 (hoisted): per-iteration
    latency of the small grid, which is bound by kernel launches. A warm-up
    run of the same length captures the GPU gene's iteration graph; the
    timed figure is the mean of three runs after it."""
    import torch

    import synth

    I, J, K, iters = 33, 33, 65, 50
    arrays = synth.make_problem(I, J, K)
    out = {}
    for mask in (ofl.OFL_MASK_ALL_CPU, ofl.OFL_MASK_ALL_GPU):
        g = ofl.Grid(arrays, torch_memory=True)
        ofl.ofl_set_offload_mask(g.handle, mask, ofl.OFL_XFER_HOISTED)
        ofl.ofl_data_enter(g.handle)
        ofl.ofl_jacobi_run(g.handle, iters, OMEGA)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 3
        st = ofl.ofl_get_stats(g.handle)
        ofl.ofl_data_exit(g.handle)
        g.close()
        launches = sum(int(x) for x in st.gpu_regions)
        out[format(mask, "03b")] = {"us_per_iteration": round(dt / iters * 1e6, 2),
                                    "glups": round(interior(I, J, K) * iters / dt / 1e9, 4),
                                    "kernel_nests_per_iteration": round(launches / (4 * iters), 2)}
        log(f"33x33x65 gene {mask:03b}: {dt / iters * 1e6:.1f} us per iteration")
    return out


def run_masks(ofl, steps_unused=None):
    """Every gene x placement on 129x129x257 for 200 iterations, end to end
    (transfers included, host arrays in pinned memory), against the all-CPU
    gene (the original program's loops) and the FP64 oracle."""
    import torch

    import oracle
    import synth

    I, J, K, iters = 129, 129, 257, 200
    arrays = synth.make_problem(I, J, K)
    log("oracle: 129x129x257 x200")
    t0 = time.perf_counter()
    p_ref, g_ref = oracle.jacobi(arrays, iters, float(OMEGA))
    t_oracle = time.perf_counter() - t0
    inner = (slice(1, -1),) * 3
    lups = interior(I, J, K) * iters
    rows = []
    for mode, mode_name in ((ofl.OFL_XFER_PER_ITER, "per-iteration"), (ofl.OFL_XFER_HOISTED, "hoisted")):
        for mask in range(8):
            g = ofl.Grid(arrays, torch_memory=True, pinned=True)
            ofl.ofl_set_offload_mask(g.handle, mask, mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gosa = ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = ofl.ofl_get_stats(g.handle)
            err = float(np.max(np.abs(g.p[inner] - p_ref[inner])) / np.max(np.abs(p_ref[inner])))
            rows.append({"mask": mask, "mask_CRS": format(mask, "03b"), "placement": mode_name, "seconds": round(dt, 4),
                         "glups": round(lups / dt / 1e9, 4), "h2d": int(st.h2d_count), "d2h": int(st.d2h_count),
                         "pcie_gb": round((st.h2d_bytes + st.d2h_bytes) / 1e9, 3), "p_rel_err": err,
                         "gosa_rel_err": abs(gosa - g_ref) / abs(g_ref)})
            log(f"mask {mask:03b} {mode_name}: {dt:.3f} s")
            g.close()
    small = run_small(ofl)
    cpu = {r["placement"]: r["seconds"] for r in rows if r["mask"] == 0}
    for r in rows:
        r["speedup_vs_all_cpu_gene"] = round(cpu[r["placement"]] / r["seconds"], 2)
        r["speedup_vs_oracle"] = round(t_oracle / r["seconds"], 2)
    return {"config": "129x129x257 FP32, 200 iterations, every gene x placement", "small_33x33x65": small,
            "oracle_seconds": round(t_oracle, 3),
            "host_threads_cpu_nests": os.environ.get("OFL_CPU_THREADS") or os.environ.get("OMP_NUM_THREADS")
            or os.cpu_count(), "rows": rows}


def run_loops(ofl):
    """Per-loop genes (the region of a GPU nest opening at its k, j or i loop):
    end-to-end times of uniform region levels at 129x129x257, both placements,
    and the loop-gene GA at 65x65x129 against the all-CPU gene."""
    import torch

    import synth

    out = {"config": "loop genes: region level per nest, mask 111", "granularity": [], "search": []}
    I, J, K = 129, 129, 257
    arrays = synth.make_problem(I, J, K)
    names = {ofl.OFL_LEVEL_K: "k", ofl.OFL_LEVEL_J: "j", ofl.OFL_LEVEL_I: "i"}
    for mode, mode_name in ((ofl.OFL_XFER_HOISTED, "hoisted"), (ofl.OFL_XFER_PER_ITER, "per-iteration")):
        for lev in (ofl.OFL_LEVEL_K, ofl.OFL_LEVEL_J, ofl.OFL_LEVEL_I):
            iters = 1 if (mode == ofl.OFL_XFER_PER_ITER and lev == ofl.OFL_LEVEL_I) else 5
            g = ofl.Grid(arrays, torch_memory=True, pinned=True)
            ofl.ofl_set_regions(g.handle, 7, [lev] * 3, mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = ofl.ofl_get_stats(g.handle)
            row = {"grid": f"{I}x{J}x{K}", "level": names[lev], "placement": mode_name, "iterations": iters,
                   "seconds": round(dt, 4), "ms_per_iteration": round(dt * 1e3 / iters, 3),
                   "launch_regions": [int(x) for x in st.gpu_regions], "h2d": int(st.h2d_count),
                   "d2h": int(st.d2h_count), "pcie_gb": round((st.h2d_bytes + st.d2h_bytes) / 1e9, 3)}
            out["granularity"].append(row)
            log(f"regions at {names[lev]}, {mode_name}: {dt:.3f} s for {iters} iterations")
            g.close()
    I, J, K, iters = 65, 65, 129, 5
    arrays = synth.make_problem(I, J, K, seed=7)
    for mode, mode_name in ((ofl.OFL_XFER_HOISTED, "hoisted"), (ofl.OFL_XFER_PER_ITER, "per-iteration")):
        g = ofl.Grid(arrays, torch_memory=True, pinned=True)
        t0 = time.perf_counter()
        r = ofl.ofl_grid_search_loops(g.handle, iters, OMEGA, mode, 0.0,
                                      ofl.ga_params(population=16, generations=12, repeats=1))
        dt = time.perf_counter() - t0
        out["search"].append({"grid": f"{I}x{J}x{K}", "iterations": iters, "placement": mode_name,
                              "gene": format(r.gene, "09b"), "mask_CRS": format(r.mask, "03b"),
                              "levels_SRC": "".join(names[r.level[n]] if (r.mask >> n) & 1 else "-" for n in range(3)),
                              "best_ms": round(r.best_ms, 3), "all_cpu_ms": round(r.cpu_ms, 3),
                              "speedup_vs_all_cpu_gene": round(r.cpu_ms / r.best_ms, 2), "gene_bits": r.gene_bits,
                              "genes_scored": r.evaluated, "patterns_measured": r.patterns,
                              "wrong": r.rejected, "timed_out": r.timed_out, "search_seconds": round(dt, 2)})
        log(f"loop-gene search, {mode_name}: gene {r.gene:09b} in {dt:.1f} s")
        g.close()
    out["frontend"] = run_frontend(ofl)
    return out


FRONTEND_PROGRAM = os.path.join(ROOT, "tests", "programs", "relax.py")


def run_frontend(ofl):
    """The same Jacobi program written in Python with its own names, read by the
    front end and offloaded through the library: analysis time, the run
    (ofl_jacobi_run, transfers included) against the same gene set through the
    interface directly, the front end's setup and write-back, and the
    interpreted program's own rate."""
    import torch

    import synth
    from paper_2011_03602_amd import frontend as fe

    src = open(FRONTEND_PROGRAM).read()
    t0 = time.perf_counter()
    prog = fe.analyse(src)
    t_analyse = time.perf_counter() - t0
    names = {lib: a for a, lib in prog.binding.items()}
    I, J, K, iters = 129, 129, 257, 200
    arrays = synth.make_problem(I, J, K)
    lups = interior(I, J, K) * iters
    res = {"program": "tests/programs/relax.py", "analysis_ms": round(t_analyse * 1e3, 2),
           "grid": f"{I}x{J}x{K}", "iterations": iters, "rows": []}
    for label, gene in (("whole nests", 0b001_001_001), ("per-plane regions", 0b010_010_010)):
        for via in ("direct", "frontend"):
            runs = []
            for _ in range(3):
                torch.cuda.synchronize()
                if via == "direct":
                    t0 = time.perf_counter()
                    g = ofl.Grid(arrays)
                    ofl.ofl_set_loop_gene(g.handle, gene, ofl.OFL_XFER_HOISTED)
                    t1 = time.perf_counter()
                    ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
                    t2 = time.perf_counter()
                    g.close()
                    tm = {"setup": t1 - t0, "run": t2 - t1, "writeback": 0.0}
                else:
                    args = {names[k]: v for k, v in arrays.items()}
                    args.update({prog.symbols["omega"]: float(OMEGA), "steps": iters})
                    tm = {}
                    fe.offload(prog, args, gene, timings=tm)
                runs.append(tm)
            best = min(runs, key=lambda t: t["run"])
            res["rows"].append({"gene": label, "via": via, "run_glups": round(lups / best["run"] / 1e9, 3),
                                "run_ms": round(best["run"] * 1e3, 2), "setup_ms": round(best["setup"] * 1e3, 2),
                                "writeback_ms": round(best["writeback"] * 1e3, 2)})
            log(f"front end: {label} via {via}: run {best['run'] * 1e3:.1f} ms")
    small = synth.make_problem(9, 7, 6)
    args = {names[k]: np.array(v, dtype=np.float32) for k, v in small.items()}
    args.update({prog.symbols["omega"]: float(OMEGA), "steps": 2})
    t0 = time.perf_counter()
    fe.run_python(src, args)
    dt = time.perf_counter() - t0
    res["interpreted_program_9x7x6_x2_glups"] = round(interior(9, 7, 6) * 2 / dt / 1e9, 8)
    return res


PEAK_FP32_MFMA_TFLOPS = 157.3
GEMM_SHAPES = ((4096, 4096, 4096), (8192, 8192, 8192), (8192, 4096, 1024))


def time_gemm(ofl, M, N, K, reps=10):
    """Average duration of ofl_gemm_f32 launches (HIP events on the launch stream)."""
    import torch

    g = torch.Generator(device="cuda").manual_seed(M + N + K)
    a = torch.rand((M, K), device="cuda", generator=g)
    b = torch.rand((K, N), device="cuda", generator=g)
    c = torch.empty((M, N), device="cuda")
    s = torch.cuda.current_stream()
    for _ in range(2):
        ofl.ofl_gemm_f32(M, N, K, a.data_ptr(), K, b.data_ptr(), N, c.data_ptr(), N, s.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        ofl.ofl_gemm_f32(M, N, K, a.data_ptr(), K, b.data_ptr(), N, c.data_ptr(), N, s.cuda_stream)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def run_blocks(ofl):
    """Function-block offload: the matrix-product routine against the FP32
    matrix-core peak, and the block trials of a Python program with three
    matrix products (each block alone, then the faster ones combined)."""
    from paper_2011_03602_amd import blocks as fb

    out = {"config": "function blocks: FP32 matrix product on the matrix cores; block trials", "gemm": []}
    for M, N, K in GEMM_SHAPES:
        sec = sorted(time_gemm(ofl, M, N, K) for _ in range(3))[1]  # median of three timings
        tflops = 2.0 * M * N * K / sec / 1e12
        out["gemm"].append({"M": M, "N": N, "K": K, "us": round(sec * 1e6, 1), "tflops": round(tflops, 2),
                            "frac_of_fp32_mfma_peak": round(tflops / PEAK_FP32_MFMA_TFLOPS, 4)})
        log(f"gemm {M}x{N}x{K}: {tflops:.1f} TFLOP/s")
    src = open(os.path.join(ROOT, "tests", "programs", "mlp.py")).read()
    prog = fb.analyse_blocks(src)
    rng = np.random.default_rng(0)
    n, d = 8192, 4096
    args = {"x": rng.uniform(-1, 1, (n, d)).astype(np.float32),
            "w1": (rng.uniform(-1, 1, (d, d)) / np.sqrt(d)).astype(np.float32),
            "w2": (rng.uniform(-1, 1, (d, d)) / np.sqrt(d)).astype(np.float32),
            "w3": (rng.uniform(-1, 1, (d, 16)) / np.sqrt(d)).astype(np.float32)}
    t0 = time.perf_counter()
    res = fb.trial_blocks(prog, args, repeats=3)
    out["trials"] = {"program": "tests/programs/mlp.py", "shapes": "x 8192x4096, w1 w2 4096x4096, w3 4096x16",
                     "blocks": [f"{b.name} (line {b.line})" for b in prog.blocks],
                     "patterns": [{"gene": format(t.gene, f"0{len(prog.blocks)}b"), "seconds": t.seconds,
                                   "status": t.status, "max_rel_err": t.max_rel_err} for t in res["trials"]],
                     "faster_alone": res["faster_alone"], "best_gene": format(res["best"].gene, f"0{len(prog.blocks)}b"),
                     "search_seconds": round(time.perf_counter() - t0, 2)}
    base = next(t for t in res["trials"] if t.gene == 0).seconds
    out["trials"]["speedup_vs_host"] = round(base / res["best"].seconds, 2)
    log(f"block trials: best {out['trials']['best_gene']}, {out['trials']['speedup_vs_host']}x the host program")
    return out


def run_precision(ofl):
    """Errors of every storage format and residual mode against the FP64
    oracle on the FP32 inputs, 257x257x513, 100 iterations."""
    import oracle
    import synth

    I, J, K = SHAPE
    arrays = synth.make_problem(I, J, K)
    log("oracle: 257x257x513 x100 (about a minute)")
    p_ref, g_ref = oracle.jacobi(arrays, ITERS, float(OMEGA))
    inner = (slice(1, -1),) * 3
    ref_inner = p_ref[inner]
    scale = float(np.max(np.abs(ref_inner)))
    out = []
    for fmt, fname in ((ofl.OFL_COEF_F32, "f32"), (ofl.OFL_COEF_BF16, "bf16-plain"),
                       (ofl.OFL_COEF_BF16_OFFSET, "bf16-offset")):
        for sm, sname in ((ofl.OFL_SUM_F64, "f64"), (ofl.OFL_SUM_KAHAN_F32, "kahan-f32")):
            g = ofl.Grid(arrays, coef_format=fmt, sum_mode=sm, torch_memory=True)
            gosa = ofl.ofl_jacobi_run(g.handle, ITERS, OMEGA)
            d = g.p[inner].astype(np.float64) - ref_inner
            out.append({"coef": fname, "residual_sum": sname,
                        "p_max_abs_err": float(np.max(np.abs(d))),
                        "p_max_rel_err": float(np.max(np.abs(d)) / scale),
                        "p_l2_rel_err": float(np.linalg.norm(d) / np.linalg.norm(ref_inner)),
                        "gosa": gosa, "gosa_rel_err": abs(gosa - g_ref) / abs(g_ref)})
            log(f"{fname} {sname}: p max rel {out[-1]['p_max_rel_err']:.2e} gosa rel {out[-1]['gosa_rel_err']:.2e}")
            g.close()
    return {"config": "257x257x513, 100 iterations, errors vs the FP64 oracle on the FP32 inputs",
            "gosa_oracle": g_ref, "rows": out}


def tune_headline(ofl, arrays, fmt):
    """The GA tile search (population 16, 12 generations, 5 iterations per
    probe, median of 3) on the headline grid; returns the tile it picks and
    the search's own figures."""
    g = ofl.Grid(arrays, coef_format=fmt, torch_memory=True)
    ofl.ofl_set_offload_mask(g.handle, ofl.OFL_MASK_ALL_GPU, ofl.OFL_XFER_HOISTED)
    default = ofl.ofl_get_tile(g.handle)
    t0 = time.perf_counter()
    r = ofl.ofl_grid_tune(g.handle, ofl.ga_params())
    dt = time.perf_counter() - t0
    g.close()
    log(f"GA tile search ({'f32' if fmt == 0 else 'bf16'}): {r.best.as_dict()} in {dt:.1f} s")
    return r.best, {"tile": r.best.as_dict(), "probe_ms": round(r.best_ms, 3), "genes_measured": r.evaluated,
                    "genes_rejected": r.rejected, "search_seconds": round(dt, 1),
                    "default_tile": default.as_dict()}


def cpu_program(ofl, arrays, iters):
    """The library's all-CPU gene (the original program's loops, on the host
    threads) on a bounded sample of the headline workload."""
    g = ofl.Grid(arrays)
    ofl.ofl_set_offload_mask(g.handle, ofl.OFL_MASK_ALL_CPU)
    log(f"all-CPU gene: {iters} iterations of 257x257x513 on the host threads")
    t0 = time.perf_counter()
    ofl.ofl_jacobi_run(g.handle, iters, OMEGA)
    dt = time.perf_counter() - t0
    g.close()
    I, J, K = SHAPE
    threads = os.environ.get("OFL_CPU_THREADS") or os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return {"value": round(interior(I, J, K) * iters / dt / 1e9, 4), "unit": "GLUP/s", "threads": int(threads),
            "sample": f"257x257x513 grid, {iters} iterations, FP32, {dt:.2f} s"}


def host_info():
    """The host the CPU baselines ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "cpus_available": len(os.sched_getaffinity(0))}


def copy_rate(ofl, reps=5):
    """The library's copy kernel on 1 GiB: the rate of a 1:1 read + write stream (GB/s moved)."""
    import torch

    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    ofl.ofl_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, s.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        ofl.ofl_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, s.cuda_stream)
    e1.record(s)
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return {"kernel": "copy_kernel, 1 GiB read + 1 GiB written (a 1:1 stream, not the sweep's pattern)",
            "gbs": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}


def pattern_ceilings(ofl, reps=5):
    """The sweep's own streaming pattern without the stencil (ofl_device_stream):
    13 FP32 reads + 1 FP32 write per point, and 1 FP32 + 12 bfloat16 reads + 1
    FP32 write, each over as many points as the headline grid's interior, 14
    separate arrays, linear order. GB/s of the pattern's bytes."""
    import torch

    I, J, K = SHAPE
    n = (interior(I, J, K) + 3) // 4 * 4
    out = {}
    s = torch.cuda.current_stream()
    for name, n32, n16, bpp in (("f32", 13, 0, 56), ("bf16", 1, 12, 32)):
        f = [torch.ones(n, dtype=torch.float32, device="cuda") for _ in range(n32)]
        h = [torch.ones(n, dtype=torch.bfloat16, device="cuda") for _ in range(n16)]
        dst = torch.empty(n, dtype=torch.float32, device="cuda")
        args = ([x.data_ptr() for x in f], [x.data_ptr() for x in h], dst.data_ptr(), n, s.cuda_stream)
        ofl.ofl_device_stream(*args)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            ofl.ofl_device_stream(*args)
        e1.record(s)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        gbs = bpp * n / (us * 1e-6) / 1e9
        out[name] = {"sources": f"{n32} FP32 + {n16} bfloat16, 1 FP32 written", "bytes_per_point": bpp,
                     "points": n, "avg_launch_us": round(us, 2), "gbs": round(gbs, 1),
                     "frac": round(gbs / PEAK_HBM_GBS, 4)}
        del f, h, dst
    return out


def widened(arrays):
    """The inputs in FP64, made before any oracle timing starts."""
    return {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in arrays.items()}


def cpu_baseline(arrays64, iters):
    """The FP64 oracle timed around its iteration loop (the inputs are widened
    beforehand): the single-thread build, and the same oracle.c built with
    OpenMP over k on every host core the run may use. Both give bit-identical
    results (checked here); the all-cores figure is the baseline, the
    single-thread one rides along. Returns (record, (p_ref, gosa_ref))."""
    import oracle
    import oracle.build as ob

    I, J, K = SHAPE
    lups = interior(I, J, K) * iters
    log(f"oracle: {iters} iterations of 257x257x513 in FP64, one host thread")
    t0 = time.perf_counter()
    p_ref, g_ref = oracle.jacobi(arrays64, iters, float(OMEGA))
    dt1 = time.perf_counter() - t0
    if not os.path.exists(ob.LIB_OMP):
        ob.build()
    with oracle.use_library(ob.LIB_OMP):
        threads = oracle.threads()
        log(f"oracle: {iters} iterations of 257x257x513 in FP64, {threads} host threads")
        t0 = time.perf_counter()
        p_all, g_all = oracle.jacobi(arrays64, iters, float(OMEGA))
        dtn = time.perf_counter() - t0
    same = bool(np.array_equal(p_all, p_ref) and g_all == g_ref)
    del p_all
    rec = {
        "value": lups / dtn / 1e9,
        "unit": "GLUP/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"257x257x513 grid, {iters} of the {ITERS} iterations, plain C FP64 oracle built with OpenMP over "
                  f"k, {threads} threads, {dtn:.2f} s around the iteration loop (inputs widened to FP64 beforehand)",
        "bit_identical_to_single_thread": same,
        "single_thread": {"value": lups / dt1 / 1e9, "unit": "GLUP/s", "cores": 1, "seconds": round(dt1, 2)},
        "host": host_info(),
    }
    return rec, (p_ref, g_ref)


def batch_check_refs(probs, iters):
    """Oracle results for four fixed grids of the batch (the smallest, the
    largest and the two around the median interior size), ``iters`` iterations."""
    import oracle

    order = sorted(range(len(probs)), key=lambda t: interior(*probs[t][0]))
    pick = sorted({order[0], order[len(order) // 2 - 1], order[len(order) // 2], order[-1]})
    log(f"oracle: {iters} iterations of batch grids {pick}")
    return {t: oracle.jacobi(probs[t][1], iters, float(OMEGA)) for t in pick}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--skip-variants", action="store_true", help="only the FP32 headline")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--batch-grids", type=int, default=64)
    ap.add_argument("--tune-batch", action=argparse.BooleanOptionalAction, default=False,
                    help="run the GA tile search before each batched run (its 5-iteration probes do not resolve the "
                         "1-2%% between the best tiles; the default batch tile holds the measured choice)")
    ap.add_argument("--batch-row-align", type=int, default=4,
                    help="device row alignment of the batched grids (4: packed rows; 0: 128-byte rows)")
    ap.add_argument("--tune", action="store_true",
                    help="also run the GA tile search on the headline grid and report the tuned tile's run")
    ap.add_argument("--oracle-iters", type=int, default=50)
    ap.add_argument("--profile-only", default=None,
                    help="headline|bf16|batch|copy|gemm: run just that under a profiler, print no JSON")
    ap.add_argument("--profile-iters", type=int, default=ITERS,
                    help="iterations per step in --profile-only runs (counter passes use a few)")
    ap.add_argument("--config", default="headline", choices=["headline", "masks", "precision", "loops", "blocks"],
                    help="headline: the benchmark line; masks: every gene x placement at 129x129x257; "
                         "precision: format/residual errors vs the FP64 oracle at 257x257x513; "
                         "loops: per-loop genes (region levels) and their GA search; "
                         "blocks: the matrix-product routine and function-block trials")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2011_03602_amd as ofl
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ofl.lib()  # fail loudly if the library is missing
    if args.config == "masks":
        print(json.dumps(run_masks(ofl)), flush=True)
        return
    if args.config == "precision":
        print(json.dumps(run_precision(ofl)), flush=True)
        return
    if args.config == "loops":
        print(json.dumps(run_loops(ofl)), flush=True)
        return
    if args.config == "blocks":
        print(json.dumps(run_blocks(ofl)), flush=True)
        return
    if args.profile_only == "gemm":
        for M, N, K in GEMM_SHAPES:
            time_gemm(ofl, M, N, K, reps=max(1, args.steps))
        log("profile run done")
        return
    if args.profile_only == "copy":
        # Copy kernel of known size: calibrates the HBM byte counters.
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(1, args.steps)):
            ofl.ofl_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, None)
        torch.cuda.synchronize()
        log(f"copied {nbytes} bytes {max(1, args.steps)} times")
        return
    I, J, K = SHAPE
    log("generating 257x257x513 inputs")
    arrays = synth.make_problem(I, J, K)

    if args.profile_only:
        it = args.profile_iters
        if args.profile_only == "headline":
            run_single(ofl, arrays, ofl.OFL_COEF_F32, args.steps, args.warmup, profile=False, iters=it)
        elif args.profile_only == "bf16":
            run_single(ofl, arrays, ofl.OFL_COEF_BF16_OFFSET, args.steps, args.warmup, profile=False, iters=it)
        elif args.profile_only == "batch":
            run_batch(ofl, synth.make_batch(args.batch_grids), ofl.OFL_COEF_F32, args.steps, args.warmup, False,
                      iters=it, row_align=args.batch_row_align)
        else:
            raise SystemExit(f"unknown --profile-only {args.profile_only}")
        log("profile run done")
        return

    log("FP32 headline")
    head = run_single(ofl, arrays, ofl.OFL_COEF_F32, args.steps, args.warmup)
    sweep_us = head["nest_ms_avg"][0] * 1e3
    lup_launch = interior(I, J, K)
    achieved = SWEEP_BYTES["f32"] * lup_launch / (sweep_us * 1e-6) / 1e9
    traffic = measured_traffic(head["tile"])
    roofline = {
        "bound": "hbm",
        "kernel": "sweep_kernel (nest S, FP32 coefficients)",
        "achieved": round(achieved, 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4),
        "traffic": traffic,
        "counter_gbs": round(traffic / (sweep_us * 1e-6) / 1e9, 1) if traffic else None,
        "counter_frac": round(traffic / (sweep_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4) if traffic else None,
        "avg_launch_us": round(sweep_us, 2),
        "timed_launches": head["nest_launches"][0],
        "algorithmic_bytes_per_launch": SWEEP_BYTES["f32"] * lup_launch,
        "nest_avg_us": {"sweep": round(sweep_us, 2), "residual": round(head["nest_ms_avg"][1] * 1e3, 2),
                        "copyback": round(head["nest_ms_avg"][2] * 1e3, 2),
                        "note": "sweep: HIP events around every sweep launch of the timed steps; residual and "
                                "copy-back: one more profiled step after them"},
    }
    out = {
        "metric": METRIC,
        "value": round(head["glups"], 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "step_ms_median": round(head["step_ms_median"], 3),
        "step_ms_min": round(head["step_ms_min"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded SplitMix64 fields)",
        "config": {
            "workload": "19-point variable-coefficient Jacobi, 257x257x513 FP32, 100 iterations per step "
                        "(sweep + residual + copy-back), every nest on the GPU, transfers hoisted, inputs resident",
            "grid_IJK": list(SHAPE),
            "iterations_per_step": ITERS,
            "omega": float(OMEGA),
            "tile": head["tile"],
        },
        "hbm_gbs_iteration": round(head["glups"] * ITER_BYTES["f32"], 1),
        "roofline": roofline,
    }
    log("streaming ceilings: the sweep's pattern without the stencil, and a 1:1 copy")
    ceil = pattern_ceilings(ofl)
    out["sweep_pattern_ceiling"] = ceil
    out["copy_1to1"] = copy_rate(ofl)
    log("headline with its host transfers (end to end)")
    out["end_to_end"] = end_to_end(ofl, arrays)
    roofline["pattern_ceiling_gbs"] = ceil["f32"]["gbs"]
    roofline["frac_of_pattern_ceiling"] = round(achieved / ceil["f32"]["gbs"], 4)
    if not args.skip_variants:
        log("bf16-offset variant")
        bf = run_single(ofl, arrays, ofl.OFL_COEF_BF16_OFFSET, args.steps, args.warmup)
        bf_sweep_us = bf["nest_ms_avg"][0] * 1e3
        out["variants"] = {
            "bf16_offset": {
                "glups": round(bf["glups"], 3),
                "ms_per_step": round(bf["ms_per_step"], 3),
                "hbm_gbs_iteration": round(bf["glups"] * ITER_BYTES["bf16"], 1),
                "sweep_avg_us": round(bf_sweep_us, 2),
                "sweep_achieved_gbs": round(SWEEP_BYTES["bf16"] * lup_launch / (bf_sweep_us * 1e-6) / 1e9, 1),
                "speedup_vs_f32": round(bf["glups"] / head["glups"], 3),
                "tile": bf["tile"],
            }
        }
        bf_gbs = out["variants"]["bf16_offset"]["sweep_achieved_gbs"]
        out["variants"]["bf16_offset"]["sweep_frac_of_hbm_peak"] = round(bf_gbs / PEAK_HBM_GBS, 4)
        out["variants"]["bf16_offset"]["sweep_frac_of_pattern_ceiling"] = round(bf_gbs / ceil["bf16"]["gbs"], 4)
        if args.tune:
            for name, fmt in (("ga_tuned_f32", ofl.OFL_COEF_F32), ("ga_tuned_bf16_offset", ofl.OFL_COEF_BF16_OFFSET)):
                best, info = tune_headline(ofl, arrays, fmt)
                tr = run_single(ofl, arrays, fmt, args.steps, args.warmup, tile=best)
                info.update(glups=round(tr["glups"], 3), ms_per_step=round(tr["ms_per_step"], 3),
                            sweep_avg_us=round(tr["nest_ms_avg"][0] * 1e3, 2))
                out["variants"][name] = info
        fuse = ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP
        for name, fmt, ib in (("fused_f32", ofl.OFL_COEF_F32, 56), ("fused_bf16_offset", ofl.OFL_COEF_BF16_OFFSET, 32)):
            log(f"{name} variant (sweep with the residual folded in, copy-back as a buffer exchange)")
            fr = run_single(ofl, arrays, fmt, args.steps, args.warmup, fusion=fuse)
            out["variants"][name] = {
                "glups": round(fr["glups"], 3),
                "ms_per_step": round(fr["ms_per_step"], 3),
                "hbm_gbs_iteration": round(fr["glups"] * ib, 1),
                "sweep_avg_us": round(fr["nest_ms_avg"][0] * 1e3, 2),
                "speedup_vs_f32": round(fr["glups"] / head["glups"], 3),
            }
    if not args.skip_cpu_baseline:
        # the oracle on a bounded sample (the first oracle_iters iterations),
        # and every single-grid form's error against it over the same iterations
        arrays64 = widened(arrays)
        out["cpu_baseline"], (p_ref, g_ref) = cpu_baseline(arrays64, args.oracle_iters)
        del arrays64
        fuse = ofl.OFL_FUSE_RESIDUAL | ofl.OFL_FUSE_COPYBACK_SWAP
        forms = [(None, ofl.OFL_COEF_F32, 0)]
        if not args.skip_variants:
            forms += [("bf16_offset", ofl.OFL_COEF_BF16_OFFSET, 0), ("fused_f32", ofl.OFL_COEF_F32, fuse),
                      ("fused_bf16_offset", ofl.OFL_COEF_BF16_OFFSET, fuse)]
        for name, fmt, fusion in forms:
            log(f"error against the oracle: {name or 'FP32 headline'}, {args.oracle_iters} iterations")
            e = single_error(ofl, arrays, fmt, fusion, args.oracle_iters, p_ref, g_ref)
            if name is None:
                out["oracle_error"] = e
            else:
                out["variants"][name]["oracle_error"] = e
        del p_ref
    if not args.skip_variants and not args.skip_batch:
        log(f"generating {args.batch_grids} uneven grids")
        probs = synth.make_batch(args.batch_grids)
        check = None if args.skip_cpu_baseline else (args.oracle_iters, batch_check_refs(probs, args.oracle_iters))
        for name, fmt in (("batched_f32", ofl.OFL_COEF_F32), ("batched_bf16_offset", ofl.OFL_COEF_BF16_OFFSET)):
            log(f"{name} variant")
            out["variants"][name] = run_batch(ofl, probs, fmt, max(1, args.steps // 2), 1, args.tune_batch,
                                              row_align=args.batch_row_align, check=check)
        del probs
    if not args.skip_variants:
        # the function-block routine (a matrix product on the matrix cores);
        # its parity against the FP64 oracle is a GPU test, not part of this line
        out["variants"]["gemm_f32"] = {"note": "ofl_gemm_f32, FP32 products and accumulation on the matrix cores; "
                                               "parity: tests/test_gpu_gemm.py against the FP64 oracle_gemm",
                                       "shapes": []}
        for M, N, K in GEMM_SHAPES[:2]:
            sec = sorted(time_gemm(ofl, M, N, K) for _ in range(3))[1]  # median of three timings
            tflops = 2.0 * M * N * K / sec / 1e12
            out["variants"]["gemm_f32"]["shapes"].append(
                {"M": M, "N": N, "K": K, "us": round(sec * 1e6, 1), "tflops": round(tflops, 2),
                 "frac_of_fp32_mfma_peak": round(tflops / PEAK_FP32_MFMA_TFLOPS, 4)})
            log(f"gemm {M}x{N}x{K}: {tflops:.1f} TFLOP/s")
    if not args.skip_cpu_baseline:
        out["cpu_program"] = cpu_program(ofl, arrays, args.oracle_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
