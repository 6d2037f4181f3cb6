"""Python binding of libofl.so, the MI355X (gfx950) offloaded-Jacobi library.

Argument marshalling only: every nest of the Jacobi program runs in the
library (HIP kernels for gene bit 1, the library's CPU loops for gene bit 0).
The functions carry the names of the C entry points declared in
include/ofl.h. PyTorch, when a GPU is present, supplies device memory (the
grid's arena) and the stream; it computes nothing.

If libofl.so has not been built the first call raises OflError: there is no
other implementation to fall back to.
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libofl.so")

OFL_OK, OFL_EINVAL, OFL_ENOMEM, OFL_EDEVICE, OFL_ESTATE, OFL_ENOTSUP = 0, -1, -2, -3, -4, -5
OFL_NEST_SWEEP, OFL_NEST_RESIDUAL, OFL_NEST_COPYBACK = 1, 2, 4
OFL_MASK_ALL_CPU, OFL_MASK_ALL_GPU = 0, 7
OFL_XFER_PER_ITER, OFL_XFER_HOISTED = 0, 1
OFL_COEF_F32, OFL_COEF_BF16, OFL_COEF_BF16_OFFSET = 0, 1, 2
OFL_SUM_F64, OFL_SUM_KAHAN_F32 = 0, 1
OFL_TILE_NT_LOADS, OFL_TILE_NT_STORES, OFL_TILE_PREFETCH, OFL_TILE_MARCH_J, OFL_TILE_XCD_REMAP = 1, 2, 4, 8, 16
ARRAY_NAMES = ("a0", "a1", "a2", "a3", "b0", "b1", "b2", "c0", "c1", "c2", "bnd", "wrk1", "p", "wrk2")
COEF_NAMES = ARRAY_NAMES[:12]
OFL_ARR_P, OFL_ARR_WRK2 = 12, 13
OFL_FUSE_RESIDUAL, OFL_FUSE_COPYBACK_SWAP = 1, 2
OFL_LEVEL_K, OFL_LEVEL_J, OFL_LEVEL_I = 0, 1, 2
OFL_NLOOPS = 10

_FP = ctypes.POINTER(ctypes.c_float)


class OflGridDesc(ctypes.Structure):
    _fields_ = [
        ("I", ctypes.c_int), ("J", ctypes.c_int), ("K", ctypes.c_int),
        ("coef_format", ctypes.c_int), ("sum_mode", ctypes.c_int),
        ("p", _FP), ("wrk2", _FP), ("coef", _FP * 12),
        ("stream", ctypes.c_void_p), ("dev_arena", ctypes.c_void_p),
        ("dev_arena_bytes", ctypes.c_size_t), ("device", ctypes.c_int), ("row_align", ctypes.c_int),
    ]


class OflTile(ctypes.Structure):
    _fields_ = [("vec", ctypes.c_int), ("rows", ctypes.c_int), ("kchunk", ctypes.c_int),
                ("flags", ctypes.c_int), ("occupancy", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class OflStats(ctypes.Structure):
    _fields_ = [
        ("h2d_count", ctypes.c_uint64), ("d2h_count", ctypes.c_uint64),
        ("h2d_bytes", ctypes.c_uint64), ("d2h_bytes", ctypes.c_uint64),
        ("gpu_nests", ctypes.c_uint64 * 3), ("cpu_nests", ctypes.c_uint64 * 3),
        ("kernel_ms", ctypes.c_double * 3), ("timed_nests", ctypes.c_uint64 * 3),
        ("gpu_regions", ctypes.c_uint64 * 3),
    ]


class OflLoopInfo(ctypes.Structure):
    _fields_ = [("nest", ctypes.c_int), ("level", ctypes.c_int), ("extent", ctypes.c_int),
                ("parallel", ctypes.c_int)]

    def as_tuple(self):
        return (self.nest, self.level, self.extent, self.parallel)


class OflXfer(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int), ("nest", ctypes.c_int), ("when", ctypes.c_int),
                ("array", ctypes.c_int), ("dir", ctypes.c_int)]

    def as_tuple(self):
        return (self.iter, self.nest, self.when, self.array, self.dir)


class OflNestVars(ctypes.Structure):
    _fields_ = [("reads", ctypes.c_uint32), ("writes", ctypes.c_uint32), ("partial", ctypes.c_uint32)]

    def as_tuple(self):
        return (self.reads, self.writes, self.partial)


class OflGaParams(ctypes.Structure):
    _fields_ = [("population", ctypes.c_int), ("generations", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("crossover", ctypes.c_double), ("mutation", ctypes.c_double), ("elite", ctypes.c_int),
                ("probe_iters", ctypes.c_int), ("repeats", ctypes.c_int), ("tolerance", ctypes.c_double)]


class OflTuneResult(ctypes.Structure):
    _fields_ = [("best", OflTile), ("best_ms", ctypes.c_double), ("evaluated", ctypes.c_int),
                ("rejected", ctypes.c_int), ("from_cache", ctypes.c_int)]


class OflGaResult(ctypes.Structure):
    _fields_ = [("best_gene", ctypes.c_uint32), ("best_time", ctypes.c_double), ("evaluated", ctypes.c_int),
                ("rejected", ctypes.c_int)]


class OflOffloadResult(ctypes.Structure):
    _fields_ = [("mask", ctypes.c_uint), ("xfer_mode", ctypes.c_int), ("best_ms", ctypes.c_double),
                ("cpu_ms", ctypes.c_double), ("evaluated", ctypes.c_int), ("rejected", ctypes.c_int)]


class OflLoopSearchResult(ctypes.Structure):
    _fields_ = [("gene", ctypes.c_uint32), ("mask", ctypes.c_uint), ("level", ctypes.c_int * 3),
                ("gene_bits", ctypes.c_int), ("best_ms", ctypes.c_double), ("cpu_ms", ctypes.c_double),
                ("evaluated", ctypes.c_int), ("patterns", ctypes.c_int), ("rejected", ctypes.c_int),
                ("timed_out", ctypes.c_int)]


OFL_GENE_EVAL = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_uint32, ctypes.c_void_p)


class OflError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"ofl error {code}: {message}")
        self.code = code
        self.message = message


_lib_handle = None

_SIGS = {
    "ofl_grid_device_bytes": ([ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "ofl_grid_create": ([ctypes.POINTER(OflGridDesc), ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "ofl_grid_destroy": ([ctypes.c_void_p], None),
    "ofl_set_offload_mask": ([ctypes.c_void_p, ctypes.c_uint, ctypes.c_int], ctypes.c_int),
    "ofl_loop_table": ([ctypes.c_void_p, ctypes.POINTER(OflLoopInfo)], ctypes.c_int),
    "ofl_set_loop_gene": ([ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int], ctypes.c_int),
    "ofl_set_regions": ([ctypes.c_void_p, ctypes.c_uint, ctypes.POINTER(ctypes.c_int), ctypes.c_int], ctypes.c_int),
    "ofl_get_regions": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint), ctypes.POINTER(ctypes.c_int),
                         ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "ofl_jacobi_run": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "ofl_jacobi_run_static": (
        [ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.POINTER(ctypes.c_double)],
        ctypes.c_int,
    ),
    "ofl_residual": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "ofl_data_enter": ([ctypes.c_void_p], ctypes.c_int),
    "ofl_update_host": ([ctypes.c_void_p], ctypes.c_int),
    "ofl_data_exit": ([ctypes.c_void_p], ctypes.c_int),
    "ofl_grid_coef_bias": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "ofl_set_fusion": ([ctypes.c_void_p, ctypes.c_uint], ctypes.c_int),
    "ofl_set_tile": ([ctypes.c_void_p, ctypes.POINTER(OflTile)], ctypes.c_int),
    "ofl_get_tile": ([ctypes.c_void_p, ctypes.POINTER(OflTile)], ctypes.c_int),
    "ofl_set_profiling": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "ofl_set_profiled_nests": ([ctypes.c_void_p, ctypes.c_uint], ctypes.c_int),
    "ofl_get_stats": ([ctypes.c_void_p, ctypes.POINTER(OflStats)], ctypes.c_int),
    "ofl_reset_stats": ([ctypes.c_void_p], ctypes.c_int),
    "ofl_plan": ([ctypes.c_uint, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint8),
                  ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(OflXfer), ctypes.c_int,
                  ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "ofl_plan_nests": ([ctypes.POINTER(OflNestVars), ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint,
                        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint8),
                        ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(OflXfer), ctypes.c_int,
                        ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "ofl_program_vars": ([ctypes.POINTER(OflNestVars), ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
    "ofl_batch_create": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(OflTile),
                          ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "ofl_batch_destroy": ([ctypes.c_void_p], None),
    "ofl_batch_set_tile": ([ctypes.c_void_p, ctypes.POINTER(OflTile)], ctypes.c_int),
    "ofl_batch_get_tile": ([ctypes.c_void_p, ctypes.POINTER(OflTile)], ctypes.c_int),
    "ofl_batch_set_fusion": ([ctypes.c_void_p, ctypes.c_uint], ctypes.c_int),
    "ofl_batch_run": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "ofl_set_tune_cache": ([ctypes.c_char_p], ctypes.c_int),
    "ofl_grid_tune": ([ctypes.c_void_p, ctypes.POINTER(OflGaParams), ctypes.POINTER(OflTuneResult)], ctypes.c_int),
    "ofl_batch_tune": ([ctypes.c_void_p, ctypes.POINTER(OflGaParams), ctypes.POINTER(OflTuneResult)], ctypes.c_int),
    "ofl_ga_search": ([ctypes.c_int, ctypes.POINTER(OflGaParams), ctypes.c_uint32, OFL_GENE_EVAL, ctypes.c_void_p,
                       ctypes.POINTER(OflGaResult)], ctypes.c_int),
    "ofl_grid_search_offload": ([ctypes.c_void_p, ctypes.POINTER(OflGaParams), ctypes.c_int, ctypes.c_float,
                                 ctypes.POINTER(OflOffloadResult)], ctypes.c_int),
    "ofl_grid_search_loops": ([ctypes.c_void_p, ctypes.POINTER(OflGaParams), ctypes.c_int, ctypes.c_float,
                               ctypes.c_int, ctypes.c_double, ctypes.POINTER(OflLoopSearchResult)], ctypes.c_int),
    "ofl_gemm_f32": ([ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "ofl_device_copy": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "ofl_device_stream": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                           ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "ofl_last_error": ([], ctypes.c_char_p),
    "ofl_version": ([], ctypes.c_char_p),
}


def lib():
    """The loaded libofl.so (raises OflError if it has not been built)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise OflError(OFL_EDEVICE, f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        h = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(h, name)
            f.argtypes = args
            f.restype = res
        _lib_handle = h
    return _lib_handle


def ofl_last_error() -> str:
    return lib().ofl_last_error().decode()


def ofl_version() -> str:
    return lib().ofl_version().decode()


def _check(rc: int):
    if rc != OFL_OK:
        raise OflError(rc, ofl_last_error())


def ofl_grid_device_bytes(I: int, J: int, K: int, coef_format: int = OFL_COEF_F32, row_align: int = 0) -> int:
    out = ctypes.c_size_t()
    _check(lib().ofl_grid_device_bytes(I, J, K, coef_format, row_align, ctypes.byref(out)))
    return out.value


def ofl_grid_create(desc: OflGridDesc) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().ofl_grid_create(ctypes.byref(desc), ctypes.byref(h)))
    return h


def ofl_grid_destroy(g) -> None:
    lib().ofl_grid_destroy(g)


def ofl_set_offload_mask(g, mask: int, xfer_mode: int = OFL_XFER_HOISTED) -> None:
    _check(lib().ofl_set_offload_mask(g, mask, xfer_mode))


def ofl_loop_table(g) -> list:
    """The program's loop statements: (nest, level, extent, parallel) per loop, in program order."""
    t = (OflLoopInfo * OFL_NLOOPS)()
    _check(lib().ofl_loop_table(g, t))
    return [x.as_tuple() for x in t]


def ofl_set_loop_gene(g, gene: int, xfer_mode: int = OFL_XFER_HOISTED) -> None:
    _check(lib().ofl_set_loop_gene(g, gene, xfer_mode))


def ofl_set_regions(g, mask: int, level: Sequence[int], xfer_mode: int = OFL_XFER_HOISTED) -> None:
    lv = (ctypes.c_int * 3)(*level)
    _check(lib().ofl_set_regions(g, mask, lv, xfer_mode))


def ofl_get_regions(g):
    """(mask, [level of S, R, C], xfer_mode)."""
    mask, mode = ctypes.c_uint(), ctypes.c_int()
    lv = (ctypes.c_int * 3)()
    _check(lib().ofl_get_regions(g, ctypes.byref(mask), lv, ctypes.byref(mode)))
    return mask.value, list(lv), mode.value


def ofl_jacobi_run(g, iters: int, omega: float) -> float:
    gosa = ctypes.c_double()
    _check(lib().ofl_jacobi_run(g, iters, omega, ctypes.byref(gosa)))
    return gosa.value


def ofl_jacobi_run_static(g, iters: int, omega: float) -> float:
    gosa = ctypes.c_double()
    _check(lib().ofl_jacobi_run_static(g, iters, omega, ctypes.byref(gosa)))
    return gosa.value


def ofl_residual(g) -> float:
    gosa = ctypes.c_double()
    _check(lib().ofl_residual(g, ctypes.byref(gosa)))
    return gosa.value


def ofl_data_enter(g) -> None:
    _check(lib().ofl_data_enter(g))


def ofl_update_host(g) -> None:
    _check(lib().ofl_update_host(g))


def ofl_data_exit(g) -> None:
    _check(lib().ofl_data_exit(g))


def ofl_grid_coef_bias(g) -> np.ndarray:
    out = (ctypes.c_float * 12)()
    _check(lib().ofl_grid_coef_bias(g, out))
    return np.array(list(out), dtype=np.float32)


def ofl_set_fusion(g, flags: int) -> None:
    _check(lib().ofl_set_fusion(g, flags))


def ofl_set_tile(g, tile: OflTile) -> None:
    _check(lib().ofl_set_tile(g, ctypes.byref(tile)))


def ofl_get_tile(g) -> OflTile:
    t = OflTile()
    _check(lib().ofl_get_tile(g, ctypes.byref(t)))
    return t


def ofl_set_profiling(g, on: bool) -> None:
    _check(lib().ofl_set_profiling(g, 1 if on else 0))


def ofl_set_profiled_nests(g, nests: int) -> None:
    _check(lib().ofl_set_profiled_nests(g, nests))


def ofl_get_stats(g) -> OflStats:
    s = OflStats()
    _check(lib().ofl_get_stats(g, ctypes.byref(s)))
    return s


def ofl_reset_stats(g) -> None:
    _check(lib().ofl_reset_stats(g))


def ofl_plan(mask: int, xfer_mode: int, iters: int, sync_host_at_end: bool = True,
             host_valid: Optional[Sequence[int]] = None, dev_valid: Optional[Sequence[int]] = None):
    """Returns (list of (iter, nest, when, array, dir), host_valid, dev_valid)."""
    hv = (ctypes.c_uint8 * 14)(*(host_valid if host_valid is not None else [1] * 14))
    dv = (ctypes.c_uint8 * 14)(*(dev_valid if dev_valid is not None else [0] * 14))
    count = ctypes.c_int()
    rc = lib().ofl_plan(mask, xfer_mode, iters, 1 if sync_host_at_end else 0, hv, dv, None, 0, ctypes.byref(count))
    if rc not in (OFL_OK, OFL_ENOMEM):
        _check(rc)
    hv = (ctypes.c_uint8 * 14)(*(host_valid if host_valid is not None else [1] * 14))
    dv = (ctypes.c_uint8 * 14)(*(dev_valid if dev_valid is not None else [0] * 14))
    buf = (OflXfer * max(1, count.value))()
    _check(lib().ofl_plan(mask, xfer_mode, iters, 1 if sync_host_at_end else 0, hv, dv, buf, count.value,
                          ctypes.byref(count)))
    return [buf[t].as_tuple() for t in range(count.value)], list(hv), list(dv)


def ofl_plan_nests(nests: Sequence[Sequence[int]], narrays: int, live_after: int, mask: int, xfer_mode: int,
                   iters: int, sync_host_at_end: bool = True, host_valid: Optional[Sequence[int]] = None,
                   dev_valid: Optional[Sequence[int]] = None):
    """The planner over any program: nests = [(reads, writes, partial) bit sets], one per nest.
    Returns (list of (iter, nest, when, array, dir), host_valid, dev_valid)."""
    nv = (OflNestVars * len(nests))(*[OflNestVars(*n) for n in nests])

    def state():
        hv = (ctypes.c_uint8 * narrays)(*(host_valid if host_valid is not None else [1] * narrays))
        dv = (ctypes.c_uint8 * narrays)(*(dev_valid if dev_valid is not None else [0] * narrays))
        return hv, dv

    hv, dv = state()
    count = ctypes.c_int()
    args = (nv, len(nests), narrays, live_after, mask, xfer_mode, iters, 1 if sync_host_at_end else 0)
    rc = lib().ofl_plan_nests(*args, hv, dv, None, 0, ctypes.byref(count))
    if rc not in (OFL_OK, OFL_ENOMEM):
        _check(rc)
    hv, dv = state()
    buf = (OflXfer * max(1, count.value))()
    _check(lib().ofl_plan_nests(*args, hv, dv, buf, count.value, ctypes.byref(count)))
    return [buf[t].as_tuple() for t in range(count.value)], list(hv), list(dv)


def ofl_program_vars():
    """The library's program as [(reads, writes, partial)] for S, R, C, and the arrays read after the loop."""
    nv = (OflNestVars * 3)()
    live = ctypes.c_uint32()
    _check(lib().ofl_program_vars(nv, ctypes.byref(live)))
    return [x.as_tuple() for x in nv], live.value


def ofl_batch_create(grids: Sequence, tile: Optional[OflTile] = None) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * len(grids))(*[g.value if isinstance(g, ctypes.c_void_p) else g for g in grids])
    h = ctypes.c_void_p()
    _check(lib().ofl_batch_create(arr, len(grids), ctypes.byref(tile) if tile is not None else None,
                                  ctypes.byref(h)))
    return h


def ofl_batch_destroy(b) -> None:
    lib().ofl_batch_destroy(b)


def ofl_batch_set_tile(b, tile: OflTile) -> None:
    _check(lib().ofl_batch_set_tile(b, ctypes.byref(tile)))


def ofl_batch_get_tile(b) -> OflTile:
    t = OflTile()
    _check(lib().ofl_batch_get_tile(b, ctypes.byref(t)))
    return t


def ofl_batch_set_fusion(b, flags: int) -> None:
    _check(lib().ofl_batch_set_fusion(b, flags))


def ofl_batch_run(b, iters: int, omega: float, n_grids: int):
    out = (ctypes.c_double * n_grids)()
    _check(lib().ofl_batch_run(b, iters, omega, out))
    return list(out)


def ga_params(population=16, generations=12, seed=2011036020, crossover=0.9, mutation=0.05, elite=1,
              probe_iters=5, repeats=3, tolerance=1e-5) -> OflGaParams:
    return OflGaParams(population, generations, seed, crossover, mutation, elite, probe_iters, repeats, tolerance)


def ofl_set_tune_cache(path: Optional[str]) -> None:
    _check(lib().ofl_set_tune_cache(os.fsencode(path) if path is not None else None))


def ofl_grid_tune(g, ga: Optional[OflGaParams] = None) -> OflTuneResult:
    r = OflTuneResult()
    _check(lib().ofl_grid_tune(g, ctypes.byref(ga) if ga is not None else None, ctypes.byref(r)))
    return r


def ofl_batch_tune(b, ga: Optional[OflGaParams] = None) -> OflTuneResult:
    r = OflTuneResult()
    _check(lib().ofl_batch_tune(b, ctypes.byref(ga) if ga is not None else None, ctypes.byref(r)))
    return r


def ofl_ga_search(bits: int, evaluate, ga: Optional[OflGaParams] = None, seed_gene: int = 0) -> OflGaResult:
    """evaluate(gene) -> time (> 0), inf (wrong result) or nan (not buildable)."""
    cb = OFL_GENE_EVAL(lambda gene, ctx: float(evaluate(int(gene))))
    r = OflGaResult()
    _check(lib().ofl_ga_search(bits, ctypes.byref(ga) if ga is not None else None, seed_gene, cb, None,
                               ctypes.byref(r)))
    return r


def ofl_grid_search_loops(g, iters: int, omega: float, xfer_mode: int = OFL_XFER_HOISTED,
                          time_limit_ms: float = 0.0, ga: Optional[OflGaParams] = None) -> OflLoopSearchResult:
    r = OflLoopSearchResult()
    _check(lib().ofl_grid_search_loops(g, ctypes.byref(ga) if ga is not None else None, iters, omega, xfer_mode,
                                       time_limit_ms, ctypes.byref(r)))
    return r


def ofl_grid_search_offload(g, iters: int, omega: float, ga: Optional[OflGaParams] = None) -> OflOffloadResult:
    r = OflOffloadResult()
    _check(lib().ofl_grid_search_offload(g, ctypes.byref(ga) if ga is not None else None, iters, omega,
                                         ctypes.byref(r)))
    return r


def ofl_gemm_f32(M: int, N: int, K: int, a_ptr: int, lda: int, b_ptr: int, ldb: int, c_ptr: int, ldc: int,
                 stream: Optional[int] = None) -> None:
    """C = A B on device pointers (row-major FP32, strides in elements), queued on stream."""
    _check(lib().ofl_gemm_f32(M, N, K, a_ptr, lda, b_ptr, ldb, c_ptr, ldc, stream))


def ofl_device_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream: Optional[int] = None) -> None:
    _check(lib().ofl_device_copy(dst_ptr, src_ptr, nbytes, stream))


def ofl_device_stream(src32_ptrs: Sequence[int], src16_ptrs: Sequence[int], dst_ptr: int, n: int,
                      stream: Optional[int] = None) -> None:
    """The sweep's streaming pattern on device arrays: dst = sum of the FP32 and bfloat16 sources."""
    s32 = (ctypes.c_void_p * max(1, len(src32_ptrs)))(*src32_ptrs)
    s16 = (ctypes.c_void_p * max(1, len(src16_ptrs)))(*src16_ptrs)
    _check(lib().ofl_device_stream(s32, len(src32_ptrs), s16, len(src16_ptrs), dst_ptr, n, stream))


def tile(vec=4, rows=4, kchunk=32, flags=0, occupancy=0) -> OflTile:
    return OflTile(vec, rows, kchunk, flags, occupancy)


class Grid:
    """Owns the host arrays of one grid and its handle.

    ``arrays`` maps the names in ARRAY_NAMES (wrk2 optional) to (K, J, I)
    arrays; they are copied into contiguous FP32 host buffers (pinned by
    PyTorch when ``pinned``), which the library borrows for the handle's life.
    ``torch_memory``: take the grid's device block from PyTorch's allocator and
    launch on a PyTorch stream (needs a GPU); otherwise the library allocates.
    ``row_align``: elements each device row is padded to (0: 128-byte rows).
    """

    def __init__(self, arrays: Dict[str, np.ndarray], coef_format: int = OFL_COEF_F32,
                 sum_mode: int = OFL_SUM_F64, torch_memory: bool = False, pinned: bool = False,
                 row_align: int = 0):
        p = np.asarray(arrays["p"])
        if p.ndim != 3:
            raise ValueError("arrays must be 3-D (K, J, I)")
        self.shape = p.shape
        K, J, I = self.shape
        self._torch_keep = []
        self.host = {}
        for name in ARRAY_NAMES:
            src = arrays.get(name)
            if src is None:
                if name != "wrk2":
                    raise KeyError(name)
                src = np.zeros(self.shape, np.float32)
            self.host[name] = self._host_buffer(np.asarray(src, dtype=np.float32), pinned)
        desc = OflGridDesc()
        desc.I, desc.J, desc.K = I, J, K
        desc.coef_format = coef_format
        desc.sum_mode = sum_mode
        desc.p = self.host["p"].ctypes.data_as(_FP)
        desc.wrk2 = self.host["wrk2"].ctypes.data_as(_FP)
        for n, name in enumerate(COEF_NAMES):
            desc.coef[n] = self.host[name].ctypes.data_as(_FP)
        desc.device = -1
        desc.row_align = row_align
        self.stream = None
        if torch_memory:
            import torch

            nbytes = ofl_grid_device_bytes(I, J, K, coef_format, row_align)
            arena = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            self.stream = torch.cuda.Stream()
            self._torch_keep += [arena, self.stream]
            desc.dev_arena = arena.data_ptr()
            desc.dev_arena_bytes = nbytes
            desc.stream = self.stream.cuda_stream
            desc.device = torch.cuda.current_device()
        self.desc = desc
        self.handle = ofl_grid_create(desc)

    def _host_buffer(self, src: np.ndarray, pinned: bool) -> np.ndarray:
        if pinned:
            import torch

            t = torch.empty(src.shape, dtype=torch.float32, pin_memory=True)
            self._torch_keep.append(t)
            buf = t.numpy()
            buf[...] = src
            return buf
        return np.ascontiguousarray(src, dtype=np.float32).copy()

    @property
    def p(self) -> np.ndarray:
        return self.host["p"]

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            ofl_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
