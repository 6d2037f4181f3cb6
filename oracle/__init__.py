"""FP64 CPU oracle of the offloaded Jacobi program and of the matrix-product
function block (ctypes front of oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package; the product library never does. It shares
no code with the GPU path. The arithmetic lives in oracle.c; this file only
converts numpy arrays to the pointers the C functions take.
"""

from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np

from . import build as _build

COEF_NAMES = ("a0", "a1", "a2", "a3", "b0", "b1", "b2", "c0", "c1", "c2", "bnd", "wrk1")

_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_FP = ctypes.POINTER(ctypes.c_float)
_COEFS = _DP * 12


_lib_path = None


def _load():
    global _lib
    if _lib is None:
        path = _lib_path or _build.LIB
        if _lib_path is None and not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        lib.oracle_sweep.argtypes = [ctypes.c_int] * 3 + [_COEFS, _DP, ctypes.c_double, _DP, _DP]
        lib.oracle_residual.argtypes = [ctypes.c_int] * 3 + [_COEFS, _DP, _DP]
        lib.oracle_jacobi.argtypes = [ctypes.c_int] * 3 + [_COEFS, _DP, ctypes.c_double, ctypes.c_int, _DP]
        for f in (lib.oracle_sweep, lib.oracle_residual, lib.oracle_jacobi):
            f.restype = ctypes.c_int
        lib.oracle_bf16_rne.argtypes = [ctypes.c_float]
        lib.oracle_bf16_rne.restype = ctypes.c_float
        lib.oracle_bf16_rne_array.argtypes = [_FP, _FP, ctypes.c_size_t]
        lib.oracle_bf16_rne_array.restype = None
        lib.oracle_gemm.argtypes = [ctypes.c_int] * 3 + [_DP, ctypes.c_int, _DP, ctypes.c_int, _DP, ctypes.c_int]
        lib.oracle_gemm.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


@contextlib.contextmanager
def use_library(path):
    """Temporarily load the oracle from another build of oracle.c (used by the
    test that plants mistakes in copies of the oracle to show the pins fail)."""
    global _lib, _lib_path
    saved = (_lib, _lib_path)
    _lib, _lib_path = None, path
    try:
        yield
    finally:
        _lib, _lib_path = saved


def threads():
    """Host threads the loaded oracle build uses (1, or the OpenMP thread count
    when loaded from the all-cores build through use_library)."""
    return int(_load().oracle_threads())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_DP)


def _coefs(arrays):
    held = [_f64(arrays[n]) for n in COEF_NAMES]
    shape = held[0].shape
    for h in held:
        if h.shape != shape:
            raise ValueError("coefficient arrays differ in shape")
    return held, _COEFS(*[_ptr(h) for h in held]), shape


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} rejected its arguments (rc={rc})")


def jacobi(arrays, iters, omega):
    """Run ``iters`` iterations from ``arrays['p']``; returns (p_final FP64 (K,J,I), gosa)."""
    held, co, shape = _coefs(arrays)
    K, J, I = shape
    p = _f64(arrays["p"]).copy()
    if p.shape != shape:
        raise ValueError("p has the wrong shape")
    gosa = ctypes.c_double()
    _check(_load().oracle_jacobi(I, J, K, co, _ptr(p), float(omega), int(iters), ctypes.byref(gosa)), "oracle_jacobi")
    return p, gosa.value


def sweep(arrays, omega, wrk2=None):
    """One sweep from ``arrays['p']``: returns (wrk2 FP64, sum of ss^2)."""
    held, co, shape = _coefs(arrays)
    K, J, I = shape
    p = _f64(arrays["p"])
    w = np.zeros(shape, np.float64) if wrk2 is None else _f64(wrk2).copy()
    gosa = ctypes.c_double()
    _check(_load().oracle_sweep(I, J, K, co, _ptr(p), float(omega), _ptr(w), ctypes.byref(gosa)), "oracle_sweep")
    return w, gosa.value


def residual(arrays):
    """Sum over the interior of ss(p)^2 for the current ``arrays['p']``."""
    held, co, shape = _coefs(arrays)
    K, J, I = shape
    p = _f64(arrays["p"])
    gosa = ctypes.c_double()
    _check(_load().oracle_residual(I, J, K, co, _ptr(p), ctypes.byref(gosa)), "oracle_residual")
    return gosa.value


def bf16_rne(x):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as FP32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty_like(x)
    _load().oracle_bf16_rne_array(x.ctypes.data_as(_FP), out.ctypes.data_as(_FP), x.size)
    return out


def offset_bf16_decode(x, bias):
    """Values a reader of offset-bf16 storage sees: fl32(bias + bf16(fl32(x - bias)))."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = np.float32(bias)
    q = bf16_rne((x - b).astype(np.float32))
    return (b + q).astype(np.float32)


def offset_bias(x):
    """Bias of the offset-bf16 encoding: 0 if every value is bfloat16-exact,
    else the FP32 mid-range fl32((min + max) / 2) computed in FP64."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    if np.array_equal(bf16_rne(x), x):
        return np.float32(0.0)
    lo = float(x.min())
    hi = float(x.max())
    return np.float32(0.5 * (lo + hi))


def gemm(a, b):
    """C = A B in FP64 of the given operands (widened), by oracle_gemm."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
    if a.ndim != 2 or b.ndim != 2 or a.shape[1] != b.shape[0]:
        raise ValueError("gemm needs an M x K and a K x N matrix")
    M, K = a.shape
    N = b.shape[1]
    c = np.zeros((M, N), dtype=np.float64)
    _check(_load().oracle_gemm(M, N, K, _ptr(a), max(K, 1), _ptr(b), max(N, 1), _ptr(c), max(N, 1)),
           "oracle_gemm")
    return c
