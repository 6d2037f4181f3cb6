"""Seeded synthetic inputs for the variable-coefficient 19-point Jacobi problem.

This module only draws numbers. It holds none of the solver's arithmetic, so
both the FP64 oracle (test infrastructure) and the GPU library can be fed the
same arrays without sharing any computation.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-style. The n-th output of a
SplitMix64 stream whose state starts at ``s`` is ``mix(s + n * GAMMA)``, so any
element can be drawn independently of the others:

    u(seed, field, idx) = (mix(seed + GAMMA * (field * 2**40 + idx + 1)) >> 11) * 2**-53

which is uniform on [0, 1) with 53 random bits.

Array layout: numpy shape ``(K, J, I)``, C-contiguous, so the linear index of
point ``(i, j, k)`` is ``i + I * (j + J * k)`` (i fastest).

Field distributions (all FP32, rounded to nearest even from FP64 draws):

=========  =====================================================
a0,a1,a2   1 + U(-0.05, 0.05)
a3         fl32(1 / (2 (a0 + a1 + a2)))  from the FP32 a-values
b0,b1,b2   U(-0.01, 0.01)
c0,c1,c2   1
bnd        1 on the interior, 0 on the one-cell boundary layer
wrk1       U(-0.1, 0.1)
p          U(0, 1) on every point, boundary included
wrk2       0
=========  =====================================================

Batch grid sizes: I, J = 33 + floor(u * 129) (so U{33..161}) and
K = 65 + floor(u * 257) (so U{65..321}); grid ``g`` of a batch uses the seed
``mix(base + (g + 1) * GAMMA)``.
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 2011036020
GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB

# Field identifiers of the counter-based streams.
FIELD_A0, FIELD_A1, FIELD_A2 = 0, 1, 2
FIELD_B0, FIELD_B1, FIELD_B2 = 3, 4, 5
FIELD_WRK1 = 6
FIELD_P0 = 7
FIELD_BATCH_SIZES = 8

# Order of the twelve read-only arrays, as every interface of this project uses it.
COEF_NAMES = ("a0", "a1", "a2", "a3", "b0", "b1", "b2", "c0", "c1", "c2", "bnd", "wrk1")

_MASK64 = (1 << 64) - 1


def mix64(z):
    """SplitMix64 output function on a uint64 numpy array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    return z


def mix64_int(z: int) -> int:
    """SplitMix64 output function on one Python int."""
    z &= _MASK64
    z = ((z ^ (z >> 30)) * _M1) & _MASK64
    z = ((z ^ (z >> 27)) * _M2) & _MASK64
    return z ^ (z >> 31)


def uniform(seed: int, field: int, n: int, start: int = 0, chunk: int = 1 << 22) -> np.ndarray:
    """``n`` FP64 draws on [0, 1) of stream ``field``, for indices start..start+n-1."""
    out = np.empty(n, dtype=np.float64)
    base = (seed + GAMMA * (field * (1 << 40) + start + 1)) & _MASK64
    scale = float(2.0 ** -53)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        idx = np.arange(lo, hi, dtype=np.uint64)
        with np.errstate(over="ignore"):
            state = np.uint64(base) + idx * np.uint64(GAMMA)
        out[lo:hi] = (mix64(state) >> np.uint64(11)).astype(np.float64) * scale
    return out


def grid_seed(g: int, base: int = BASE_SEED) -> int:
    """Seed of grid ``g`` inside a batch."""
    return mix64_int(base + (g + 1) * GAMMA)


def batch_sizes(n_grids: int, base: int = BASE_SEED):
    """Uneven batch shapes: list of (I, J, K) with I, J in 33..161 and K in 65..321."""
    u = uniform(base, FIELD_BATCH_SIZES, 3 * n_grids)
    sizes = []
    for g in range(n_grids):
        I = 33 + int(np.floor(u[3 * g] * 129))
        J = 33 + int(np.floor(u[3 * g + 1] * 129))
        K = 65 + int(np.floor(u[3 * g + 2] * 257))
        sizes.append((I, J, K))
    return sizes


def _sym(seed, field, n, half_width):
    u = uniform(seed, field, n)
    return (half_width * (2.0 * u - 1.0)).astype(np.float32)


def make_problem(I: int, J: int, K: int, seed: int = BASE_SEED) -> dict:
    """All fourteen FP32 arrays of one grid, shape (K, J, I).

    Returns a dict with the twelve read-only arrays named as in COEF_NAMES plus
    ``p`` (initial iterate) and ``wrk2`` (zeros).
    """
    if min(I, J, K) < 3:
        raise ValueError("every grid dimension must be >= 3")
    n = I * J * K
    shape = (K, J, I)
    arr = {}
    for name, field in (("a0", FIELD_A0), ("a1", FIELD_A1), ("a2", FIELD_A2)):
        arr[name] = (1.0 + _sym(seed, field, n, 0.05).astype(np.float64)).astype(np.float32).reshape(shape)
    asum = arr["a0"].astype(np.float64) + arr["a1"].astype(np.float64) + arr["a2"].astype(np.float64)
    arr["a3"] = (1.0 / (2.0 * asum)).astype(np.float32)
    for name, field in (("b0", FIELD_B0), ("b1", FIELD_B1), ("b2", FIELD_B2)):
        arr[name] = _sym(seed, field, n, 0.01).reshape(shape)
    for name in ("c0", "c1", "c2"):
        arr[name] = np.ones(shape, dtype=np.float32)
    bnd = np.zeros(shape, dtype=np.float32)
    bnd[1:-1, 1:-1, 1:-1] = 1.0
    arr["bnd"] = bnd
    arr["wrk1"] = _sym(seed, FIELD_WRK1, n, 0.1).reshape(shape)
    arr["p"] = uniform(seed, FIELD_P0, n).astype(np.float32).reshape(shape)
    arr["wrk2"] = np.zeros(shape, dtype=np.float32)
    return arr


def make_batch(n_grids: int, base: int = BASE_SEED):
    """A batch of uneven grids: list of (shape, arrays) pairs."""
    out = []
    for g, (I, J, K) in enumerate(batch_sizes(n_grids, base)):
        out.append(((I, J, K), make_problem(I, J, K, grid_seed(g, base))))
    return out


def interior_points(I: int, J: int, K: int) -> int:
    return (I - 2) * (J - 2) * (K - 2)
