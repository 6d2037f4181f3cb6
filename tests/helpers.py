"""Shared test helpers: error norms and oracle comparisons."""

import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ofl.h")
OMEGA = np.float32(0.8)
INNER = (slice(1, -1),) * 3

# Tolerances for FP32 arithmetic against the FP64 oracle (relative, max-norm
# over the interior for p; relative for the residual sum).
TOL_P_F32 = 1e-5
TOL_GOSA_F32 = 1e-4
# bfloat16-stored coefficients and batched forms.
TOL_BF16 = 1e-3


def p_rel_err(p, p_ref):
    p = np.asarray(p, np.float64)
    p_ref = np.asarray(p_ref, np.float64)
    return float(np.max(np.abs(p[INNER] - p_ref[INNER])) / np.max(np.abs(p_ref[INNER])))


def rel_err(x, ref):
    return abs(float(x) - float(ref)) / abs(float(ref))


def boundary_equal(p, p0):
    shell = np.ones(p.shape, bool)
    shell[INNER] = False
    return np.array_equal(np.asarray(p)[shell], np.asarray(p0)[shell])


def header_functions():
    import re

    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ofl_[a-z0-9_]+)\s*\(", text)))
