"""Plant plausible mistakes in copies of oracle.c (on the CPU) and check that
the pins in test_oracle_pins.py catch every one of them."""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import test_oracle_gemm as gpins
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, original text, replacement); each original must occur exactly once.
MUTANTS = [
    ("b0 bracket sign", "- AT(p, i + 1, j - 1, k)", "+ AT(p, i + 1, j - 1, k)"),
    ("b1/b2 swapped", "co[B1][c] * cross_jk", "co[B2][c] * cross_jk"),
    ("b2 bracket k-index", "- AT(p, i + 1, j, k - 1)", "- AT(p, i + 1, j, k + 1)"),
    ("wrk1 dropped", "+ face_minus + co[WRK1][c];", "+ face_minus;"),
    ("a3 misplaced", "(co[A3][c] * s0 - p[c])", "co[A3][c] * (s0 - p[c])"),
    ("bnd ignored", "return (co[A3][c] * s0 - p[c]) * co[BND][c];", "return (co[A3][c] * s0 - p[c]);"),
    ("c2 neighbour wrong", "+ co[C2][c] * AT(p, i, j, k - 1);", "+ co[C2][c] * AT(p, i, j, k + 1);"),
    ("a1 uses i-neighbour", "+ co[A1][c] * AT(p, i, j + 1, k)", "+ co[A1][c] * AT(p, i + 1, j, k)"),
    ("omega not applied", "AT(p, i, j, k) + omega * ss;", "AT(p, i, j, k) + ss;"),
    ("gauss-seidel", "oracle_sweep(I, J, K, co, p, omega, wrk2, &last) != 0", "oracle_sweep(I, J, K, co, p, omega, p, &last) != 0"),
    ("residual sum restarted per plane", "        plane[k - 1] = sum;\n    }\n    if (gosa)",
     "        plane[k - 1] = sum;\n    }\n    plane[0] = 0.0;\n    if (gosa)"),
    ("interior short in i", "for (int i = 1; i < I - 1; ++i) {\n                double ss = ss_at(I, J, co, p, i, j, k);\n                AT(wrk2",
     "for (int i = 1; i < I - 2; ++i) {\n                double ss = ss_at(I, J, co, p, i, j, k);\n                AT(wrk2"),
    ("residual of new iterate", "    free(wrk2);\n    *gosa = last;", "    oracle_residual(I, J, K, co, p, &last);\n    free(wrk2);\n    *gosa = last;"),
    ("bf16 ties away", "(low == 0x8000u && lsb)", "(low == 0x8000u)"),
    # matrix product (each stays inside the operands' bounds)
    ("gemm first term dropped", "for (int k = 0; k < K; ++k)\n                sum +=",
     "for (int k = 1; k < K; ++k)\n                sum +="),
    ("gemm last term dropped", "for (int k = 0; k < K; ++k)\n                sum +=",
     "for (int k = 0; k < K - 1; ++k)\n                sum +="),
    ("gemm product subtracted", "                sum += a[", "                sum -= a["),
    ("gemm sum never reset", "            double sum = 0.0;\n            for (int k", "            static double sum = 0.0;\n            for (int k"),
]

PIN_CHECKS = [
    pins.test_hand_3x3x3,
    pins.test_hand_4x3x3_jacobi_order,
    lambda: pins.test_eigenmode_closed_form((9, 7, 11), (3, 2, 5), 0.8, 4),
    pins.test_constant_field_fixed_point,
    pins.test_delta_probe_recovers_stencil_table,
    lambda: pins.test_bilinear_probe_isolates_cross_term("ij", "b0"),
    lambda: pins.test_bilinear_probe_isolates_cross_term("jk", "b1"),
    lambda: pins.test_bilinear_probe_isolates_cross_term("ik", "b2"),
    lambda: pins.test_mirror_symmetry("i"),
    pins.test_bnd_zero_freezes_point_and_boundary_is_untouched,
    pins.test_residual_of_current_iterate,
    lambda: pins.test_brute_force_matrix_formulation((5, 5, 5)),
    pins.test_bf16_ties_to_even,
    gpins.test_hand_worked_product,
    lambda: gpins.test_ones_sum_to_k(3, 5, 7),
    gpins.test_identity_and_diagonal_scaling,
    gpins.test_permutation_moves_rows_not_columns,
    gpins.test_outer_product_and_transpose_identity,
    gpins.test_small_integer_products_against_brute_force,
]


# Plausible mistakes in the offset-bfloat16 bias (oracle.offset_bias, the one
# oracle function written in Python), planted by replacing the function.
def _bias_mean(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    if np.array_equal(oracle.bf16_rne(x), x):
        return np.float32(0.0)
    return np.float32(np.mean(x, dtype=np.float64))


def _bias_no_exact_rule(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    return np.float32(0.5 * (float(x.min()) + float(x.max())))


def _bias_min(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    if np.array_equal(oracle.bf16_rne(x), x):
        return np.float32(0.0)
    return np.float32(x.min())


def _bias_exact_rule_inverted(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    if not np.array_equal(oracle.bf16_rne(x), x):
        return np.float32(0.0)
    return np.float32(0.5 * (float(x.min()) + float(x.max())))


BIAS_MUTANTS = [("bias is the mean", _bias_mean), ("bias without the exactness rule", _bias_no_exact_rule),
                ("bias is the minimum", _bias_min), ("exactness rule inverted", _bias_exact_rule_inverted)]

BIAS_PIN_CHECKS = [
    pins.test_offset_bias_is_the_mid_range_not_the_mean,
    pins.test_offset_bias_halves_the_range_of_a_skewed_draw,
    pins.test_offset_bias_is_zero_for_bfloat16_exact_arrays,
    pins.test_offset_encoding_rule,
]


def test_unmutated_bias_passes_every_check():
    for check in BIAS_PIN_CHECKS:
        check()


@pytest.mark.parametrize("name,fn", BIAS_MUTANTS, ids=[m[0] for m in BIAS_MUTANTS])
def test_pins_catch_bias_mutant(monkeypatch, name, fn):
    monkeypatch.setattr(oracle, "offset_bias", fn)
    caught = []
    for n, check in enumerate(BIAS_PIN_CHECKS):
        try:
            check()
        except AssertionError:
            caught.append(n)
    assert caught, f"no pin caught mutant {name!r}"


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mutants_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _build_mutant(workdir, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor for {name!r} not unique"
    tag = "".join(c if c.isalnum() else "_" for c in name)
    src = os.path.join(workdir, f"{tag}.c")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    shutil.copy(os.path.join(os.path.dirname(SRC), "oracle.h"), workdir)
    lib = os.path.join(workdir, f"lib{tag}.so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-Wno-unknown-pragmas", "-o", lib,
                    src, "-lm"], check=True)
    return lib


def test_unmutated_oracle_passes_every_check():
    for check in PIN_CHECKS:
        check()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(workdir, name, old, new):
    lib = _build_mutant(workdir, name, old, new)
    caught = []
    with oracle.use_library(lib):
        for n, check in enumerate(PIN_CHECKS):
            try:
                check()
            except (AssertionError, ValueError):
                caught.append(n)
    assert caught, f"no pin caught mutant {name!r}"
