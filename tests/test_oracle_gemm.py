"""Pins of the oracle's matrix product (the definition the matrix-product
function block is checked against): small cases worked out by hand, closed
forms, and identities a transposed operand, a dropped term or a wrong index
would break."""

import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_hand_worked_product():
    case = json.load(open(os.path.join(HERE, "golden", "gemm_2x3x2.json")))
    c = oracle.gemm(np.array(case["A"]), np.array(case["B"]))
    assert c.tolist() == case["C"]


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (3, 5, 7), (8, 2, 9), (4, 4, 0)])
def test_ones_sum_to_k(M, N, K):
    assert np.array_equal(oracle.gemm(np.ones((M, K)), np.ones((K, N))), np.full((M, N), float(K)))


def test_identity_and_diagonal_scaling():
    rng = np.random.default_rng(3)
    b = rng.integers(-9, 10, size=(5, 6)).astype(float)
    assert np.array_equal(oracle.gemm(np.eye(5), b), b)
    d = np.array([1.0, -2.0, 3.0, 0.5, 4.0])
    assert np.array_equal(oracle.gemm(np.diag(d), b), d[:, None] * b)
    assert np.array_equal(oracle.gemm(b.T, np.diag(d)), b.T * d[None, :])


def test_permutation_moves_rows_not_columns():
    # catches a transposed operand: P A permutes A's rows, P^T A the inverse way
    a = np.arange(20, dtype=float).reshape(4, 5)
    perm = [2, 0, 3, 1]
    p = np.zeros((4, 4))
    p[np.arange(4), perm] = 1.0
    assert np.array_equal(oracle.gemm(p, a), a[perm])


def test_outer_product_and_transpose_identity():
    rng = np.random.default_rng(5)
    u = rng.integers(-5, 6, size=(6, 1)).astype(float)
    v = rng.integers(-5, 6, size=(1, 4)).astype(float)
    assert np.array_equal(oracle.gemm(u, v), u[:, 0][:, None] * v[0][None, :])
    a = rng.integers(-5, 6, size=(3, 7)).astype(float)
    b = rng.integers(-5, 6, size=(7, 2)).astype(float)
    assert np.array_equal(oracle.gemm(a, b).T, oracle.gemm(b.T, a.T))


def test_small_integer_products_against_brute_force():
    rng = np.random.default_rng(11)
    for M, N, K in [(2, 3, 4), (5, 1, 3), (1, 6, 2)]:
        a = rng.integers(-4, 5, size=(M, K))
        b = rng.integers(-4, 5, size=(K, N))
        want = [[sum(int(a[i, k]) * int(b[k, j]) for k in range(K)) for j in range(N)] for i in range(M)]
        assert oracle.gemm(a, b).tolist() == want
