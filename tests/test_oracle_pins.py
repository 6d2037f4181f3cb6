"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test is chosen so that a plausible slip in oracle.c (a dropped term, a
wrong sign or index, a transposed operand, Gauss-Seidel instead of Jacobi, the
wrong iterate's residual) fails at least one of them:

* hand-worked dyadic cases (tests/golden/*.json), exact in FP64;
* the eigenmode closed form of the constant-coefficient operator;
* the constant-field fixed point;
* the 19-point stencil table read back with delta probes;
* bilinear probes that isolate each cross term and its sign;
* mirror and transposition symmetries;
* invariants: bnd = 0 freezes a point, the boundary never moves, split runs,
  linearity in (p, wrk1);
* brute force against an independently assembled sparse-matrix formulation;
* bfloat16 rounding against torch's own conversion.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
COEFS = oracle.COEF_NAMES


def _blank(I, J, K, fill=0.0):
    return {n: np.full((K, J, I), fill, np.float64) for n in COEFS + ("p",)}


def _random_problem(I, J, K, seed):
    rng = np.random.default_rng(seed)
    arr = {}
    for n in COEFS:
        arr[n] = rng.uniform(-1.0, 1.0, (K, J, I))
    arr["bnd"] = np.ones((K, J, I))
    arr["p"] = rng.uniform(-1.0, 1.0, (K, J, I))
    return arr


# ---------------------------------------------------------------- hand cases


def test_hand_3x3x3():
    fx = json.load(open(os.path.join(GOLDEN, "hand_3x3x3.json")))
    I, J, K = fx["shape_IJK"]
    arr = _blank(I, J, K, fx["off_centre_coefficient_value"])
    for n, v in fx["centre_coefficients"].items():
        arr[n][1, 1, 1] = v
    k, j, i = np.meshgrid(np.arange(K), np.arange(J), np.arange(I), indexing="ij")
    arr["p"] = (i + 3 * j + 9 * k + i * j + 2 * j * k + 3 * i * k).astype(np.float64)
    for case in fx["expected"]:
        p, gosa = oracle.jacobi(arr, case["iters"], fx["omega"])
        assert p[1, 1, 1] == case["p_centre"]
        assert gosa == case["gosa"]
        mask = np.ones_like(p, bool)
        mask[1, 1, 1] = False
        assert np.array_equal(p[mask], arr["p"][mask])


def test_hand_4x3x3_jacobi_order():
    fx = json.load(open(os.path.join(GOLDEN, "hand_4x3x3.json")))
    I, J, K = fx["shape_IJK"]
    arr = _blank(I, J, K)
    for n, v in fx["coefficients_everywhere"].items():
        arr[n][:] = v
    arr["p"][1, 1, 1] = 8
    arr["p"][1, 1, 2] = 16
    arr["p"][1, 1, 3] = 32
    for case in fx["expected"]:
        p, gosa = oracle.jacobi(arr, case["iters"], fx["omega"])
        assert p[1, 1, 1] == case["p_1"]
        assert p[1, 1, 2] == case["p_2"]
        assert gosa == case["gosa"]


def test_zero_iterations():
    arr = _random_problem(5, 4, 3, 1)
    p, gosa = oracle.jacobi(arr, 0, 0.8)
    assert np.array_equal(p, arr["p"])
    assert math.isnan(gosa)


def test_bad_arguments_rejected():
    arr = _random_problem(2, 4, 4, 1)
    with pytest.raises(ValueError):
        oracle.jacobi(arr, 1, 0.8)
    arr = _random_problem(4, 4, 4, 1)
    with pytest.raises(ValueError):
        oracle.jacobi(arr, -1, 0.8)


# ------------------------------------------------------------ closed forms


@pytest.mark.parametrize("dims,lmn,omega,iters", [
    ((9, 7, 11), (1, 1, 1), 0.8, 5),
    ((9, 7, 11), (3, 2, 5), 0.8, 4),
    ((12, 6, 8), (7, 4, 1), 1.0, 3),
    ((6, 6, 6), (2, 3, 4), 0.5, 6),
])
def test_eigenmode_closed_form(dims, lmn, omega, iters):
    """a=c=1, b=0, a3=1/6, wrk1=0, zero boundary: a product of sines is an
    eigenvector of the neighbour average with eigenvalue
    lam = (cos(pi l/(I-1)) + cos(pi m/(J-1)) + cos(pi n/(K-1)))/3, so one
    iteration multiplies it by mu = 1 - omega (1 - lam) and the residual of the
    last sweep is (1-lam)^2 mu^(2(N-1)) (I-1)(J-1)(K-1)/8."""
    I, J, K = dims
    l, m, n = lmn
    arr = _blank(I, J, K)
    for name in ("a0", "a1", "a2", "c0", "c1", "c2", "bnd"):
        arr[name][:] = 1.0
    arr["a3"][:] = 1.0 / 6.0
    k, j, i = np.meshgrid(np.arange(K), np.arange(J), np.arange(I), indexing="ij")
    e = (np.sin(np.pi * l * i / (I - 1)) * np.sin(np.pi * m * j / (J - 1))
         * np.sin(np.pi * n * k / (K - 1)))
    arr["p"] = e.copy()
    lam = (math.cos(math.pi * l / (I - 1)) + math.cos(math.pi * m / (J - 1))
           + math.cos(math.pi * n / (K - 1))) / 3.0
    mu = 1.0 - omega * (1.0 - lam)
    p, gosa = oracle.jacobi(arr, iters, omega)
    np.testing.assert_allclose(p, mu ** iters * e, rtol=0, atol=1e-13)
    want = (1.0 - lam) ** 2 * mu ** (2 * (iters - 1)) * (I - 1) * (J - 1) * (K - 1) / 8.0
    assert gosa == pytest.approx(want, rel=1e-12)


def test_constant_field_fixed_point():
    """With c_d = a_d, wrk1 = 0 and a3 = 1/(sum a + sum c) the constant field is
    a fixed point whatever the cross coefficients are."""
    I, J, K = 8, 7, 9
    rng = np.random.default_rng(5)
    arr = _blank(I, J, K)
    for d in range(3):
        a = rng.uniform(0.9, 1.1, (K, J, I))
        arr[f"a{d}"] = a
        arr[f"c{d}"] = a.copy()
    for d in range(3):
        arr[f"b{d}"] = rng.uniform(-0.5, 0.5, (K, J, I))
    arr["a3"] = 1.0 / (2.0 * (arr["a0"] + arr["a1"] + arr["a2"]))
    arr["bnd"][:] = 1.0
    arr["p"][:] = 0.37
    p, gosa = oracle.jacobi(arr, 10, 0.8)
    assert np.max(np.abs(p - 0.37)) < 1e-15
    assert gosa < 1e-28


# ---------------------------------------------------------- stencil wiring

# The 19-point stencil read as a table: offset (di, dj, dk) of the neighbour,
# the coefficient that multiplies it, and its sign.
STENCIL = {
    (1, 0, 0): ("a0", 1), (0, 1, 0): ("a1", 1), (0, 0, 1): ("a2", 1),
    (-1, 0, 0): ("c0", 1), (0, -1, 0): ("c1", 1), (0, 0, -1): ("c2", 1),
    (1, 1, 0): ("b0", 1), (1, -1, 0): ("b0", -1), (-1, 1, 0): ("b0", -1), (-1, -1, 0): ("b0", 1),
    (0, 1, 1): ("b1", 1), (0, -1, 1): ("b1", -1), (0, 1, -1): ("b1", -1), (0, -1, -1): ("b1", 1),
    (1, 0, 1): ("b2", 1), (-1, 0, 1): ("b2", -1), (1, 0, -1): ("b2", -1), (-1, 0, -1): ("b2", 1),
}


def test_delta_probe_recovers_stencil_table():
    """p = delta at q: the sweep at x sees q only through the coefficient of
    offset q - x, so ss(x) = a3(x) * sign * coef(x) - [x == q]."""
    I, J, K = 7, 6, 8
    rng = np.random.default_rng(11)
    arr = {n: rng.uniform(0.5, 2.0, (K, J, I)) for n in COEFS}
    arr["bnd"][:] = 1.0
    arr["wrk1"][:] = 0.0
    q = (3, 2, 4)  # (i, j, k) of the delta
    arr["p"] = np.zeros((K, J, I))
    arr["p"][q[2], q[1], q[0]] = 1.0
    wrk2, _ = oracle.sweep(arr, 1.0)
    for k in range(1, K - 1):
        for j in range(1, J - 1):
            for i in range(1, I - 1):
                off = (q[0] - i, q[1] - j, q[2] - k)
                if off == (0, 0, 0):
                    want = -1.0
                elif off in STENCIL:
                    name, sign = STENCIL[off]
                    want = arr["a3"][k, j, i] * sign * arr[name][k, j, i]
                else:
                    want = 0.0
                got = wrk2[k, j, i] - arr["p"][k, j, i]
                assert got == pytest.approx(want, abs=1e-15), (i, j, k, off)
    assert len(STENCIL) + 1 == 19


@pytest.mark.parametrize("poly,coef", [("ij", "b0"), ("jk", "b1"), ("ik", "b2")])
def test_bilinear_probe_isolates_cross_term(poly, coef):
    """For p = x*y every mixed second difference vanishes except the x-y one,
    which equals 4; with a = c = 0, a3 = 1: ss = 4*b_xy - p."""
    I, J, K = 6, 7, 5
    rng = np.random.default_rng(3)
    arr = _blank(I, J, K)
    for name in ("b0", "b1", "b2"):
        arr[name] = rng.uniform(-1, 1, (K, J, I))
    arr["a3"][:] = 1.0
    arr["bnd"][:] = 1.0
    k, j, i = np.meshgrid(np.arange(K), np.arange(J), np.arange(I), indexing="ij")
    arr["p"] = {"ij": i * j, "jk": j * k, "ik": i * k}[poly].astype(np.float64)
    wrk2, _ = oracle.sweep(arr, 1.0)
    sl = (slice(1, -1),) * 3
    np.testing.assert_allclose((wrk2 - arr["p"])[sl], (4.0 * arr[coef] - arr["p"])[sl], rtol=0, atol=1e-13)


# ---------------------------------------------------------------- symmetry


def _mirror(arr, axis_name):
    ax = {"i": 2, "j": 1, "k": 0}[axis_name]
    d = {"i": 0, "j": 1, "k": 2}[axis_name]
    out = {n: np.flip(v, axis=ax).copy() for n, v in arr.items()}
    out[f"a{d}"], out[f"c{d}"] = out[f"c{d}"], out[f"a{d}"]
    negate = {"i": ("b0", "b2"), "j": ("b0", "b1"), "k": ("b1", "b2")}[axis_name]
    for n in negate:
        out[n] = -out[n]
    return out, ax


@pytest.mark.parametrize("axis_name", ["i", "j", "k"])
def test_mirror_symmetry(axis_name):
    arr = _random_problem(7, 6, 8, 21)
    p_ref, g_ref = oracle.jacobi(arr, 3, 0.8)
    marr, ax = _mirror(arr, axis_name)
    p_m, g_m = oracle.jacobi(marr, 3, 0.8)
    np.testing.assert_allclose(np.flip(p_m, axis=ax), p_ref, rtol=0, atol=1e-13)
    assert g_m == pytest.approx(g_ref, rel=1e-13)


def test_ij_transposition_symmetry():
    arr = _random_problem(7, 7, 6, 22)
    p_ref, g_ref = oracle.jacobi(arr, 3, 0.8)
    t = {n: np.swapaxes(v, 1, 2).copy() for n, v in arr.items()}
    t["a0"], t["a1"] = t["a1"], t["a0"]
    t["c0"], t["c1"] = t["c1"], t["c0"]
    t["b1"], t["b2"] = t["b2"], t["b1"]
    p_t, g_t = oracle.jacobi(t, 3, 0.8)
    np.testing.assert_allclose(np.swapaxes(p_t, 1, 2), p_ref, rtol=0, atol=1e-13)
    assert g_t == pytest.approx(g_ref, rel=1e-13)


# -------------------------------------------------------------- invariants


def test_bnd_zero_freezes_point_and_boundary_is_untouched():
    arr = _random_problem(6, 5, 7, 31)
    arr["bnd"][3, 2, 2] = 0.0
    p, _ = oracle.jacobi(arr, 4, 0.8)
    assert p[3, 2, 2] == arr["p"][3, 2, 2]
    shell = np.ones(p.shape, bool)
    shell[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(p[shell], arr["p"][shell])
    assert not np.array_equal(p[1:-1, 1:-1, 1:-1], arr["p"][1:-1, 1:-1, 1:-1])


def test_split_runs_equal_one_run():
    arr = _random_problem(6, 7, 5, 41)
    p_full, g_full = oracle.jacobi(arr, 6, 0.8)
    p_half, _ = oracle.jacobi(arr, 3, 0.8)
    arr2 = dict(arr, p=p_half)
    p_two, g_two = oracle.jacobi(arr2, 3, 0.8)
    assert np.array_equal(p_two, p_full)
    assert g_two == g_full


def test_linear_in_p_and_wrk1():
    """p^(N) is linear in (p^(0), wrk1) jointly: F(x + y) = F(x) + F(y)."""
    base = _random_problem(6, 6, 6, 51)
    rng = np.random.default_rng(52)
    x = dict(base, p=rng.uniform(-1, 1, base["p"].shape), wrk1=rng.uniform(-1, 1, base["p"].shape))
    y = dict(base, p=rng.uniform(-1, 1, base["p"].shape), wrk1=rng.uniform(-1, 1, base["p"].shape))
    xy = dict(base, p=x["p"] + y["p"], wrk1=x["wrk1"] + y["wrk1"])
    fx, _ = oracle.jacobi(x, 3, 0.8)
    fy, _ = oracle.jacobi(y, 3, 0.8)
    fxy, _ = oracle.jacobi(xy, 3, 0.8)
    np.testing.assert_allclose(fxy, fx + fy, rtol=0, atol=1e-12)


def test_residual_of_current_iterate():
    """oracle_residual(p) equals the gosa the next sweep reports."""
    arr = _random_problem(6, 5, 6, 61)
    r0 = oracle.residual(arr)
    _, g1 = oracle.jacobi(arr, 1, 0.8)
    assert r0 == g1


def test_manufactured_solution():
    """Choose a smooth target field, then pick wrk1 (on the interior) so the
    target is a fixed point: wrk1 := -ss0/a3 where ss0 is the sweep's ss for
    the target with wrk1 = 0. From the target the residual is round-off and p
    stays put; from a perturbed start a diagonally dominant set converges."""
    I, J, K = 9, 8, 10
    rng = np.random.default_rng(71)
    arr = {n: np.zeros((K, J, I)) for n in COEFS}
    for d in range(3):
        arr[f"a{d}"] = rng.uniform(0.95, 1.05, (K, J, I))
        arr[f"c{d}"] = rng.uniform(0.95, 1.05, (K, J, I))
        arr[f"b{d}"] = rng.uniform(-0.01, 0.01, (K, J, I))
    diag = sum(arr[f"a{d}"] + arr[f"c{d}"] for d in range(3))
    arr["a3"] = 1.0 / diag
    arr["bnd"][1:-1, 1:-1, 1:-1] = 1.0
    k, j, i = np.meshgrid(np.arange(K), np.arange(J), np.arange(I), indexing="ij")
    target = np.sin(0.3 * i) * np.cos(0.2 * j) + 0.01 * k * k
    arr["p"] = target.copy()
    wrk2, _ = oracle.sweep(arr, 1.0)
    ss0 = wrk2 - target
    arr["wrk1"] = np.zeros_like(target)
    arr["wrk1"][1:-1, 1:-1, 1:-1] = -ss0[1:-1, 1:-1, 1:-1] / arr["a3"][1:-1, 1:-1, 1:-1]
    p, gosa = oracle.jacobi(arr, 5, 0.8)
    assert gosa < 1e-26
    np.testing.assert_allclose(p, target, rtol=0, atol=1e-13)
    pert = target.copy()
    pert[1:-1, 1:-1, 1:-1] += rng.uniform(-0.1, 0.1, (K - 2, J - 2, I - 2))
    errs = []
    for n in (1, 10, 40):
        pn, _ = oracle.jacobi(dict(arr, p=pert), n, 0.8)
        errs.append(np.max(np.abs(pn - target)))
    assert errs[0] > errs[1] > errs[2]


# ------------------------------------------------------------- brute force


def _assembled_step(arr, omega):
    """Test-only formulation: assemble the stencil as a sparse matrix over all
    points, then p_interior <- p + omega * bnd * (a3 * (M p + wrk1) - p)."""
    import scipy.sparse as sp

    K, J, I = arr["p"].shape
    n = I * J * K
    lin = lambda i, j, k: i + I * (j + J * k)
    rows, cols, vals = [], [], []
    for k in range(1, K - 1):
        for j in range(1, J - 1):
            for i in range(1, I - 1):
                r = lin(i, j, k)
                for (di, dj, dk), (name, sign) in STENCIL.items():
                    rows.append(r)
                    cols.append(lin(i + di, j + dj, k + dk))
                    vals.append(sign * arr[name][k, j, i])
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    p = arr["p"].reshape(-1)
    interior = np.zeros((K, J, I), bool)
    interior[1:-1, 1:-1, 1:-1] = True
    interior = interior.reshape(-1)
    a3 = arr["a3"].reshape(-1)
    ss = (a3 * (M @ p + arr["wrk1"].reshape(-1)) - p) * arr["bnd"].reshape(-1)
    new = p.copy()
    new[interior] = p[interior] + omega * ss[interior]
    return new.reshape(K, J, I), float(np.sum(ss[interior] ** 2))


@pytest.mark.parametrize("dims", [(3, 3, 3), (4, 3, 5), (5, 5, 5), (3, 5, 4)])
def test_brute_force_matrix_formulation(dims):
    I, J, K = dims
    arr = _random_problem(I, J, K, 81 + I + J + K)
    arr["bnd"] = np.random.default_rng(9).choice([0.0, 1.0], size=arr["p"].shape, p=[0.2, 0.8])
    cur = dict(arr)
    for it in range(3):
        want_p, want_g = _assembled_step(cur, 0.8)
        cur = dict(cur, p=want_p)
    p, g = oracle.jacobi(arr, 3, 0.8)
    np.testing.assert_allclose(p, want_p, rtol=0, atol=1e-13)
    assert g == pytest.approx(want_g, rel=1e-12, abs=1e-15)


# ---------------------------------------------------------------- bfloat16


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(91)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32),
        rng.uniform(0.95, 1.05, 20000).astype(np.float32),
        np.array([0.0, -0.0, 1.0, np.inf, -np.inf, 3.3895314e38, 1e-40, -1e-42], np.float32),
    ])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = oracle.bf16_rne(x)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert np.isnan(oracle.bf16_rne(np.array([np.nan], np.float32))[0])


def test_bf16_ties_to_even():
    one_half_ulp = np.float32(1.0 + 2.0 ** -8)         # halfway 1 .. 1+2^-7 -> even (1)
    three_half = np.float32(1.0 + 3.0 * 2.0 ** -8)     # halfway 1+2^-7 .. 1+2^-6 -> even (1+2^-6)
    above = np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)    # just above halfway -> up
    got = oracle.bf16_rne(np.array([one_half_ulp, three_half, above], np.float32))
    assert got.tolist() == [1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7]


def test_offset_encoding_rule():
    a = synth.make_problem(9, 8, 7)
    assert oracle.offset_bias(a["c0"]) == 0.0
    assert oracle.offset_bias(a["bnd"]) == 0.0
    assert abs(float(oracle.offset_bias(a["a0"])) - 1.0) < 1e-3
    assert abs(float(oracle.offset_bias(a["a3"])) - 1.0 / 6.0) < 2e-3
    dec = oracle.offset_bf16_decode(a["a0"], oracle.offset_bias(a["a0"]))
    plain = oracle.bf16_rne(a["a0"])
    err_off = np.max(np.abs(dec.astype(np.float64) - a["a0"]))
    err_plain = np.max(np.abs(plain.astype(np.float64) - a["a0"]))
    assert err_off <= 0.05 * 2.0 ** -8 * 1.01 + 2.0 ** -24
    assert err_plain > 8 * err_off


def test_all_cores_build_is_bit_identical():
    """The same oracle.c built with -fopenmp (the all-cores CPU baseline) runs
    the planes on several threads; each plane is still summed in j, i order
    and the plane sums in k order, so p and the residual are bit-identical to
    the single-thread build's."""
    import oracle.build as ob

    if not os.path.exists(ob.LIB_OMP):
        ob.build()
    a = synth.make_problem(37, 29, 41, seed=23)
    p1, g1 = oracle.jacobi(a, 6, 0.8)
    r1 = oracle.residual(dict(a, p=p1))
    with oracle.use_library(ob.LIB_OMP):
        threads = oracle.threads()
        p2, g2 = oracle.jacobi(a, 6, 0.8)
        r2 = oracle.residual(dict(a, p=p2))
    assert oracle.threads() == 1 and threads >= 1
    assert np.array_equal(p1, p2) and g1 == g2 and r1 == r2


def test_offset_bias_is_the_mid_range_not_the_mean():
    """Hand-worked: [1+e, 1+e, 1+e, 1.5+e] with e = 2^-20 (not bfloat16-exact)
    has mid-range 1.25+e and mean 1.125+e; the bias is the mid-range, exactly
    (1.25+e is an FP32 value)."""
    e = 2.0 ** -20
    x = np.array([1 + e, 1 + e, 1 + e, 1.5 + e], np.float32)
    assert oracle.offset_bias(x) == np.float32(1.25 + e)
    # one value off the bfloat16 grid is enough: [-3, 0.5, 1, 1.5+e] -> -0.75 + e/2
    x = np.array([1.0, 0.5, -3.0, 1.5 + e], np.float32)
    assert oracle.offset_bias(x) == np.float32(-0.75 + e / 2)


def test_offset_bias_halves_the_range_of_a_skewed_draw():
    """The mid-range is the one bias that makes max|x - bias| half the range;
    on a draw crowded at the bottom of [0.95, 1.05] (mean about 0.964) any
    other centre, the mean among them, leaves some value farther away."""
    rng = np.random.default_rng(7)
    x = (0.95 + 0.1 * rng.uniform(0, 1, 4096) ** 6).astype(np.float32)
    b = float(oracle.offset_bias(x))
    lo, hi = float(x.min()), float(x.max())
    half = (hi - lo) / 2
    dev = np.max(np.abs(x.astype(np.float64) - b))
    assert dev <= half + 2.0 ** -24 and dev >= half - 2.0 ** -24
    assert abs(b - float(x.mean(dtype=np.float64))) > 0.03


def test_offset_bias_is_zero_for_bfloat16_exact_arrays():
    """Every value already on the bfloat16 grid: no bias (the encoding is then
    exact), whatever the range."""
    x = np.array([1.0, 0.5, -3.0, 1.5, 2.0 ** -10, 96.0], np.float32)
    assert oracle.offset_bias(x) == 0.0
    assert oracle.offset_bias(np.full(10, 0.25, np.float32)) == 0.0


# ------------------------------------------------------- generator contract


def test_generator_matches_published_splitmix64():
    """SplitMix64 with state 0 yields 0xE220A8397B1DCDAF first (the published
    reference sequence of the algorithm)."""
    assert synth.mix64_int(synth.GAMMA) == 0xE220A8397B1DCDAF
    got = synth.mix64(np.array([synth.GAMMA, 2 * synth.GAMMA & ((1 << 64) - 1)], np.uint64))
    assert int(got[0]) == 0xE220A8397B1DCDAF
    assert int(got[1]) == 0x6E789E6AA1B965F4


def test_generator_distributions():
    a = synth.make_problem(17, 9, 11)
    for n in ("a0", "a1", "a2"):
        assert 0.95 <= a[n].min() and a[n].max() <= 1.05
    np.testing.assert_array_equal(a["a3"], (1.0 / (2.0 * (a["a0"].astype(np.float64) + a["a1"] + a["a2"]))).astype(np.float32))
    for n in ("b0", "b1", "b2"):
        assert -0.01 <= a[n].min() and a[n].max() <= 0.01
    assert np.all(a["c0"] == 1) and np.all(a["wrk2"] == 0)
    assert a["bnd"].sum() == synth.interior_points(17, 9, 11)
    assert 0 <= a["p"].min() and a["p"].max() < 1
    b = synth.make_problem(17, 9, 11)
    assert all(np.array_equal(a[n], b[n]) for n in a)
    sizes = synth.batch_sizes(64)
    assert all(33 <= I <= 161 and 33 <= J <= 161 and 65 <= K <= 321 for I, J, K in sizes)
