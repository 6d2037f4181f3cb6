"""GPU parity of the matrix-product routine (ofl_gemm_f32, the MFMA kernel a
recognised matrix-product block is replaced with) against the FP64 oracle.

Bar, per element: |C - C_ref| <= 2 K 2^-24 (|A| |B|)_ij, the error bound of
an FP32 sum of K products (the FP32 products and sums of the matrix cores, in
any order)."""

import sys

import numpy as np
import pytest

import oracle
import paper_2011_03602_amd as ofl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, skipped there
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="needs a GPU")]


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def check(a, b, c):
    ref = oracle.gemm(a, b)
    bound = 2.0 * max(a.shape[1], 1) * 2.0 ** -24 * oracle.gemm(np.abs(a), np.abs(b)) + 1e-30
    err = np.abs(c.astype(np.float64) - ref)
    assert np.all(err <= bound), f"worst excess {float(np.max(err / bound)):.3f} of the bound"


def run(a, b, lda=None, ldb=None, ldc=None):
    """C = A B through the C interface, operands placed with the given row strides."""
    M, K = a.shape
    N = b.shape[1]
    lda, ldb, ldc = lda or max(K, 1), ldb or max(N, 1), ldc or max(N, 1)
    da = torch.zeros((max(M, 1), lda), dtype=torch.float32, device="cuda")
    db = torch.zeros((max(K, 1), ldb), dtype=torch.float32, device="cuda")
    dc = torch.full((max(M, 1), ldc), 7.0, dtype=torch.float32, device="cuda")
    if M and K:
        da[:M, :K] = torch.from_numpy(a)
    if K and N:
        db[:K, :N] = torch.from_numpy(b)
    ofl.ofl_gemm_f32(M, N, K, da.data_ptr(), lda, db.data_ptr(), ldb, dc.data_ptr(), ldc, None)
    torch.cuda.synchronize()
    out = dc.cpu().numpy()
    if ldc > N and M:
        assert np.all(out[:M, N:] == 7.0), "wrote past the row"
    return out[:M, :N]


SHAPES = [(1, 1, 1), (2, 3, 5), (33, 17, 5), (128, 128, 16), (129, 257, 33), (256, 128, 17), (300, 200, 64),
          (64, 512, 1), (511, 129, 300), (1000, 1000, 1000)]


@pytest.mark.parametrize("M,N,K", SHAPES)
def test_matches_oracle(M, N, K):
    say("gemm", M, N, K)
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    a = rng.uniform(-1, 1, (M, K)).astype(np.float32)
    b = rng.uniform(-1, 1, (K, N)).astype(np.float32)
    check(a, b, run(a, b))


@pytest.mark.parametrize("lda,ldb,ldc", [(67, 131, 133), (65, 130, 129), (68, 132, 136)])
def test_strided_and_unaligned_rows(lda, ldb, ldc):
    say("gemm strides", lda, ldb, ldc)
    rng = np.random.default_rng(1)
    a = rng.uniform(-1, 1, (150, 65)).astype(np.float32)
    b = rng.uniform(-1, 1, (65, 129)).astype(np.float32)
    check(a, b, run(a, b, lda, ldb, ldc))


def test_empty_and_zero_depth():
    say("gemm empty / K = 0")
    a = np.zeros((5, 0), np.float32)
    b = np.zeros((0, 4), np.float32)
    assert np.array_equal(run(a, b), np.zeros((5, 4), np.float32))
    ofl.ofl_gemm_f32(0, 4, 3, 0, 3, 0, 4, 0, 4, None)  # nothing to do, nothing touched
    ofl.ofl_gemm_f32(5, 0, 3, 0, 3, 0, 1, 0, 1, None)


def test_large_square_sampled():
    say("gemm 4096^3, sampled rows")
    M = N = K = 4096
    g = torch.Generator(device="cuda").manual_seed(9)
    da = torch.rand((M, K), device="cuda", generator=g) * 2 - 1
    db = torch.rand((K, N), device="cuda", generator=g) * 2 - 1
    dc = torch.empty((M, N), device="cuda")
    ofl.ofl_gemm_f32(M, N, K, da.data_ptr(), K, db.data_ptr(), N, dc.data_ptr(), N, None)
    torch.cuda.synchronize()
    rows = [0, 1, 127, 128, 2049, 4095]
    a = da[rows].cpu().numpy()
    b = db.cpu().numpy()
    check(a, b, dc[rows].cpu().numpy())


# Large ragged products on both tile heights: 4000 x 4000 fills whole rounds of
# 128-row tiles (512 tiles), 6000 x 6144 fills the rounds of 64-row tiles better
# (2256 tiles against 1128 in 2.2 rounds); rows near both ends and a tile edge.
@pytest.mark.parametrize("M,N,K", [(4000, 4000, 257), (6000, 6144, 129)])
def test_large_ragged_sampled(M, N, K):
    say("gemm", M, N, K, "sampled rows")
    g = torch.Generator(device="cuda").manual_seed(M + K)
    da = torch.rand((M, K), device="cuda", generator=g) * 2 - 1
    db = torch.rand((K, N), device="cuda", generator=g) * 2 - 1
    dc = torch.empty((M, N), device="cuda")
    ofl.ofl_gemm_f32(M, N, K, da.data_ptr(), K, db.data_ptr(), N, dc.data_ptr(), N, None)
    torch.cuda.synchronize()
    rows = [0, 63, 64, 127, 128, M // 2 + 1, M - 65, M - 2, M - 1]
    check(da[rows].cpu().numpy(), db.cpu().numpy(), dc[rows].cpu().numpy())
