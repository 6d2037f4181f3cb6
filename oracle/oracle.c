/*
 * oracle.c -- plain FP64 CPU reference for the offloaded Jacobi program.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may include, link,
 * load or call this file. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it. It shares no code, header, table or
 * helper with the GPU path.
 *
 * What it computes.
 * The paper (Sec. 3.2.1 and Sec. 4.2.2) offloads the loop nests of a CPU
 * program and keeps an offload pattern only if its results match the original
 * program's (Sec. 4.2.2: otherwise the pattern's time is set to infinity).
 * The paper does not print the program. The program used here is a 3D
 * variable-coefficient 19-point Jacobi relaxation with three loop nests per
 * iteration:
 *
 *   S (sweep), for every interior point (i,j,k), from the OLD iterate p:
 *     s0 = a0*p(i+1,j,k) + a1*p(i,j+1,k) + a2*p(i,j,k+1)
 *        + b0*[p(i+1,j+1,k) - p(i+1,j-1,k) - p(i-1,j+1,k) + p(i-1,j-1,k)]
 *        + b1*[p(i,j+1,k+1) - p(i,j-1,k+1) - p(i,j+1,k-1) + p(i,j-1,k-1)]
 *        + b2*[p(i+1,j,k+1) - p(i-1,j,k+1) - p(i+1,j,k-1) + p(i-1,j,k-1)]
 *        + c0*p(i-1,j,k) + c1*p(i,j-1,k) + c2*p(i,j,k-1) + wrk1
 *     ss   = (a3*s0 - p(i,j,k)) * bnd
 *     wrk2 = p(i,j,k) + omega*ss
 *   R (residual):  gosa = sum over the interior of ss^2
 *   C (copy-back): p <- wrk2 on the interior
 *
 * Every coefficient is taken at the centre point (i,j,k). The interior is
 * {1..I-2} x {1..J-2} x {1..K-2}; the outer one-cell layer of p is a Dirichlet
 * boundary and never changes. The update is Jacobi: all of wrk2 is computed
 * from the old p before any point of p changes.
 *
 * Arithmetic: FP64 throughout, inputs widened exactly from what the caller
 * stores. The residual is a plain sum over the interior in a fixed order: each
 * k-plane's squares are added in j, then i order, and the plane sums are then
 * added in k order. Build with -ffp-contract=off so that no multiply-add is
 * fused.
 *
 * The loops over k carry OpenMP directives. The plain build ignores them; a
 * build with -fopenmp runs the planes on all host cores, which is how the
 * oracle is timed on every core. Each plane is still computed by one thread in
 * the same order and the plane sums are added in k order afterwards, so both
 * builds give bit-identical results.
 *
 * Layout: linear index of (i,j,k) is i + I*(j + J*k), i fastest.
 * Coefficient order: a0 a1 a2 a3 b0 b1 b2 c0 c1 c2 bnd wrk1.
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { A0, A1, A2, A3, B0, B1, B2, C0, C1, C2, BND, WRK1, NCOEF };

#define AT(arr, i, j, k) (arr)[(size_t)(i) + (size_t)I * ((size_t)(j) + (size_t)J * (size_t)(k))]

static int dims_ok(int I, int J, int K)
{
    return I >= 3 && J >= 3 && K >= 3;
}

static int coefs_ok(const double *const co[ORACLE_NCOEF])
{
    if (!co)
        return 0;
    for (int n = 0; n < NCOEF; ++n)
        if (!co[n])
            return 0;
    return 1;
}

/* ss at one interior point, straight from the definition above. */
static double ss_at(int I, int J, const double *const co[ORACLE_NCOEF], const double *p, int i, int j, int k)
{
    const size_t c = (size_t)i + (size_t)I * ((size_t)j + (size_t)J * (size_t)k);
    double face_plus = co[A0][c] * AT(p, i + 1, j, k)
                     + co[A1][c] * AT(p, i, j + 1, k)
                     + co[A2][c] * AT(p, i, j, k + 1);
    double cross_ij = AT(p, i + 1, j + 1, k) - AT(p, i + 1, j - 1, k)
                    - AT(p, i - 1, j + 1, k) + AT(p, i - 1, j - 1, k);
    double cross_jk = AT(p, i, j + 1, k + 1) - AT(p, i, j - 1, k + 1)
                    - AT(p, i, j + 1, k - 1) + AT(p, i, j - 1, k - 1);
    double cross_ik = AT(p, i + 1, j, k + 1) - AT(p, i - 1, j, k + 1)
                    - AT(p, i + 1, j, k - 1) + AT(p, i - 1, j, k - 1);
    double face_minus = co[C0][c] * AT(p, i - 1, j, k)
                      + co[C1][c] * AT(p, i, j - 1, k)
                      + co[C2][c] * AT(p, i, j, k - 1);
    double s0 = face_plus + co[B0][c] * cross_ij + co[B1][c] * cross_jk + co[B2][c] * cross_ik
              + face_minus + co[WRK1][c];
    return (co[A3][c] * s0 - p[c]) * co[BND][c];
}

/* Sum of plane[0..n) in index order (the residual's plane sums, k order). */
static double sum_planes(const double *plane, int n)
{
    double sum = 0.0;
    for (int t = 0; t < n; ++t)
        sum += plane[t];
    return sum;
}

int oracle_sweep(int I, int J, int K, const double *const co[ORACLE_NCOEF], const double *p, double omega,
                 double *wrk2, double *gosa)
{
    if (!dims_ok(I, J, K) || !coefs_ok(co) || !p || !wrk2)
        return -1;
    double *plane = (double *)calloc((size_t)(K - 2), sizeof(double));
    if (!plane)
        return -2;
#pragma omp parallel for schedule(static)
    for (int k = 1; k < K - 1; ++k) {
        double sum = 0.0;
        for (int j = 1; j < J - 1; ++j)
            for (int i = 1; i < I - 1; ++i) {
                double ss = ss_at(I, J, co, p, i, j, k);
                AT(wrk2, i, j, k) = AT(p, i, j, k) + omega * ss;
                sum += ss * ss;
            }
        plane[k - 1] = sum;
    }
    if (gosa)
        *gosa = sum_planes(plane, K - 2);
    free(plane);
    return 0;
}

int oracle_residual(int I, int J, int K, const double *const co[ORACLE_NCOEF], const double *p, double *gosa)
{
    if (!dims_ok(I, J, K) || !coefs_ok(co) || !p || !gosa)
        return -1;
    double *plane = (double *)calloc((size_t)(K - 2), sizeof(double));
    if (!plane)
        return -2;
#pragma omp parallel for schedule(static)
    for (int k = 1; k < K - 1; ++k) {
        double sum = 0.0;
        for (int j = 1; j < J - 1; ++j)
            for (int i = 1; i < I - 1; ++i) {
                double ss = ss_at(I, J, co, p, i, j, k);
                sum += ss * ss;
            }
        plane[k - 1] = sum;
    }
    *gosa = sum_planes(plane, K - 2);
    free(plane);
    return 0;
}

int oracle_jacobi(int I, int J, int K, const double *const co[ORACLE_NCOEF], double *p, double omega, int iters,
                  double *gosa)
{
    if (!dims_ok(I, J, K) || !coefs_ok(co) || !p || !gosa || iters < 0)
        return -1;
    const size_t n = (size_t)I * (size_t)J * (size_t)K;
    double *wrk2 = (double *)calloc(n, sizeof(double));
    if (!wrk2)
        return -2;
    double last = NAN;
    for (int it = 0; it < iters; ++it) {
        /* nests S and R: new values from the old iterate, residual of the old iterate */
        if (oracle_sweep(I, J, K, co, p, omega, wrk2, &last) != 0) {
            free(wrk2);
            return -2;
        }
        /* nest C: copy back on the interior only */
#pragma omp parallel for schedule(static)
        for (int k = 1; k < K - 1; ++k)
            for (int j = 1; j < J - 1; ++j)
                for (int i = 1; i < I - 1; ++i)
                    AT(p, i, j, k) = AT(wrk2, i, j, k);
    }
    free(wrk2);
    *gosa = last;
    return 0;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Round an FP32 value to the nearest bfloat16 (ties to even), returned widened
 * back to FP32. bfloat16 keeps the sign, the 8 exponent bits and the top 7
 * fraction bits of the FP32 encoding, so rounding acts on the low 16 bits.
 * NaN stays NaN (quietened); overflow past the largest finite bfloat16 gives
 * infinity, as round-to-nearest requires.
 */
float oracle_bf16_rne(float x)
{
    uint32_t u;
    memcpy(&u, &x, sizeof u);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu) != 0) {
        u = (u | 0x00400000u) & 0xFFFF0000u;
    } else {
        uint32_t low = u & 0xFFFFu;
        uint32_t high = u & 0xFFFF0000u;
        uint32_t lsb = (u >> 16) & 1u;
        if (low > 0x8000u || (low == 0x8000u && lsb))
            high += 0x10000u;
        u = high;
    }
    float y;
    memcpy(&y, &u, sizeof y);
    return y;
}

void oracle_bf16_rne_array(const float *in, float *out, size_t n)
{
    for (size_t t = 0; t < n; ++t)
        out[t] = oracle_bf16_rne(in[t]);
}

/*
 * Matrix product, the definition written out: each element of C is the sum
 * over k of the products along row i of A and column j of B, accumulated in
 * FP64 in increasing k.
 */
int oracle_gemm(int M, int N, int K, const double *a, int lda, const double *b, int ldb, double *c, int ldc)
{
    if (M < 0 || N < 0 || K < 0 || lda < K || ldb < N || ldc < N)
        return -1;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j) {
            double sum = 0.0;
            for (int k = 0; k < K; ++k)
                sum += a[(size_t)i * lda + k] * b[(size_t)k * ldb + j];
            c[(size_t)i * ldc + j] = sum;
        }
    return 0;
}
