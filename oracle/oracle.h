/*
 * oracle.h -- declarations of the FP64 CPU reference (test infrastructure only;
 * never included by the product library).
 *
 * All arrays are I*J*K doubles, linear index i + I*(j + J*k). co[] holds the
 * twelve read-only arrays in the order a0 a1 a2 a3 b0 b1 b2 c0 c1 c2 bnd wrk1.
 * Functions return 0 on success, -1 on bad arguments (a dimension below 3, a
 * NULL pointer, iters < 0) and -2 when memory runs out.
 */
#ifndef ORACLE_H
#define ORACLE_H

#include <stddef.h>

#define ORACLE_NCOEF 12

#ifdef __cplusplus
extern "C" {
#endif

/* One sweep (nest S) plus the residual of the old iterate: writes wrk2 on the
 * interior only, p unchanged; *gosa = sum of ss^2 (gosa may be NULL). */
int oracle_sweep(int I, int J, int K, const double *const co[ORACLE_NCOEF], const double *p, double omega,
                 double *wrk2, double *gosa);

/* Residual of the current iterate: *gosa = sum over the interior of ss(p)^2. */
int oracle_residual(int I, int J, int K, const double *const co[ORACLE_NCOEF], const double *p, double *gosa);

/* iters x (sweep, residual, copy-back). p is updated in place on the interior;
 * *gosa = residual of the last sweep, i.e. of p after iters-1 iterations
 * (NaN when iters == 0). */
int oracle_jacobi(int I, int J, int K, const double *const co[ORACLE_NCOEF], double *p, double omega, int iters,
                  double *gosa);

/* Host threads the loops over k use: 1 for the plain build, the OpenMP
 * thread count for a build with -fopenmp (both give bit-identical results). */
int oracle_threads(void);

/* FP32 -> nearest bfloat16 (ties to even) -> FP32. */
float oracle_bf16_rne(float x);
void oracle_bf16_rne_array(const float *in, float *out, size_t n);

/* Matrix product C = A B in FP64 (row-major; lda, ldb, ldc are row strides in
 * elements): c[i][j] = sum over k of a[i][k] * b[k][j], summed in k order.
 * The plain definition of the matrix-product function block. Returns 0, or -1
 * for negative sizes or strides shorter than the rows. */
int oracle_gemm(int M, int N, int K, const double *a, int lda, const double *b, int ldb, double *c, int ldc);

#ifdef __cplusplus
}
#endif

#endif
