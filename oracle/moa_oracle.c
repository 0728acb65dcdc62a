/*
 * moa_oracle.c -- plain CPU reference for the MoA matrix product.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The product path
 * (the HIP library) shares no code, header or table with it.
 *
 * What it computes (paper, section "MoA Matrix Multiplication", Eq. 1-3):
 *   rho A = <m, n>, rho B = <n, p>, rho C = <m, p>, all row-major and
 *   contiguous, and for 0 <= i < m, 0 <= j < p:
 *       C[i*p + j] := sum_{k=0}^{n-1} A[i*n + k] * B[k*p + j]
 *
 * Evaluation order (paper, section "From Normal Form to C Program"): the
 * generic C program walks row i of C; for each k in ascending order it adds
 * the scalar A[i,k] times the contiguous row k of B into row i of C. That is
 * the scalar-vector decomposition of Fig. 1. Every element C[i,j] therefore
 * receives sum_k in ascending k, which is also what the textbook row-column
 * dot product computes, operation for operation.
 *
 * The paper's program adds into C (C = C + ...), while Eq. 3 assigns (:=).
 * Both are offered: accumulate == 0 starts each row from +0.0 (Eq. 3);
 * accumulate != 0 starts from the C the caller passes in (the C program).
 *
 * Splitting the row loop over threads is the paper's dimension lifting of i
 * over processors (section "Dimension Lifting to Machine Coordinates"); it
 * does not change any element's operation sequence, so results do not depend
 * on the thread count.
 *
 * Build with -ffp-contract=off and without -ffast-math: each product is
 * rounded to the working precision before it is added. The *_fma variants
 * instead use one fused multiply-add per step (same order); they model a
 * kernel that contracts multiply and add, for bitwise comparisons.
 *
 * Sizes are int64_t; an empty dimension is valid (n == 0 gives the empty
 * sum, so C := 0, or C unchanged when accumulating).
 */
#include <math.h>
#include <stdint.h>

#define ORACLE_ROW_LOOP _Pragma("omp parallel for schedule(dynamic, 1)")

/* Eq. 3 in FP64, product rounded, then added. */
void moa_oracle_gemm_f64(int64_t m, int64_t n, int64_t p,
                         const double *A, const double *B, double *C,
                         int accumulate)
{
    ORACLE_ROW_LOOP
    for (int64_t i = 0; i < m; ++i) {
        double *c_row = C + i * p;
        if (!accumulate)
            for (int64_t j = 0; j < p; ++j)
                c_row[j] = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            const double a = A[i * n + k];
            const double *b_row = B + k * p;
            for (int64_t j = 0; j < p; ++j) {
                const double prod = a * b_row[j];
                c_row[j] = c_row[j] + prod;
            }
        }
    }
}

/* Eq. 3 in FP64, same order, one fused multiply-add per step. */
void moa_oracle_gemm_f64_fma(int64_t m, int64_t n, int64_t p,
                             const double *A, const double *B, double *C,
                             int accumulate)
{
    ORACLE_ROW_LOOP
    for (int64_t i = 0; i < m; ++i) {
        double *c_row = C + i * p;
        if (!accumulate)
            for (int64_t j = 0; j < p; ++j)
                c_row[j] = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            const double a = A[i * n + k];
            const double *b_row = B + k * p;
            for (int64_t j = 0; j < p; ++j)
                c_row[j] = fma(a, b_row[j], c_row[j]);
        }
    }
}

/* Eq. 3 in FP32, same order, one fused multiply-add per step. This is the
 * exact operation sequence of an FP32 kernel that keeps k ascending for
 * every element and contracts multiply and add. */
void moa_oracle_gemm_f32_fma(int64_t m, int64_t n, int64_t p,
                             const float *A, const float *B, float *C,
                             int accumulate)
{
    ORACLE_ROW_LOOP
    for (int64_t i = 0; i < m; ++i) {
        float *c_row = C + i * p;
        if (!accumulate)
            for (int64_t j = 0; j < p; ++j)
                c_row[j] = 0.0f;
        for (int64_t k = 0; k < n; ++k) {
            const float a = A[i * n + k];
            const float *b_row = B + k * p;
            for (int64_t j = 0; j < p; ++j)
                c_row[j] = fmaf(a, b_row[j], c_row[j]);
        }
    }
}

/* Normwise relative error in FP64: ||X - R||_F / ||R||_F, with both sums
 * taken in ascending index order. Returns sqrt(sum (X-R)^2) when R == 0. */
double moa_oracle_rel_err_f64(int64_t count, const double *X, const double *R)
{
    double num = 0.0, den = 0.0;
    for (int64_t t = 0; t < count; ++t) {
        const double d = X[t] - R[t];
        num += d * d;
        den += R[t] * R[t];
    }
    if (den == 0.0)
        return sqrt(num);
    return sqrt(num) / sqrt(den);
}
