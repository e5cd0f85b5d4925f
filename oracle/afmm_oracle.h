/*
 * CPU oracle for AFMM -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded C that spells out what the AFMM method
 * computes (Singh, Chakraborty, Mallick, "An Adaptable Fast Matrix
 * Multiplication (AFMM) Algorithm", arXiv 1308.2400).  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never does, and the two share no code.
 *
 * Matrices are dense, row-major, 0-based (Section 2 recommends the plain
 * two-dimensional array).  X is the pre-factor, Y the post-factor.  The
 * paper's matrices are n x n; the _ex forms take X as m x kd with leading
 * dimension ldx, Y as kd x n with ldy and Z as m x n with ldz (element (r, c)
 * of X at X[r * ldx + c]), and the square forms are m = kd = n with every
 * leading dimension n.
 *   Case A: X real (float), Y integer (int32)   -- Section 2, Case-A loop.
 *   Case B: X integer (int32), Y real (float)   -- Section 2, Case-B loop.
 *
 * Readings of the paper this oracle takes (the paper is silent, garbled or
 * self-contradictory on these points):
 *  R1  The inner sum's upper bound is the Rep-factor of the current (i,k,j)
 *      (Y[k,j] in case A, X[i,k] in case B), not the printed floor(mu): the
 *      loop assigns Rep-factor and the correctness argument of Section 2.1
 *      processes the base Y[K,J] times.
 *  R2  Case B's zero-base test skips only the current (k,j) (continues the
 *      j loop); skipping the rest of row k would not give the product that
 *      Section 2.1 claims.
 *  R3  Each addition goes straight into Z[i,j] (Z = Z + Base, Rep-factor
 *      times, in the order i, k, j, p), not into a separately formed sum.
 *  R4  Loops run 0..n-1 ascending.
 *  R5  A non-positive Rep-factor performs no additions (the empty sum).
 *  R6  "EQUALS 0" is IEEE equality, so -0.0 is skipped as well.
 *  R7  An "addition" is one execution of Z = Z + Base (Section 2.2); tests,
 *      comparisons and index arithmetic are not counted.
 *  R8  Floating point is IEEE binary32 (binary64 for the true product),
 *      round to nearest even, denormals kept, no contraction.
 *  R9  Rectangular shapes run the same loops with the I, K and J bounds
 *      taken separately (m, kd, n): the product of an m x kd and a kd x n
 *      matrix, which is what the loops compute once their bounds differ.
 */
#ifndef AFMM_ORACLE_H
#define AFMM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Flag bits reported by afmm_oracle_count. */
#define AFMM_ORACLE_NEGATIVE   1u  /* an integer entry is < 0                 */
#define AFMM_ORACLE_ABOVE255   2u  /* an integer entry is > 255               */
#define AFMM_ORACLE_ABOVE256   4u  /* an integer entry is > 256               */
#define AFMM_ORACLE_OVERFLOW   8u  /* the add count does not fit in 64 bits   */
#define AFMM_ORACLE_FPENV     16u  /* the CPU flushes denormals: results void */

/*
 * Strict FP32, case A, the paper's loop order.  Computes the rows listed in
 * `rows` (nrows of them; rows == NULL means all n rows in order) into
 * Z[t * n + j] for the t-th listed row.  With x_rows_only set, the t-th
 * listed row of X is read from X[t * n + k] (callers may pass only the
 * sampled rows of X); otherwise X is the full matrix.  Returns the number of
 * additions performed, or UINT64_MAX when the FPU flushes denormals.
 */
uint64_t afmm_oracle_caseA_f32(int64_t n, const float *X, const int32_t *Y,
                               float *Z, const int64_t *rows, int64_t nrows,
                               int x_rows_only);

/* Strict FP32, case B, the paper's loop order; same conventions. */
uint64_t afmm_oracle_caseB_f32(int64_t n, const int32_t *X, const float *Y,
                               float *Z, const int64_t *rows, int64_t nrows,
                               int x_rows_only);

/*
 * Rectangular forms of the two strict loops (reading R9): rows == NULL means
 * all m rows; the t-th listed row goes to Z[t * ldz + j]; with x_rows_only
 * the t-th listed row of X is read from X[t * ldx + k].
 */
uint64_t afmm_oracle_caseA_f32_ex(int64_t m, int64_t kd, int64_t n, const float *X, int64_t ldx,
                                  const int32_t *Y, int64_t ldy, float *Z, int64_t ldz,
                                  const int64_t *rows, int64_t nrows, int x_rows_only);
uint64_t afmm_oracle_caseB_f32_ex(int64_t m, int64_t kd, int64_t n, const int32_t *X, int64_t ldx,
                                  const float *Y, int64_t ldy, float *Z, int64_t ldz,
                                  const int64_t *rows, int64_t nrows, int x_rows_only);

/*
 * True product Z = X . Y in binary64, k ascending, for the listed rows
 * (rows == NULL: all), case_id 0 = A (X float, Y int32), 1 = B (X int32,
 * Y float).  With x_rows_only the t-th listed row of X is X[t * n + k].
 */
void afmm_oracle_product_f64(int case_id, int64_t n, const void *X, const void *Y,
                             double *Z, const int64_t *rows, int64_t nrows,
                             int x_rows_only);
void afmm_oracle_product_f64_ex(int case_id, int64_t m, int64_t kd, int64_t n, const void *X,
                                int64_t ldx, const void *Y, int64_t ldy, double *Z, int64_t ldz,
                                const int64_t *rows, int64_t nrows, int x_rows_only);

/*
 * Number of additions the algorithm performs, from its definition summed in
 * closed form (Section 2.2): for case A, each non-zero X[i,k] is added
 * max(Y[k,j],0) times for every j, so the count is
 *     sum_k nnz(X[:,k]) * sum_j max(Y[k,j],0);
 * for case B, X[i,k] repetitions of every non-zero Y[k,j]:
 *     sum_k sum_i max(X[i,k],0) * nnz(Y[k,:]).
 * Writes the total (saturated at 2^64-1) and, when row_counts is non-NULL,
 * the count of each row i of Z.  Returns the flag bits above.
 */
unsigned afmm_oracle_count(int case_id, int64_t n, const void *X, const void *Y,
                           uint64_t *total, uint64_t *row_counts);
/* Rectangular form (reading R9): m rows of Z, kd, n; row_counts has m entries. */
unsigned afmm_oracle_count_ex(int case_id, int64_t m, int64_t kd, int64_t n, const void *X,
                              int64_t ldx, const void *Y, int64_t ldy, uint64_t *total,
                              uint64_t *row_counts);

/*
 * Split of binary32 values into three bfloat16 terms, each the round-to-
 * nearest-even bfloat16 of what the previous terms leave:
 *     hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid),
 * with both differences exact in binary32.  Outputs are bfloat16 bit
 * patterns.  Used to pin the split-precision form.
 */
void afmm_oracle_split_bf16x3(int64_t count, const float *x, uint16_t *hi,
                              uint16_t *mid, uint16_t *lo);

#ifdef __cplusplus
}
#endif

#endif
