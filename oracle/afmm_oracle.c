/*
 * CPU oracle for AFMM -- TEST INFRASTRUCTURE ONLY (see afmm_oracle.h).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (x86-64 SSE, where every
 * float operation rounds to binary32/binary64 as written).  Each function
 * cites the part of the paper it follows.
 */
#include "afmm_oracle.h"

#include <stdlib.h>
#include <string.h>
#include <xmmintrin.h>

/* Denormals must be kept (reading R8): MXCSR FTZ (bit 15) and DAZ (bit 6). */
static int fpenv_ok(void)
{
    return (_mm_getcsr() & 0x8040u) == 0;
}

static inline int64_t row_of(const int64_t *rows, int64_t t)
{
    return rows ? rows[t] : t;
}

/*
 * Case A (Section 2): X real, Y integer.  Every element starts at +0.0 and,
 * for k ascending, receives the real entry X[i,k] added to it Y[k,j] times,
 * one binary32 addition after another, straight into the element; a zero
 * X[i,k] contributes nothing (readings R1, R3-R7; separate extents m, kd, n,
 * reading R9).  Rows of Z are computed one after another.
 */
uint64_t afmm_oracle_caseA_f32_ex(int64_t m, int64_t kd, int64_t n, const float *X, int64_t ldx,
                                  const int32_t *Y, int64_t ldy, float *Z, int64_t ldz,
                                  const int64_t *rows, int64_t nrows, int x_rows_only)
{
    if (!fpenv_ok()) return UINT64_MAX;
    if (!rows) nrows = m;
    uint64_t adds = 0;
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = row_of(rows, t);
        const float *xrow = X + (x_rows_only ? t : i) * ldx;
        float *zrow = Z + t * ldz;
        for (int64_t j = 0; j < n; ++j) zrow[j] = 0.0f;
        for (int64_t k = 0; k < kd; ++k) {
            const float x = xrow[k];
            if (x == 0.0f) continue;                               /* adds nothing */
            const int32_t *yrow = Y + k * ldy;
            for (int64_t j = 0; j < n; ++j) {
                const int32_t times = yrow[j];                     /* <= 0: none */
                for (int32_t p = 0; p < times; ++p) {
                    zrow[j] = zrow[j] + x;                         /* one addition */
                    ++adds;
                }
            }
        }
    }
    return adds;
}

uint64_t afmm_oracle_caseA_f32(int64_t n, const float *X, const int32_t *Y,
                               float *Z, const int64_t *rows, int64_t nrows,
                               int x_rows_only)
{
    return afmm_oracle_caseA_f32_ex(n, n, n, X, n, Y, n, Z, n, rows, nrows, x_rows_only);
}

/*
 * Case B (Section 2): X integer, Y real.  Every element starts at +0.0 and,
 * for k ascending, receives the real entry Y[k,j] added to it X[i,k] times,
 * one binary32 addition after another; a zero Y[k,j] contributes nothing to
 * that element only (reading R2), and a count <= 0 nothing at all (reading
 * R5), which is why the count is tested once per k.
 */
uint64_t afmm_oracle_caseB_f32_ex(int64_t m, int64_t kd, int64_t n, const int32_t *X, int64_t ldx,
                                  const float *Y, int64_t ldy, float *Z, int64_t ldz,
                                  const int64_t *rows, int64_t nrows, int x_rows_only)
{
    if (!fpenv_ok()) return UINT64_MAX;
    if (!rows) nrows = m;
    uint64_t adds = 0;
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = row_of(rows, t);
        const int32_t *xrow = X + (x_rows_only ? t : i) * ldx;
        float *zrow = Z + t * ldz;
        for (int64_t j = 0; j < n; ++j) zrow[j] = 0.0f;
        for (int64_t k = 0; k < kd; ++k) {
            const int32_t times = xrow[k];
            if (times <= 0) continue;
            const float *yrow = Y + k * ldy;
            for (int64_t j = 0; j < n; ++j) {
                const float y = yrow[j];
                if (y == 0.0f) continue;                           /* this element only */
                for (int32_t p = 0; p < times; ++p) {
                    zrow[j] = zrow[j] + y;                         /* one addition */
                    ++adds;
                }
            }
        }
    }
    return adds;
}

uint64_t afmm_oracle_caseB_f32(int64_t n, const int32_t *X, const float *Y,
                               float *Z, const int64_t *rows, int64_t nrows,
                               int x_rows_only)
{
    return afmm_oracle_caseB_f32_ex(n, n, n, X, n, Y, n, Z, n, rows, nrows, x_rows_only);
}

/*
 * The product the method computes (abstract; Section 2.1, point 1):
 * Z[i,j] = sum_k X[i,k] * Y[k,j], here in binary64 with k ascending.  Every
 * term is exact in binary64 (a binary32 times an integer below 2^29).
 */
void afmm_oracle_product_f64_ex(int case_id, int64_t m, int64_t kd, int64_t n, const void *X,
                                int64_t ldx, const void *Y, int64_t ldy, double *Z, int64_t ldz,
                                const int64_t *rows, int64_t nrows, int x_rows_only)
{
    if (!rows) nrows = m;
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = row_of(rows, t);
        const int64_t xr = (x_rows_only ? t : i) * ldx;
        double *zrow = Z + t * ldz;
        for (int64_t j = 0; j < n; ++j) zrow[j] = 0.0;
        for (int64_t k = 0; k < kd; ++k) {
            double x;
            if (case_id == 0) x = (double)((const float *)X)[xr + k];
            else x = (double)((const int32_t *)X)[xr + k];
            if (x == 0.0) continue;
            if (case_id == 0) {
                const int32_t *yrow = (const int32_t *)Y + k * ldy;
                for (int64_t j = 0; j < n; ++j) zrow[j] += x * (double)yrow[j];
            } else {
                const float *yrow = (const float *)Y + k * ldy;
                for (int64_t j = 0; j < n; ++j) zrow[j] += x * (double)yrow[j];
            }
        }
    }
}

void afmm_oracle_product_f64(int case_id, int64_t n, const void *X, const void *Y,
                             double *Z, const int64_t *rows, int64_t nrows,
                             int x_rows_only)
{
    afmm_oracle_product_f64_ex(case_id, n, n, n, X, n, Y, n, Z, n, rows, nrows, x_rows_only);
}

typedef unsigned __int128 u128;

static uint64_t sat64(u128 v, unsigned *flags)
{
    if (v > (u128)UINT64_MAX) {
        *flags |= AFMM_ORACLE_OVERFLOW;
        return UINT64_MAX;
    }
    return (uint64_t)v;
}

static void int_flags(int32_t v, unsigned *flags)
{
    if (v < 0) *flags |= AFMM_ORACLE_NEGATIVE;
    if (v > 255) *flags |= AFMM_ORACLE_ABOVE255;
    if (v > 256) *flags |= AFMM_ORACLE_ABOVE256;
}

/*
 * Addition count (Section 2.2).  The paper's estimate n * (n^2 d1) * mu
 * counts, for each non-zero of the Base factor, the Rep-factors it is
 * repeated by; summing that count exactly over the matrix gives, per row i,
 *   case A: r_i = sum_k [X[i,k] != 0] * sum_j max(Y[k,j], 0)
 *   case B: r_i = sum_k max(X[i,k], 0) * #{j : Y[k,j] != 0}
 * and the total is sum_i r_i (i < m, k < kd, j < n).
 */
unsigned afmm_oracle_count_ex(int case_id, int64_t m, int64_t kd, int64_t n, const void *X,
                              int64_t ldx, const void *Y, int64_t ldy, uint64_t *total,
                              uint64_t *row_counts)
{
    unsigned flags = 0;
    /* wk[k]: weight of the post-factor's row k (its positive sum in case A,
     * its number of non-zeros in case B); at most n * 2^31 < 2^64. */
    uint64_t *wk = (uint64_t *)malloc((size_t)(kd > 0 ? kd : 1) * sizeof(uint64_t));
    if (!wk) return AFMM_ORACLE_OVERFLOW;
    for (int64_t k = 0; k < kd; ++k) {
        u128 s = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (case_id == 0) {
                const int32_t v = ((const int32_t *)Y)[k * ldy + j];
                int_flags(v, &flags);
                if (v > 0) s += (u128)v;
            } else {
                const float v = ((const float *)Y)[k * ldy + j];
                if (v != 0.0f) s += 1;
            }
        }
        wk[k] = (uint64_t)s;
    }
    u128 tot = 0;
    for (int64_t i = 0; i < m; ++i) {
        u128 r = 0;
        for (int64_t k = 0; k < kd; ++k) {
            if (case_id == 0) {
                const float x = ((const float *)X)[i * ldx + k];
                if (x != 0.0f) r += (u128)wk[k];
            } else {
                const int32_t x = ((const int32_t *)X)[i * ldx + k];
                int_flags(x, &flags);
                if (x > 0) r += (u128)(uint64_t)x * (u128)wk[k];
            }
        }
        if (row_counts) row_counts[i] = sat64(r, &flags);
        tot += r;
    }
    *total = sat64(tot, &flags);
    free(wk);
    if (!fpenv_ok()) flags |= AFMM_ORACLE_FPENV;
    return flags;
}

unsigned afmm_oracle_count(int case_id, int64_t n, const void *X, const void *Y,
                           uint64_t *total, uint64_t *row_counts)
{
    return afmm_oracle_count_ex(case_id, n, n, n, X, n, Y, n, total, row_counts);
}

/* Round-to-nearest-even of a binary32 to its upper 16 bits (bfloat16). */
static uint16_t bf16_rne(float x)
{
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu))
        return (uint16_t)((b >> 16) | 0x0040u); /* NaN stays NaN */
    const uint32_t low = b & 0xFFFFu;
    uint32_t up = b >> 16;
    if (low > 0x8000u || (low == 0x8000u && (up & 1u))) up += 1; /* carries into the exponent */
    return (uint16_t)up;
}

static float bf16_to_f32(uint16_t h)
{
    const uint32_t b = (uint32_t)h << 16;
    float f;
    memcpy(&f, &b, 4);
    return f;
}

void afmm_oracle_split_bf16x3(int64_t count, const float *x, uint16_t *hi,
                              uint16_t *mid, uint16_t *lo)
{
    for (int64_t t = 0; t < count; ++t) {
        const float v = x[t];
        const uint16_t h = bf16_rne(v);
        const float r1 = v - bf16_to_f32(h);
        const uint16_t m = bf16_rne(r1);
        const float r2 = r1 - bf16_to_f32(m);
        hi[t] = h;
        mid[t] = m;
        lo[t] = bf16_rne(r2);
    }
}
