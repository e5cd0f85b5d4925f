/*
 * Seeded synthetic inputs for AFMM workloads (host only).
 *
 * This module holds no arithmetic of the method itself: it only draws the
 * random matrices the paper's experiments are built on (Section 2: a real
 * factor with a given density of non-zeros and an integer factor whose
 * non-zero entries have a stated mean).  It is shared by the CPU oracle's
 * tests, the GPU parity tests and the benchmark, and by nothing else.
 *
 * Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used counter-style: the
 * idx-th draw of stream s under seed S is
 *     mix64(key(S, s) + (idx + 1) * 0x9E3779B97F4A7C15)
 * with key(S, s) = mix64(S ^ (s << 32) + 0x9E3779B97F4A7C15) and mix64 the
 * SplitMix64 finaliser.  Element (r, c) of a matrix with `ncols` columns uses
 * idx = r * ncols + c, so any subset of rows regenerates bit-identically, in
 * any thread count.
 */
#ifndef AFMM_GEN_H
#define AFMM_GEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Real-valued distributions of kept (non-masked) entries. */
enum afmm_gen_real_dist {
    AFMM_GEN_UNIFORM01 = 0,  /* (h >> 40) * 2^-24            in [0, 1), exact FP32 */
    AFMM_GEN_UNIFORMPM1 = 1, /* (h >> 40) * 2^-23 - 1        in [-1, 1), exact FP32, never -0 */
    AFMM_GEN_NORMAL = 2      /* Box-Muller in double from two streams, rounded to FP32 */
};

/* Integer-valued distributions of kept entries. */
enum afmm_gen_int_dist {
    AFMM_GEN_INT_UNIFORM = 0,  /* Uniform{a..b}, Lemire multiply-shift on the high 32 bits */
    AFMM_GEN_INT_POISSON = 1,  /* Poisson(a), inversion of the CDF in double */
    AFMM_GEN_INT_GEOMETRIC = 2 /* failures before the first success, p = a: floor(log U / log(1-p)) */
};

/* One raw 64-bit draw. */
uint64_t afmm_gen_draw(uint64_t seed, uint64_t stream, uint64_t idx);

/*
 * Fill out[(r - row0) * ncols + c] for r in [row0, row0 + nrows), c in [0, ncols).
 * An entry is kept when the 24-bit mask draw (stream_mask) is below
 * round(density * 2^24); kept entries take the value draw (stream_val, and
 * stream_val ^ 0x100 for the second Box-Muller uniform); others are +0.0f.
 */
void afmm_gen_real(float *out, int64_t nrows, int64_t ncols, int64_t row0,
                   uint64_t seed, uint64_t stream_mask, uint64_t stream_val,
                   double density, int dist);

/*
 * Integer counterpart: kept entries are drawn from `dist` with parameters
 * (a, b) and clipped to [clip_lo, clip_hi]; others are 0.
 */
void afmm_gen_int(int32_t *out, int64_t nrows, int64_t ncols, int64_t row0,
                  uint64_t seed, uint64_t stream_mask, uint64_t stream_val,
                  double density, int dist, double a, double b,
                  int32_t clip_lo, int32_t clip_hi);

#ifdef __cplusplus
}
#endif

#endif
