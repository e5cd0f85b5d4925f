/*
 * Seeded synthetic inputs for AFMM workloads; see afmm_gen.h.
 * Pure functions of (seed, stream, index): OpenMP only splits rows, so the
 * output does not depend on the thread count.
 */
#include "afmm_gen.h"

#include <math.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream)
{
    return mix64((seed ^ (stream << 32)) + GOLDEN);
}

static inline uint64_t draw_k(uint64_t key, uint64_t idx)
{
    return mix64(key + (idx + 1) * GOLDEN);
}

uint64_t afmm_gen_draw(uint64_t seed, uint64_t stream, uint64_t idx)
{
    return draw_k(stream_key(seed, stream), idx);
}

static inline uint32_t mask_threshold(double density)
{
    if (!(density > 0.0)) return 0;
    if (density >= 1.0) return 1u << 24;
    return (uint32_t)llround(density * 16777216.0);
}

static inline int keep(uint64_t h, uint32_t thr)
{
    return (uint32_t)(h >> 40) < thr;
}

/* Uniform double in (0, 1]. */
static inline double u53_open0(uint64_t h)
{
    return ((double)(h >> 11) + 1.0) * 0x1p-53;
}

/* Uniform double in [0, 1). */
static inline double u53(uint64_t h)
{
    return (double)(h >> 11) * 0x1p-53;
}

void afmm_gen_real(float *out, int64_t nrows, int64_t ncols, int64_t row0,
                   uint64_t seed, uint64_t stream_mask, uint64_t stream_val,
                   double density, int dist)
{
    const uint64_t km = stream_key(seed, stream_mask);
    const uint64_t kv = stream_key(seed, stream_val);
    const uint64_t kv2 = stream_key(seed, stream_val ^ 0x100);
    const uint32_t thr = mask_threshold(density);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        float *o = out + r * ncols;
        const uint64_t base = (uint64_t)(row0 + r) * (uint64_t)ncols;
        for (int64_t c = 0; c < ncols; ++c) {
            const uint64_t idx = base + (uint64_t)c;
            if (!keep(draw_k(km, idx), thr)) {
                o[c] = 0.0f;
                continue;
            }
            const uint64_t h = draw_k(kv, idx);
            float v;
            switch (dist) {
            case AFMM_GEN_UNIFORM01:
                v = (float)((double)(h >> 40) * 0x1p-24);
                break;
            case AFMM_GEN_UNIFORMPM1:
                v = (float)((double)(h >> 40) * 0x1p-23 - 1.0);
                break;
            default: { /* AFMM_GEN_NORMAL */
                const double u1 = u53_open0(h);
                const double u2 = u53(draw_k(kv2, idx));
                v = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
                break;
            }
            }
            o[c] = v;
        }
    }
}

static int32_t poisson_inv(double u, double lambda)
{
    double p = exp(-lambda), F = p;
    int32_t k = 0;
    while (u >= F && k < 100000) {
        ++k;
        p = p * lambda / (double)k;
        F += p;
        if (p == 0.0) break;
    }
    return k;
}

void afmm_gen_int(int32_t *out, int64_t nrows, int64_t ncols, int64_t row0,
                  uint64_t seed, uint64_t stream_mask, uint64_t stream_val,
                  double density, int dist, double a, double b,
                  int32_t clip_lo, int32_t clip_hi)
{
    const uint64_t km = stream_key(seed, stream_mask);
    const uint64_t kv = stream_key(seed, stream_val);
    const uint32_t thr = mask_threshold(density);
    const int64_t ia = (int64_t)a, ib = (int64_t)b;
    const uint64_t span = (uint64_t)(ib - ia + 1);
    const double lq = log1p(-a);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int32_t *o = out + r * ncols;
        const uint64_t base = (uint64_t)(row0 + r) * (uint64_t)ncols;
        for (int64_t c = 0; c < ncols; ++c) {
            const uint64_t idx = base + (uint64_t)c;
            if (!keep(draw_k(km, idx), thr)) {
                o[c] = 0;
                continue;
            }
            const uint64_t h = draw_k(kv, idx);
            int64_t v;
            switch (dist) {
            case AFMM_GEN_INT_UNIFORM:
                v = ia + (int64_t)(((h >> 32) * span) >> 32);
                break;
            case AFMM_GEN_INT_POISSON:
                v = poisson_inv(u53(h), a);
                break;
            default: /* AFMM_GEN_INT_GEOMETRIC */
                v = (int64_t)floor(log(u53_open0(h)) / lq);
                break;
            }
            if (v < clip_lo) v = clip_lo;
            if (v > clip_hi) v = clip_hi;
            o[c] = (int32_t)v;
        }
    }
}
