/*
 * Seeded synthetic-input generator (native part).
 *
 * Holds none of the aggregate-evaluation arithmetic: it only draws random
 * columns from a counter-based generator and sorts key tuples, so that the
 * CPU oracle and the GPU engine consume byte-identical relations.
 *
 * Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) used in counter mode.  Draw i of a stream
 * with 64-bit key K is mix64(K + (i + 1) * GAMMA), where mix64 is the
 * SplitMix64 output finaliser and GAMMA the golden-ratio increment.  A
 * uniform double in [0,1) keeps the top 53 bits.  Normal draws use the
 * Box-Muller transform on draws 2i and 2i+1.  Discrete draws from a table
 * (bounded Zipf) invert a cumulative table supplied by the caller.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define DG_GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t draw_u64(uint64_t key, int64_t i) {
    return mix64(key + (uint64_t)(i + 1) * DG_GAMMA);
}

static inline double draw_unit(uint64_t key, int64_t i) {
    return (double)(draw_u64(key, i) >> 11) * 0x1.0p-53;
}

/* FNV-1a over the name, then mixed with the seed. */
uint64_t dg_stream_key(uint64_t seed, const char *name) {
    uint64_t h = 0xcbf29ce484222325ULL;
    for (const unsigned char *p = (const unsigned char *)name; *p; ++p) {
        h ^= *p;
        h *= 0x100000001b3ULL;
    }
    return mix64(mix64(seed * DG_GAMMA + 1ULL) ^ h);
}

void dg_fill_u64(uint64_t key, int64_t n, uint64_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = draw_u64(key, i);
}

void dg_fill_unit_f64(uint64_t key, int64_t n, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = draw_unit(key, i);
}

/* x = lo + (hi - lo) * u, computed in double and rounded to fp32. */
void dg_fill_uniform_f32(uint64_t key, int64_t n, double lo, double hi, float *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = (float)(lo + (hi - lo) * draw_unit(key, i));
}

/* Box-Muller: z = sqrt(-2 ln(1 - u1)) * cos(2 pi u2), u1 = draw 2i, u2 = draw 2i+1. */
void dg_fill_normal_f32(uint64_t key, int64_t n, double mean, double sd, float *out) {
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double u1 = draw_unit(key, 2 * i);
        double u2 = draw_unit(key, 2 * i + 1);
        double z = sqrt(-2.0 * log(1.0 - u1)) * cos(two_pi * u2);
        out[i] = (float)(mean + sd * z);
    }
}

/* Same draw as dg_fill_normal_f32 but kept in double (thresholds are drawn
 * this way, then rounded by the caller). */
void dg_fill_normal_f64(uint64_t key, int64_t n, double mean, double sd, double *out) {
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t i = 0; i < n; ++i) {
        double u1 = draw_unit(key, 2 * i);
        double u2 = draw_unit(key, 2 * i + 1);
        out[i] = mean + sd * sqrt(-2.0 * log(1.0 - u1)) * cos(two_pi * u2);
    }
}

/* Uniform integer in [lo, hi): lo + floor(u * (hi - lo)). */
void dg_fill_uniform_i32(uint64_t key, int64_t n, int32_t lo, int32_t hi, int32_t *out) {
    const double span = (double)hi - (double)lo;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = (int64_t)floor(draw_unit(key, i) * span);
        if (v >= (int64_t)(hi - lo)) v = hi - lo - 1;
        out[i] = lo + (int32_t)v;
    }
}

/* Inverse-CDF draw: out[i] = smallest k with u < cdf[k] (cdf ascending, cdf[m-1] >= 1). */
void dg_fill_from_cdf_i32(uint64_t key, int64_t n, const double *cdf, int32_t m, int32_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double u = draw_unit(key, i);
        int32_t lo = 0, hi = m - 1;
        while (lo < hi) {
            int32_t mid = lo + (hi - lo) / 2;
            if (u < cdf[mid]) hi = mid; else lo = mid + 1;
        }
        out[i] = lo;
    }
}

/* ---- sorting of key tuples ------------------------------------------- */

/* LSD radix sort of 64-bit unsigned values, 11-bit digits, parallel
 * histogram and scatter.  Digits that are constant across the array are
 * skipped.  Uses a scratch buffer of n elements. */
int dg_sort_u64(uint64_t *a, int64_t n) {
    if (n <= 1) return 0;
    uint64_t *tmp = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    if (!tmp) return -1;
    const int BITS = 11, NB = 1 << 11;
    uint64_t orv = 0, andv = ~0ULL;
    for (int64_t i = 0; i < n; ++i) { orv |= a[i]; andv &= a[i]; }
    const uint64_t varying = orv ^ andv;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    int64_t *hist = (int64_t *)malloc((size_t)nthreads * NB * sizeof(int64_t));
    if (!hist) { free(tmp); return -1; }
    uint64_t *src = a, *dst = tmp;
    for (int shift = 0; shift < 64; shift += BITS) {
        uint64_t mask = (uint64_t)(NB - 1) << shift;
        if ((varying & mask) == 0) continue;
        memset(hist, 0, (size_t)nthreads * NB * sizeof(int64_t));
#pragma omp parallel num_threads(nthreads)
        {
            int t = 0, nt = 1;
#ifdef _OPENMP
            t = omp_get_thread_num(); nt = omp_get_num_threads();
#endif
            int64_t b = n * t / nt, e = n * (t + 1) / nt;
            int64_t *h = hist + (size_t)t * NB;
            for (int64_t i = b; i < e; ++i) h[(src[i] >> shift) & (NB - 1)]++;
#pragma omp barrier
#pragma omp single
            {
                int64_t run = 0;
                for (int d = 0; d < NB; ++d)
                    for (int tt = 0; tt < nt; ++tt) {
                        int64_t c = hist[(size_t)tt * NB + d];
                        hist[(size_t)tt * NB + d] = run;
                        run += c;
                    }
            }
            for (int64_t i = b; i < e; ++i) {
                uint64_t v = src[i];
                dst[h[(v >> shift) & (NB - 1)]++] = v;
            }
        }
        uint64_t *sw = src; src = dst; dst = sw;
    }
    if (src != a) memcpy(a, src, (size_t)n * sizeof(uint64_t));
    free(hist);
    free(tmp);
    return 0;
}

/* Mixed-radix composition of nk key columns (most significant first). */
void dg_compose(int64_t n, int nk, const int32_t *const *cols, const int64_t *radix, uint64_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t v = 0;
        for (int k = 0; k < nk; ++k) v = v * (uint64_t)radix[k] + (uint64_t)cols[k][i];
        out[i] = v;
    }
}

void dg_decompose(int64_t n, int nk, const uint64_t *in, const int64_t *radix, int32_t *const *cols) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t v = in[i];
        for (int k = nk - 1; k >= 0; --k) {
            cols[k][i] = (int32_t)(v % (uint64_t)radix[k]);
            v /= (uint64_t)radix[k];
        }
    }
}
