/*
 * synth.c -- seeded synthetic inputs for the SpMV library and its oracle.
 *
 * This file holds input generation only: it draws coordinate-format (triplet) matrices,
 * their values and dense x vectors.  None of the SpMV method's arithmetic lives here, so
 * the oracle and the GPU path may both take their inputs from it.
 *
 * Randomness: every draw is a pure function of (seed, stream, counter), so the output does
 * not depend on the thread count.  The mixer is SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014): the i-th output of a SplitMix64
 * sequence whose state starts at s is mix(s + (i + 1) * GOLDEN), which is what draw() returns.
 *
 * Streams: 0 = structure (row/col), 1 = values, 2 = x, 3 = relabelling permutation keys.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Starting state of the SplitMix64 sequence for (seed, stream). */
static inline uint64_t stream_state(uint64_t seed, uint64_t stream) {
    return sm64_mix(seed * GOLDEN + sm64_mix(stream + 0x632BE59BD9B4E019ULL));
}

static inline uint64_t draw(uint64_t state, uint64_t ctr) {
    return sm64_mix(state + (ctr + 1) * GOLDEN);
}

/* 53-bit uniform in [0, 1). */
static inline double unit_double(uint64_t u) { return (double)(u >> 11) * 0x1.0p-53; }

uint64_t synth_draw(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return draw(stream_state(seed, stream), ctr);
}

/*
 * R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): each of the E edges descends `scale`
 * levels of the 2x2 quadrant recursion, most significant bit first.  At each level a 32-bit
 * uniform u picks top-left when u < a, top-right when u < a+b, bottom-left when u < a+b+c,
 * bottom-right otherwise.  No noise, no relabelling, self-loops and repeats kept.
 * Thresholds are fixed-point (probability * 2^32, rounded) so the choice is exact integer work.
 */
void synth_rmat(int scale, int64_t E, double a, double b, double c, uint64_t seed,
                int32_t* row, int32_t* col) {
    const uint64_t st = stream_state(seed, 0);
    const uint64_t tA = (uint64_t)llround(a * 4294967296.0);
    const uint64_t tAB = (uint64_t)llround((a + b) * 4294967296.0);
    const uint64_t tABC = (uint64_t)llround((a + b + c) * 4294967296.0);
    const int per_edge = (scale + 1) / 2; /* two 32-bit uniforms per 64-bit draw */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        uint32_t r = 0, q = 0;
        for (int l = 0; l < scale; ++l) {
            uint64_t w = draw(st, (uint64_t)e * (uint64_t)per_edge + (uint64_t)(l >> 1));
            uint64_t u = (l & 1) ? (w & 0xFFFFFFFFULL) : (w >> 32);
            uint32_t rb, cb;
            if (u < tA) { rb = 0; cb = 0; }
            else if (u < tAB) { rb = 0; cb = 1; }
            else if (u < tABC) { rb = 1; cb = 0; }
            else { rb = 1; cb = 1; }
            r = (r << 1) | rb;
            q = (q << 1) | cb;
        }
        row[e] = (int32_t)r;
        col[e] = (int32_t)q;
    }
}

/*
 * Chung-Lu style power law: vertex i has weight w_i = (i+1)^(-1/(gamma-1)).  Each of the E
 * samples draws its row and its column independently with probability proportional to w,
 * by inverse CDF over the cumulative weights (summed in index order, in double precision).
 */
int synth_chunglu(int32_t n, int64_t E, double gamma, uint64_t seed, int32_t* row, int32_t* col) {
    double* cdf = (double*)malloc(sizeof(double) * (size_t)n);
    if (!cdf) return -1;
    const double expo = -1.0 / (gamma - 1.0);
    double acc = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        acc += pow((double)(i + 1), expo);
        cdf[i] = acc;
    }
    const double total = acc;
    const uint64_t st = stream_state(seed, 0);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        for (int side = 0; side < 2; ++side) {
            double t = unit_double(draw(st, 2 * (uint64_t)e + (uint64_t)side)) * total;
            int32_t lo = 0, hi = n - 1; /* first index with cdf > t */
            while (lo < hi) {
                int32_t mid = lo + (hi - lo) / 2;
                if (cdf[mid] > t) hi = mid; else lo = mid + 1;
            }
            if (side == 0) row[e] = lo; else col[e] = lo;
        }
    }
    free(cdf);
    return 0;
}

/* Erdos-Renyi style uniform sampling: E entries with row and column uniform over [0,m)x[0,n). */
void synth_uniform(int32_t m, int32_t n, int64_t E, uint64_t seed, int32_t* row, int32_t* col) {
    const uint64_t st = stream_state(seed, 0);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        uint64_t w = draw(st, (uint64_t)e);
        row[e] = (int32_t)(((w >> 32) * (uint64_t)m) >> 32);
        col[e] = (int32_t)(((w & 0xFFFFFFFFULL) * (uint64_t)n) >> 32);
    }
}

/*
 * Values for counter range [0, len) of `stream`.
 * kind 0: uniform(-1, 1) doubles; kind 1: integers uniform over {-3,...,3} stored as double.
 */
void synth_values(int64_t len, uint64_t seed, uint64_t stream, int kind, double* out) {
    const uint64_t st = stream_state(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < len; ++i) {
        uint64_t u = draw(st, (uint64_t)i);
        if (kind == 0) out[i] = unit_double(u) * 2.0 - 1.0;
        else out[i] = (double)((int64_t)(((u >> 32) * 7ULL) >> 32) - 3);
    }
}

/* Raw 64-bit draws (used for random relabelling keys). */
void synth_u64(int64_t len, uint64_t seed, uint64_t stream, uint64_t* out) {
    const uint64_t st = stream_state(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < len; ++i) out[i] = draw(st, (uint64_t)i);
}
