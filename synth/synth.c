/*
 * Seeded synthetic inputs for the all-pairs shortest-path solver and its
 * tests.  Holds none of the shortest-path arithmetic: it only draws graphs.
 *
 * Every value is a pure function of (seed, graph index g, i, j), so any
 * entry can be regenerated on its own and the result does not depend on the
 * thread count.  The draw is splitmix64 applied twice:
 *
 *   key = splitmix64(seed XOR g * 0x9E3779B97F4A7C15)
 *   x   = splitmix64(key XOR (i << 32 | j))
 *
 * splitmix64 is the finaliser published by Steele, Lea and Flood
 * ("Fast splittable pseudorandom number generators", OOPSLA 2014).
 *
 * An ordered pair i != j carries an edge iff lo32(x) < floor(p * 2^32).
 * Integer weights: lo + ((hi32(x) * (hi - lo + 1)) >> 32), uniform on [lo, hi].
 * Float weights:   a + (b - a) * u, u = (hi32(x) >> 8) * 2^-24, computed in
 *                  double and rounded once to float.
 * The diagonal is 0; an absent edge is written as the caller's sentinel.
 */
#include <stdint.h>
#include <math.h>

static inline uint64_t smix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

static inline uint64_t graph_key(uint64_t seed, uint64_t g) {
    return smix(seed ^ (g * 0x9E3779B97F4A7C15ULL));
}

static inline uint64_t draw(uint64_t key, uint64_t i, uint64_t j) {
    return smix(key ^ ((i << 32) | (j & 0xFFFFFFFFULL)));
}

static inline uint64_t edge_threshold(double p) {
    if (p <= 0.0) return 0;
    if (p >= 1.0) return 1ULL << 32;
    return (uint64_t)floor(p * 4294967296.0);
}

uint64_t synth_draw(uint64_t seed, uint64_t g, uint64_t i, uint64_t j) {
    return draw(graph_key(seed, g), i, j);
}

/* Dense int32 weight matrix, row-major with leading dimension ld. */
void synth_graph_i32(int32_t *out, int64_t n, int64_t ld, uint64_t seed,
                     uint64_t g, double p, int32_t lo, int32_t hi,
                     int32_t absent) {
    const uint64_t key = graph_key(seed, g);
    const uint64_t thr = edge_threshold(p);
    const uint64_t span = (uint64_t)((int64_t)hi - (int64_t)lo + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int32_t *row = out + i * ld;
        for (int64_t j = 0; j < n; ++j) {
            if (i == j) { row[j] = 0; continue; }
            uint64_t x = draw(key, (uint64_t)i, (uint64_t)j);
            if ((x & 0xFFFFFFFFULL) < thr)
                row[j] = (int32_t)((int64_t)lo + (int64_t)(((x >> 32) * span) >> 32));
            else
                row[j] = absent;
        }
    }
}

/* Dense float32 weight matrix; absent edges are +infinity. */
void synth_graph_f32(float *out, int64_t n, int64_t ld, uint64_t seed,
                     uint64_t g, double p, double a, double b) {
    const uint64_t key = graph_key(seed, g);
    const uint64_t thr = edge_threshold(p);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        float *row = out + i * ld;
        for (int64_t j = 0; j < n; ++j) {
            if (i == j) { row[j] = 0.0f; continue; }
            uint64_t x = draw(key, (uint64_t)i, (uint64_t)j);
            if ((x & 0xFFFFFFFFULL) < thr) {
                double u = (double)((x >> 32) >> 8) * (1.0 / 16777216.0);
                row[j] = (float)(a + (b - a) * u);
            } else {
                row[j] = INFINITY;
            }
        }
    }
}

/* count integers uniform on [lo, hi]: entry t uses draw(seed, g, 0xFFFFFFFF, t). */
void synth_uniform_int(int64_t *out, int64_t count, uint64_t seed, uint64_t g,
                       int64_t lo, int64_t hi) {
    const uint64_t key = graph_key(seed, g);
    const uint64_t span = (uint64_t)(hi - lo + 1);
    for (int64_t t = 0; t < count; ++t) {
        uint64_t x = draw(key, 0xFFFFFFFFULL, (uint64_t)t);
        out[t] = lo + (int64_t)(((x >> 32) * span) >> 32);
    }
}

/* Standard normal float32 values by the Box-Muller transform; entry t uses
 * draw(seed, g, i, j) with (i, j) = (t / ncols, t % ncols) of an n x ncols grid.
 * u1 in (0, 1] from the high 24 bits of hi32, u2 in [0, 1) from lo32's top 24. */
void synth_normal_f32(float *out, int64_t rows, int64_t cols, int64_t ld,
                      uint64_t seed, uint64_t g) {
    const uint64_t key = graph_key(seed, g);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; ++i) {
        for (int64_t j = 0; j < cols; ++j) {
            uint64_t x = draw(key, (uint64_t)i, (uint64_t)j);
            double u1 = ((double)((x >> 40) & 0xFFFFFF) + 1.0) * (1.0 / 16777216.0);
            double u2 = (double)((x >> 8) & 0xFFFFFF) * (1.0 / 16777216.0);
            out[i * ld + j] = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
        }
    }
}
