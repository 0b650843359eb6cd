/*
 * Result validators for all-pairs shortest paths.
 *
 * TEST INFRASTRUCTURE ONLY (see fw_oracle.c).  They check any (D, NX) pair --
 * the oracle's own or a solver's -- against the input weights W:
 *
 *  - D[i][i] == 0 and NX[i][i] == i;
 *  - D[i][j] is "infinite" exactly when NX[i][j] == -1;
 *  - otherwise the successor walk i -> NX[i][j] -> NX[NX[i][j]][j] -> ...
 *    reaches j within n - 1 hops, every hop is an edge of W, and the summed
 *    edge weights equal D[i][j] (int32: exactly; float: within rtol).
 *
 * The walk check is the definition of a valid next-hop matrix for a given
 * distance matrix: it holds for every correct answer even when several
 * shortest paths tie.
 */
#include <stdint.h>
#include <math.h>

#define VAL_INF_I32 1073741824   /* 2^30 */

/* Returns the number of bad pairs among rows[0..nrows); writes the first bad
 * (i, j) and a reason code into first_bad[0..2] (reason: 1 diagonal,
 * 2 INF/-1 mismatch, 3 walk leaves the graph or loops, 4 sum differs). */
int64_t validate_walk_i32(const int32_t *W, int64_t ldw, const int32_t *D,
                          const int32_t *NX, int64_t ld, int64_t n,
                          const int64_t *rows, int64_t nrows, int64_t *first_bad) {
    int64_t bad = 0;
    first_bad[0] = first_bad[1] = -1;
    first_bad[2] = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+:bad)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        for (int64_t j = 0; j < n; ++j) {
            const int32_t d = D[i * ld + j];
            const int32_t h0 = NX[i * ld + j];
            int reason = 0;
            if (i == j) {
                if (d != 0 || h0 != (int32_t)i) reason = 1;
            } else if (d >= VAL_INF_I32 || h0 < 0) {
                if (!(d == VAL_INF_I32 && h0 == -1)) reason = 2;
            } else {
                int64_t u = i, sum = 0, hops = 0;
                while (u != j) {
                    int32_t h = NX[u * ld + j];
                    if (h < 0 || h >= n || h == u || hops >= n - 1) { reason = 3; break; }
                    int32_t w = W[u * ldw + h];
                    if (w >= VAL_INF_I32 || w < 0) { reason = 3; break; }
                    sum += w;
                    u = h;
                    ++hops;
                }
                if (!reason && sum != (int64_t)d) reason = 4;
            }
            if (reason) {
                ++bad;
#pragma omp critical
                {
                    if (first_bad[0] < 0 || i < first_bad[0] || (i == first_bad[0] && j < first_bad[1])) {
                        first_bad[0] = i;
                        first_bad[1] = j;
                        first_bad[2] = reason;
                    }
                }
            }
        }
    }
    return bad;
}

/* Float32 weights and distances (absent = +inf); the walk sum is taken in
 * float64 and must agree with D[i][j] within rtol * max(|D|, |sum|). */
int64_t validate_walk_f32(const float *W, int64_t ldw, const float *D,
                          const int32_t *NX, int64_t ld, int64_t n,
                          const int64_t *rows, int64_t nrows, double rtol,
                          int64_t *first_bad) {
    int64_t bad = 0;
    first_bad[0] = first_bad[1] = -1;
    first_bad[2] = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+:bad)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        for (int64_t j = 0; j < n; ++j) {
            const float d = D[i * ld + j];
            const int32_t h0 = NX[i * ld + j];
            int reason = 0;
            if (i == j) {
                if (d != 0.0f || h0 != (int32_t)i) reason = 1;
            } else if (isinf(d) || h0 < 0) {
                if (!(isinf(d) && d > 0 && h0 == -1)) reason = 2;
            } else {
                int64_t u = i, hops = 0;
                double sum = 0.0;
                while (u != j) {
                    int32_t h = NX[u * ld + j];
                    if (h < 0 || h >= n || h == u || hops >= n - 1) { reason = 3; break; }
                    float w = W[u * ldw + h];
                    if (isinf(w) || isnan(w) || w < 0.0f) { reason = 3; break; }
                    sum += (double)w;
                    u = h;
                    ++hops;
                }
                if (!reason) {
                    double dd = (double)d;
                    double scale = fabs(dd) > fabs(sum) ? fabs(dd) : fabs(sum);
                    if (fabs(sum - dd) > rtol * scale) reason = 4;
                }
            }
            if (reason) {
                ++bad;
#pragma omp critical
                {
                    if (first_bad[0] < 0 || i < first_bad[0] || (i == first_bad[0] && j < first_bad[1])) {
                        first_bad[0] = i;
                        first_bad[1] = j;
                        first_bad[2] = reason;
                    }
                }
            }
        }
    }
    return bad;
}

/* float64 distances: the same checks with the walk summed in float64 and
 * compared within rtol. */
int64_t validate_walk_f64(const double *W, int64_t ldw, const double *D,
                          const int32_t *NX, int64_t ld, int64_t n,
                          const int64_t *rows, int64_t nrows, double rtol,
                          int64_t *first_bad) {
    int64_t bad = 0;
    first_bad[0] = first_bad[1] = -1;
    first_bad[2] = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+:bad)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        for (int64_t j = 0; j < n; ++j) {
            const double d = D[i * ld + j];
            const int32_t h0 = NX[i * ld + j];
            int reason = 0;
            if (i == j) {
                if (d != 0.0 || h0 != (int32_t)i) reason = 1;
            } else if (isinf(d) || h0 < 0) {
                if (!(isinf(d) && d > 0 && h0 == -1)) reason = 2;
            } else {
                int64_t u = i, hops = 0;
                double sum = 0.0;
                while (u != j) {
                    int32_t h = NX[u * ld + j];
                    if (h < 0 || h >= n || h == u || hops >= n - 1) { reason = 3; break; }
                    double w = W[u * ldw + h];
                    if (isinf(w) || isnan(w) || w < 0.0) { reason = 3; break; }
                    sum += w;
                    u = h;
                    ++hops;
                }
                if (!reason) {
                    double scale = fabs(d) > fabs(sum) ? fabs(d) : fabs(sum);
                    if (fabs(sum - d) > rtol * scale) reason = 4;
                }
            }
            if (reason) {
                ++bad;
#pragma omp critical
                {
                    if (first_bad[0] < 0 || i < first_bad[0] || (i == first_bad[0] && j < first_bad[1])) {
                        first_bad[0] = i;
                        first_bad[1] = j;
                        first_bad[2] = reason;
                    }
                }
            }
        }
    }
    return bad;
}
