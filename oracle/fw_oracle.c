/*
 * CPU oracle for all-pairs shortest paths.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may call anything in this directory.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * What it computes (Floyd-Warshall, Section 2.3 and Fig. 1 of Calderon, Rucci
 * and Chichizola, "Enhanced OpenMP Algorithm to Compute All-Pairs Shortest
 * Path on x86 Architectures"): given a dense n x n distance matrix D whose
 * entry (i, j) is the weight of edge i -> j, or "infinite" when there is no
 * edge, step k (k = 0 .. n-1, in order) tries every pair (i, j) through the
 * intermediate vertex k and keeps D[i][k] + D[k][j] when it is shorter.  After
 * step n-1, D[i][j] is the length of a shortest walk from i to j.
 *
 * Readings of the paper used here (each listed in the design notes):
 *  - Fig. 1 writes the test as ">="; this oracle uses the strict "<", which
 *    leaves every distance unchanged and keeps the path matrix free of
 *    self-references on ties.
 *  - The paper's path matrix P stores the last intermediate k; this oracle
 *    keeps the successor ("next hop") instead: NX[i][j] is the vertex after i
 *    on the chosen path, NX[i][i] = i, NX[i][j] = -1 when j is unreachable.
 *    The update that goes with "D[i][j] <- D[i][k] + D[k][j]" is
 *    "NX[i][j] <- NX[i][k]".
 *  - "Infinite" (the footnote of Section 2.3: the largest positive value) is
 *    2^30 for int32 weights (inputs at or above it are absent) and +inf for
 *    floating point weights.
 *  - The diagonal is forced to 0 (self-loops are ignored); negative weights
 *    are rejected (return -1).
 *
 * Parity status: pinned.  Distances are checked against brute-force path
 * enumeration, Dijkstra from every source, a library shortest-path routine
 * and closed forms; the next-hop matrix against path walks and, on graphs with
 * unique shortest paths, against the Dijkstra shortest-path tree.
 *
 * The outer k loop is sequential.  Within one step the loop over i may run on
 * several threads: at step k, row k and column k do not change (D[k][k] = 0
 * and the test is strict), so every (i, j) update reads only values that are
 * fixed during that step and the result does not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>
#include <omp.h>

#define ORACLE_INF_I32 1073741824   /* 2^30 */

static void set_threads(int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

/* ------------------------------------------------------------------ FW, int32 */
int oracle_fw_i32(const int32_t *W, int64_t n, int64_t ldw,
                  int32_t *D, int32_t *NX, int64_t ld, int nthreads) {
    set_threads(nthreads);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            if (W[i * ldw + j] < 0 && i != j) return -1;
    /* initial state: the input matrix, diagonal 0, absent = INF */
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            int32_t w = W[i * ldw + j];
            int32_t d = (i == j) ? 0 : (w >= ORACLE_INF_I32 ? ORACLE_INF_I32 : w);
            D[i * ld + j] = d;
            if (NX) NX[i * ld + j] = (i == j) ? (int32_t)i : (d < ORACLE_INF_I32 ? (int32_t)j : -1);
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        const int32_t *Dk = D + k * ld;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int32_t *Di = D + i * ld;
            const int64_t dik = Di[k];
            if (dik >= ORACLE_INF_I32) continue;   /* INF + anything is never shorter */
            int32_t *Ni = NX ? NX + i * ld : NULL;
            const int32_t nik = Ni ? Ni[k] : 0;
            for (int64_t j = 0; j < n; ++j) {
                int64_t s = dik + (int64_t)Dk[j];
                if (s < (int64_t)Di[j]) {
                    Di[j] = (int32_t)s;
                    if (Ni) Ni[j] = nik;
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------ FW, float64 */
/* Float weights arrive as float64 (float32 inputs convert exactly); every sum
 * is one float64 addition. */
int oracle_fw_f64(const double *W, int64_t n, int64_t ldw,
                  double *D, int32_t *NX, int64_t ld, int nthreads) {
    set_threads(nthreads);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double w = W[i * ldw + j];
            if (i != j && (w < 0.0 || isnan(w))) return -1;
        }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double d = (i == j) ? 0.0 : W[i * ldw + j];
            D[i * ld + j] = d;
            if (NX) NX[i * ld + j] = (i == j) ? (int32_t)i : (isinf(d) ? -1 : (int32_t)j);
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        const double *Dk = D + k * ld;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double *Di = D + i * ld;
            const double dik = Di[k];
            if (isinf(dik)) continue;
            int32_t *Ni = NX ? NX + i * ld : NULL;
            const int32_t nik = Ni ? Ni[k] : 0;
            for (int64_t j = 0; j < n; ++j) {
                double s = dik + Dk[j];
                if (s < Di[j]) {
                    Di[j] = s;
                    if (Ni) Ni[j] = nik;
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------ FW, float32 */
/* The same steps with every sum rounded to float32 (the paper's "float"
 * data type); used where a float32-precision decision is wanted. */
int oracle_fw_f32(const float *W, int64_t n, int64_t ldw,
                  float *D, int32_t *NX, int64_t ld, int nthreads) {
    set_threads(nthreads);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            float w = W[i * ldw + j];
            if (i != j && (w < 0.0f || isnan(w))) return -1;
        }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            float d = (i == j) ? 0.0f : W[i * ldw + j];
            D[i * ld + j] = d;
            if (NX) NX[i * ld + j] = (i == j) ? (int32_t)i : (isinf(d) ? -1 : (int32_t)j);
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        const float *Dk = D + k * ld;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            float *Di = D + i * ld;
            const float dik = Di[k];
            if (isinf(dik)) continue;
            int32_t *Ni = NX ? NX + i * ld : NULL;
            const int32_t nik = Ni ? Ni[k] : 0;
            for (int64_t j = 0; j < n; ++j) {
                float s = dik + Dk[j];
                if (s < Di[j]) {
                    Di[j] = s;
                    if (Ni) Ni[j] = nik;
                }
            }
        }
    }
    return 0;
}

/* --------------------------------------------- single source (Dijkstra) */
/* One row of the distance matrix by Dijkstra's algorithm (dense O(n^2)
 * form): the row of sources srcs[t] goes to out + t * n.  Weights are int32
 * with absent >= 2^30; unreachable entries are 2^30.  Sums in int64. */
void oracle_sssp_i32(const int32_t *W, int64_t n, int64_t ldw,
                     const int64_t *srcs, int64_t nsrc, int32_t *out, int nthreads) {
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nsrc; ++t) {
        int64_t *dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        unsigned char *done = (unsigned char *)calloc((size_t)n, 1);
        const int64_t inf = INT64_MAX;
        for (int64_t v = 0; v < n; ++v) dist[v] = inf;
        dist[srcs[t]] = 0;
        for (int64_t it = 0; it < n; ++it) {
            int64_t u = -1, best = inf;
            for (int64_t v = 0; v < n; ++v)
                if (!done[v] && dist[v] < best) { best = dist[v]; u = v; }
            if (u < 0) break;
            done[u] = 1;
            const int32_t *Wu = W + u * ldw;
            for (int64_t v = 0; v < n; ++v) {
                if (done[v] || v == u) continue;
                int32_t w = Wu[v];
                if (w >= ORACLE_INF_I32) continue;
                if (best + w < dist[v]) dist[v] = best + w;
            }
        }
        for (int64_t v = 0; v < n; ++v)
            out[t * n + v] = dist[v] == inf ? ORACLE_INF_I32 : (int32_t)dist[v];
        free(dist);
        free(done);
    }
}

/* Dijkstra on float32 weights (absent = +inf), sums in float64. */
void oracle_sssp_f64(const float *W, int64_t n, int64_t ldw,
                     const int64_t *srcs, int64_t nsrc, double *out, int nthreads) {
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nsrc; ++t) {
        double *dist = out + t * n;
        unsigned char *done = (unsigned char *)calloc((size_t)n, 1);
        for (int64_t v = 0; v < n; ++v) dist[v] = INFINITY;
        dist[srcs[t]] = 0.0;
        for (int64_t it = 0; it < n; ++it) {
            int64_t u = -1;
            double best = INFINITY;
            for (int64_t v = 0; v < n; ++v)
                if (!done[v] && dist[v] < best) { best = dist[v]; u = v; }
            if (u < 0) break;
            done[u] = 1;
            const float *Wu = W + u * ldw;
            for (int64_t v = 0; v < n; ++v) {
                if (done[v] || v == u) continue;
                double w = (double)Wu[v];
                if (isinf(w)) continue;
                if (best + w < dist[v]) dist[v] = best + w;
            }
        }
        free(done);
    }
}
