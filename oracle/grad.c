/*
 * Reference gradient of the shortest-path distances -- TEST INFRASTRUCTURE
 * ONLY (see fw_oracle.c).
 *
 * A distance the solver returns is the sum of the edge weights along the path
 * its successor matrix selects, i -> NX[i][j] -> NX[NX[i][j]][j] -> ... -> j.
 * For a loss L(D) with upstream gradient G = dL/dD, the derivative with
 * respect to one edge weight W[u][v] is therefore the sum of G[i][j] over the
 * pairs (i, j), i != j, whose selected path uses the edge (u, v).  Diagonal
 * entries (always 0) and unreachable pairs (always "infinite") do not depend
 * on W and contribute nothing.
 *
 * This file computes that definition literally: it walks every path and adds
 * G[i][j] to each edge on it, in float64.  The work is the total length of all
 * selected paths.
 */
#include <stdint.h>

/* out[u * ldo + v] = sum of G[i][j] over the pairs whose walk uses (u, v).
 * Returns the number of pairs whose walk leaves [0, n) or does not reach j
 * within n - 1 hops (0 for a valid successor matrix); such a walk adds
 * nothing beyond the hops it took. */
int64_t oracle_grad_f64(const float *G, int64_t ldg, const int32_t *NX, int64_t ld, int64_t n,
                        double *out, int64_t ldo) {
    for (int64_t u = 0; u < n; ++u)
        for (int64_t v = 0; v < n; ++v) out[u * ldo + v] = 0.0;
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (i == j || NX[i * ld + j] < 0) continue;
            const double g = (double)G[i * ldg + j];
            int64_t u = i, hops = 0;
            while (u != j) {
                const int64_t h = NX[u * ld + j];
                if (h < 0 || h >= n || hops >= n - 1) {
                    ++bad;
                    break;
                }
                out[u * ldo + h] += g;
                u = h;
                ++hops;
            }
        }
    }
    return bad;
}
