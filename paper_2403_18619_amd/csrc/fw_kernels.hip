// Blocked Floyd-Warshall kernels for gfx950 (MI355X).
//
// A solve runs R = ceil(n / BS) rounds (Section 2.3, "Blocked FW").  Round K
// owns the band of vertices [K*BS, K*BS + bk), bk = min(BS, n - K*BS):
//   phase 1  closes the diagonal block (K,K) in place, one k at a time;
//   phase 2  updates the row band (K,*) and the column band (*,K) -- the
//            paper's phases 2 and 3 -- against the closed diagonal block;
//   phase 3  updates every remaining element -- the paper's phase 4, nearly
//            all of the O(n^3) work -- by the min-plus product of the column
//            band (*,K) and the row band (K,*).
//
// Phases 2 and 3 are one kernel, "C <- min(C, A (x) B)" over the bk k's of the
// band, taking A and B as they were when the kernel started:
//   row band    : C = D[band][J],  A = D[band][band] (closed), B = old C
//   column band : C = D[I][band],  A = old C,  B = D[band][band] (closed)
//   remainder   : C = D[I][J],     A = D[I][band],  B = D[band][J]
// For the bands this "product form" gives the same distances as the paper's
// in-place k loop: a path from the band to J splits at its last vertex in the
// band, a path from I to the band at its first one.
//
// Successor matrix: when C[i][j] strictly improves, NX[i][j] takes the
// successor of the A operand's entry, NX[i][K*BS + k*], where k* is the first
// k (in increasing order) that reaches the new minimum.  With a strict
// comparison that choice is the same in every schedule and tile order.
//
// Arithmetic: int32 distances run as uint32 (INF = 2^30, INF + INF = 2^31
// does not wrap); float32 as IEEE single.  Every relaxation is a single
// rounded add, so the k order does not change any distance.
#include "fw_internal.h"

namespace fw {
namespace {

constexpr int KC = 32;            // k-chunk staged in LDS per step
constexpr int LDP = kTile + 4;    // LDS row pitch (elements), keeps 16-byte alignment
constexpr uint32_t kInfU = 1u << 30;

__host__ __device__ __forceinline__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }

template <typename U> struct Arith;
template <> struct Arith<uint32_t> {
    using V4 = uint4;
    static __device__ __forceinline__ uint32_t inf() { return kInfU; }
    static __device__ __forceinline__ uint32_t mn(uint32_t a, uint32_t b) { return min(a, b); }
};
template <> struct Arith<float> {
    using V4 = float4;
    static __device__ __forceinline__ float inf() { return __builtin_inff(); }
    static __device__ __forceinline__ float mn(float a, float b) { return __builtin_fminf(a, b); }
};

// ------------------------------------------------------------------ init
// Normalise the input in place: diagonal 0, int32 entries >= 2^30 (or < 0)
// become INF, float -0 becomes +0 and NaN +inf; NX gets its first state
// (i on the diagonal, j for an edge, -1 for none).  Validate mode records a
// negative or NaN weight in the device error word.
__device__ __forceinline__ uint32_t norm_weight(uint32_t v, bool diag, bool &bad) {
    const int32_t s = (int32_t)v;
    bad = !diag && s < 0;
    if (diag) return 0u;
    return (s < 0 || s >= (int32_t)kInfU) ? kInfU : v;
}
__device__ __forceinline__ float norm_weight(float v, bool diag, bool &bad) {
    bad = !diag && (v < 0.0f || v != v);
    if (diag) return 0.0f;
    if (v != v) return __builtin_inff();
    return v == 0.0f ? 0.0f : v;
}

template <typename U>
__global__ __launch_bounds__(256) void init_kernel(U *__restrict__ D, int32_t *__restrict__ NX,
                                                   int64_t n, int64_t ld, int validate,
                                                   int *__restrict__ err) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    bool any_bad = false;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        const int64_t o = i * ld + j;
        bool bad;
        const U w = norm_weight(D[o], i == j, bad);
        any_bad |= bad;
        D[o] = w;
        if (NX) NX[o] = (i == j) ? (int32_t)i : (w < Arith<U>::inf() ? (int32_t)j : -1);
    }
    if (validate && any_bad) atomicCAS(err, 0, 1);
}

// --------------------------------------------------------------- phase 1
// Closure of the diagonal block in place (the paper's phase 1), one
// workgroup.  Each thread keeps an M x M patch of the block in registers;
// at step k only row k and column k are read, and they do not change during
// step k (D[k][k] = 0, strict test), so the owners publish them into a
// double-buffered LDS row / column and one barrier per step suffices.
template <typename U, bool NEXT, int BS>
__global__ __launch_bounds__(256) void phase1_kernel(U *__restrict__ D, int32_t *__restrict__ NX,
                                                     int64_t n, int64_t ld, int K) {
    constexpr int M = BS / 16;
    __shared__ U rowb[2][BS];
    __shared__ U colb[2][BS];
    __shared__ int32_t nxb[2][BS];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t b0 = (int64_t)K * BS;
    const int bk = (int)imin64((int64_t)BS, n - b0);

    U d[M][M];
    int32_t nx[M][M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const int li = ty * M + r, lj = tx * M + c;
            if (li < bk && lj < bk) {
                const int64_t o = (b0 + li) * ld + b0 + lj;
                d[r][c] = D[o];
                nx[r][c] = NEXT ? NX[o] : 0;
            } else {
                d[r][c] = (li == lj) ? U(0) : Arith<U>::inf();
                nx[r][c] = -1;
            }
        }
    }
    if (ty == 0) {
#pragma unroll
        for (int c = 0; c < M; ++c) rowb[0][tx * M + c] = d[0][c];
    }
    if (tx == 0) {
#pragma unroll
        for (int r = 0; r < M; ++r) {
            colb[0][ty * M + r] = d[r][0];
            if (NEXT) nxb[0][ty * M + r] = nx[r][0];
        }
    }
    __syncthreads();

    for (int kb = 0; kb * M < bk; ++kb) {
#pragma unroll
        for (int r0 = 0; r0 < M; ++r0) {
            const int k = kb * M + r0;
            if (k < bk) {                       // uniform across the workgroup
                const int cur = k & 1;
                U a[M], b[M];
                int32_t na[M];
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    a[r] = colb[cur][ty * M + r];
                    if (NEXT) na[r] = nxb[cur][ty * M + r];
                }
#pragma unroll
                for (int c = 0; c < M; ++c) b[c] = rowb[cur][tx * M + c];
#pragma unroll
                for (int r = 0; r < M; ++r) {
#pragma unroll
                    for (int c = 0; c < M; ++c) {
                        const U s = a[r] + b[c];
                        const bool lt = s < d[r][c];
                        d[r][c] = lt ? s : d[r][c];
                        if (NEXT) nx[r][c] = lt ? na[r] : nx[r][c];
                    }
                }
                // publish row / column k+1 for the next step
                const int r1 = (r0 + 1 == M) ? 0 : r0 + 1;
                const int kb1 = (r0 + 1 == M) ? kb + 1 : kb;
                if (k + 1 < bk) {
                    if (ty == kb1) {
#pragma unroll
                        for (int c = 0; c < M; ++c) rowb[cur ^ 1][tx * M + c] = d[r1][c];
                    }
                    if (tx == kb1) {
#pragma unroll
                        for (int r = 0; r < M; ++r) {
                            colb[cur ^ 1][ty * M + r] = d[r][r1];
                            if (NEXT) nxb[cur ^ 1][ty * M + r] = nx[r][r1];
                        }
                    }
                }
                __syncthreads();
            }
        }
    }

#pragma unroll
    for (int r = 0; r < M; ++r) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const int li = ty * M + r, lj = tx * M + c;
            if (li < bk && lj < bk) {
                const int64_t o = (b0 + li) * ld + b0 + lj;
                D[o] = d[r][c];
                if (NEXT) NX[o] = nx[r][c];
            }
        }
    }
}

// ---------------------------------------------------- phases 2 and 3
// Thread (tx, ty) of the 16 x 16 grid owns an 8 x 8 patch of the 128 x 128
// output tile: rows ty*4 + {0..3} and 64 + ty*4 + {0..3}, columns likewise
// with tx, so that every LDS read of four consecutive entries is one 16-byte
// access and a wave's global row accesses are 256 contiguous bytes.
__device__ __forceinline__ int patch_off(int q, int r) { return (r < 4) ? q * 4 + r : 64 + q * 4 + (r - 4); }

template <typename U>
__device__ __forceinline__ void load_row4(const U *__restrict__ p, int64_t col, int lim_valid,
                                          bool vec, U out[4]) {
    // entries p[col .. col+3]; entry e exists iff (local index + e) < lim_valid,
    // where col's local index is folded into lim_valid by the caller.
    if (vec && lim_valid >= 4) {
        const typename Arith<U>::V4 v = *reinterpret_cast<const typename Arith<U>::V4 *>(p + col);
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) out[e] = (e < lim_valid) ? p[col + e] : Arith<U>::inf();
    }
}

template <typename U, bool NEXT>
__global__ __launch_bounds__(256, 2) void minplus_kernel(U *__restrict__ D, int32_t *__restrict__ NX,
                                                         int64_t n, int64_t ld, int K, int BS,
                                                         int phase, int nt, int vec) {
    __shared__ __attribute__((aligned(16))) U As[KC][LDP];   // As[k][i] = A[i][k]
    __shared__ __attribute__((aligned(16))) U Bs[KC][LDP];   // Bs[k][j] = B[k][j]

    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t b0 = (int64_t)K * BS;
    const int bk = (int)imin64((int64_t)BS, n - b0);
    const int64_t b1 = b0 + bk;

    int mode;             // 0 remainder, 1 row band, 2 column band
    int64_t row0, col0;
    if (phase == 3) {
        const int64_t tiles = (int64_t)nt * nt;
        // Workgroups are dealt to the eight XCDs round-robin; give each XCD a
        // contiguous run of tiles so that tiles sharing a row of A meet in
        // the same L2.
        const int64_t per = (tiles + 7) / 8;
        const int64_t tid = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
        if (tid >= tiles) return;
        row0 = (tid / nt) * kTile;
        col0 = (tid % nt) * kTile;
        if (row0 >= b0 && imin64(row0 + kTile, n) <= b1) return;   // all rows in the band
        if (col0 >= b0 && imin64(col0 + kTile, n) <= b1) return;   // all columns in the band
        mode = 0;
    } else if (blockIdx.y == 0) {
        mode = 1;
        row0 = b0;
        col0 = (int64_t)blockIdx.x * kTile;
        if (col0 >= b0 && imin64(col0 + kTile, n) <= b1) return;
    } else {
        mode = 2;
        row0 = (int64_t)blockIdx.x * kTile;
        col0 = b0;
        if (row0 >= b0 && imin64(row0 + kTile, n) <= b1) return;
    }
    // number of valid rows / columns of C (and of A's rows, B's columns)
    const int rows_valid = (mode == 1) ? bk : (int)imin64(kTile, n - row0);
    const int cols_valid = (mode == 2) ? bk : (int)imin64(kTile, n - col0);
    const bool use_vec = vec != 0;

    // ---- load C
    U acc[8][8];
    int32_t idx[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int li = patch_off(ty, r);
        const bool rv = li < rows_valid;
        const U *rowp = D + (row0 + (rv ? li : 0)) * ld + col0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int lj = h * 64 + tx * 4;
            U v[4];
            if (rv) {
                load_row4(rowp, lj, cols_valid - lj, use_vec, v);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = Arith<U>::inf();
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc[r][h * 4 + e] = v[e];
                idx[r][h * 4 + e] = -1;
            }
        }
    }

    // ---- k loop: stage KC k's of A and B in LDS, then relax
    const int a_il = t >> 1, a_kq = (t & 1) * 16;     // A staging: row, first k
    const int b_kk = t >> 3, b_jq = (t & 7) * 16;     // B staging: k, first column
    for (int kc = 0; kc < bk; kc += KC) {
        if (kc) __syncthreads();
        {   // A: As[kk][il] = D[row0 + il][b0 + kc + kk]
            const bool rv = a_il < rows_valid;
            const U *p = D + (row0 + (rv ? a_il : 0)) * ld + b0 + kc;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int kk = a_kq + q * 4;
                U v[4];
                if (rv) {
                    load_row4(p, kk, bk - kc - kk, use_vec, v);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = Arith<U>::inf();
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) As[kk + e][a_il] = v[e];
            }
        }
        {   // B: Bs[kk][jl] = D[b0 + kc + kk][col0 + jl]
            const bool kv = kc + b_kk < bk;
            const U *p = D + (b0 + kc + (kv ? b_kk : 0)) * ld + col0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int jl = b_jq + q * 4;
                U v[4];
                if (kv) {
                    load_row4(p, jl, cols_valid - jl, use_vec, v);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = Arith<U>::inf();
                }
                typename Arith<U>::V4 w;
                w.x = v[0]; w.y = v[1]; w.z = v[2]; w.w = v[3];
                *reinterpret_cast<typename Arith<U>::V4 *>(&Bs[b_kk][jl]) = w;
            }
        }
        __syncthreads();

        if (NEXT) {
#pragma unroll 2
            for (int kk = 0; kk < KC; ++kk) {
                U a[8], b[8];
                const typename Arith<U>::V4 a0 = *reinterpret_cast<const typename Arith<U>::V4 *>(&As[kk][ty * 4]);
                const typename Arith<U>::V4 a1 = *reinterpret_cast<const typename Arith<U>::V4 *>(&As[kk][64 + ty * 4]);
                const typename Arith<U>::V4 c0 = *reinterpret_cast<const typename Arith<U>::V4 *>(&Bs[kk][tx * 4]);
                const typename Arith<U>::V4 c1 = *reinterpret_cast<const typename Arith<U>::V4 *>(&Bs[kk][64 + tx * 4]);
                a[0] = a0.x; a[1] = a0.y; a[2] = a0.z; a[3] = a0.w;
                a[4] = a1.x; a[5] = a1.y; a[6] = a1.z; a[7] = a1.w;
                b[0] = c0.x; b[1] = c0.y; b[2] = c0.z; b[3] = c0.w;
                b[4] = c1.x; b[5] = c1.y; b[6] = c1.z; b[7] = c1.w;
                const int kg = kc + kk;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const U s = a[r] + b[c];
                        const bool lt = s < acc[r][c];
                        acc[r][c] = lt ? s : acc[r][c];
                        idx[r][c] = lt ? kg : idx[r][c];
                    }
                }
            }
        } else {
#pragma unroll 1
            for (int kk = 0; kk < KC; kk += 2) {
                U a[8], b[8], a2[8], b2[8];
                const typename Arith<U>::V4 a0 = *reinterpret_cast<const typename Arith<U>::V4 *>(&As[kk][ty * 4]);
                const typename Arith<U>::V4 a1 = *reinterpret_cast<const typename Arith<U>::V4 *>(&As[kk][64 + ty * 4]);
                const typename Arith<U>::V4 c0 = *reinterpret_cast<const typename Arith<U>::V4 *>(&Bs[kk][tx * 4]);
                const typename Arith<U>::V4 c1 = *reinterpret_cast<const typename Arith<U>::V4 *>(&Bs[kk][64 + tx * 4]);
                const typename Arith<U>::V4 e0 = *reinterpret_cast<const typename Arith<U>::V4 *>(&As[kk + 1][ty * 4]);
                const typename Arith<U>::V4 e1 = *reinterpret_cast<const typename Arith<U>::V4 *>(&As[kk + 1][64 + ty * 4]);
                const typename Arith<U>::V4 f0 = *reinterpret_cast<const typename Arith<U>::V4 *>(&Bs[kk + 1][tx * 4]);
                const typename Arith<U>::V4 f1 = *reinterpret_cast<const typename Arith<U>::V4 *>(&Bs[kk + 1][64 + tx * 4]);
                a[0] = a0.x; a[1] = a0.y; a[2] = a0.z; a[3] = a0.w;
                a[4] = a1.x; a[5] = a1.y; a[6] = a1.z; a[7] = a1.w;
                b[0] = c0.x; b[1] = c0.y; b[2] = c0.z; b[3] = c0.w;
                b[4] = c1.x; b[5] = c1.y; b[6] = c1.z; b[7] = c1.w;
                a2[0] = e0.x; a2[1] = e0.y; a2[2] = e0.z; a2[3] = e0.w;
                a2[4] = e1.x; a2[5] = e1.y; a2[6] = e1.z; a2[7] = e1.w;
                b2[0] = f0.x; b2[1] = f0.y; b2[2] = f0.z; b2[3] = f0.w;
                b2[4] = f1.x; b2[5] = f1.y; b2[6] = f1.z; b2[7] = f1.w;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        acc[r][c] = Arith<U>::mn(acc[r][c], Arith<U>::mn(a[r] + b[c], a2[r] + b2[c]));
                    }
                }
            }
        }
    }

    // ---- successor gather (reads A's NX before anything is written: for the
    // column band A is C itself)
    if (NEXT) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int li = patch_off(ty, r);
            const int32_t *nrow = NX + (row0 + (li < rows_valid ? li : 0)) * ld + b0;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (idx[r][c] >= 0) idx[r][c] = nrow[idx[r][c]];
            }
        }
        __syncthreads();
    }

    // ---- store (rows / columns of the band itself are not part of phase 3)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int li = patch_off(ty, r);
        const int64_t gi = row0 + li;
        bool rs = li < rows_valid;
        if (mode != 1) rs = rs && !(gi >= b0 && gi < b1);
        if (!rs) continue;
        U *drow = D + gi * ld + col0;
        int32_t *nrow = NEXT ? NX + gi * ld + col0 : nullptr;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int lj = h * 64 + tx * 4;
            bool cs[4];
            bool all = true;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gj = col0 + lj + e;
                cs[e] = (lj + e) < cols_valid && (mode == 2 || !(gj >= b0 && gj < b1));
                all = all && cs[e];
            }
            if (NEXT) {
                // Only improved entries change.  After the gather idx holds the
                // successor of an improved entry (>= 0: its A entry is finite)
                // and -1 elsewhere.
                bool ch[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) ch[e] = cs[e] && idx[r][h * 4 + e] >= 0;
                if (use_vec && all) {
                    if (ch[0] || ch[1] || ch[2] || ch[3]) {
                        typename Arith<U>::V4 w;
                        w.x = acc[r][h * 4 + 0]; w.y = acc[r][h * 4 + 1];
                        w.z = acc[r][h * 4 + 2]; w.w = acc[r][h * 4 + 3];
                        *reinterpret_cast<typename Arith<U>::V4 *>(drow + lj) = w;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (ch[e]) drow[lj + e] = acc[r][h * 4 + e];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (ch[e]) nrow[lj + e] = idx[r][h * 4 + e];
            } else {
                if (use_vec && all) {
                    typename Arith<U>::V4 w;
                    w.x = acc[r][h * 4 + 0]; w.y = acc[r][h * 4 + 1];
                    w.z = acc[r][h * 4 + 2]; w.w = acc[r][h * 4 + 3];
                    *reinterpret_cast<typename Arith<U>::V4 *>(drow + lj) = w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (cs[e]) drow[lj + e] = acc[r][h * 4 + e];
                }
            }
        }
    }
}

template <typename U>
hipError_t init_t(const Plan &p) {
    dim3 grid((unsigned)((p.n + 255) / 256), (unsigned)imin64(p.n, 65535));
    hipLaunchKernelGGL(init_kernel<U>, grid, dim3(256), 0, p.stream, (U *)p.dist, p.next, p.n, p.ld,
                       p.validate ? 1 : 0, p.work->err);
    return hipGetLastError();
}

template <typename U, bool NEXT>
hipError_t phase1_t(const Plan &p, int K) {
    switch (p.bs) {
    case 32: hipLaunchKernelGGL((phase1_kernel<U, NEXT, 32>), dim3(1), dim3(256), 0, p.stream, (U *)p.dist, p.next, p.n, p.ld, K); break;
    case 64: hipLaunchKernelGGL((phase1_kernel<U, NEXT, 64>), dim3(1), dim3(256), 0, p.stream, (U *)p.dist, p.next, p.n, p.ld, K); break;
    case 128: hipLaunchKernelGGL((phase1_kernel<U, NEXT, 128>), dim3(1), dim3(256), 0, p.stream, (U *)p.dist, p.next, p.n, p.ld, K); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename U, bool NEXT>
hipError_t minplus_t(const Plan &p, int K, int phase) {
    dim3 grid;
    if (phase == 2) {
        grid = dim3((unsigned)p.nt, 2);
    } else {
        const int64_t tiles = (int64_t)p.nt * p.nt;
        grid = dim3((unsigned)(8 * ((tiles + 7) / 8)));
    }
    hipLaunchKernelGGL((minplus_kernel<U, NEXT>), grid, dim3(256), 0, p.stream, (U *)p.dist, p.next,
                       p.n, p.ld, K, p.bs, phase, p.nt, p.vec ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init(const Plan &p) {
    return p.dtype == DType::I32 ? init_t<uint32_t>(p) : init_t<float>(p);
}

hipError_t launch_phase1(const Plan &p, int K) {
    if (p.dtype == DType::I32) return p.next ? phase1_t<uint32_t, true>(p, K) : phase1_t<uint32_t, false>(p, K);
    return p.next ? phase1_t<float, true>(p, K) : phase1_t<float, false>(p, K);
}

hipError_t launch_phase2(const Plan &p, int K) {
    if (p.dtype == DType::I32) return p.next ? minplus_t<uint32_t, true>(p, K, 2) : minplus_t<uint32_t, false>(p, K, 2);
    return p.next ? minplus_t<float, true>(p, K, 2) : minplus_t<float, false>(p, K, 2);
}

hipError_t launch_phase3(const Plan &p, int K) {
    if (p.dtype == DType::I32) return p.next ? minplus_t<uint32_t, true>(p, K, 3) : minplus_t<uint32_t, false>(p, K, 3);
    return p.next ? minplus_t<float, true>(p, K, 3) : minplus_t<float, false>(p, K, 3);
}

}  // namespace fw
