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
// Geometry of the 128 x 128 output tile.  Thread (tx, ty) of a TXN x 16 grid
// owns 8 rows -- ty*4 + {0..3} and 64 + ty*4 + {0..3} -- and CPT columns --
// tx*4 + {0..3}, plus 64 + tx*4 + {0..3} when CPT = 8 -- so that each LDS read
// of four consecutive entries is one 16-byte access and a wave's global row
// accesses are contiguous runs of at least 256 bytes.
template <int NT> struct Geo {
    static constexpr int threads = NT;
    static constexpr int cpt = (NT == 512) ? 4 : 8;     // columns per thread
    static constexpr int txn = kTile / cpt;             // threads along a row
    static constexpr int waves = NT / 64;
    static __device__ __forceinline__ int row_off(int ty, int r) { return (r >> 2) * 64 + ty * 4 + (r & 3); }
    static __device__ __forceinline__ int col_off(int tx, int c) { return (c >> 2) * (txn * 4) + tx * 4 + (c & 3); }
};

template <typename U>
__device__ __forceinline__ void load_row4(const U *__restrict__ p, int64_t col, int lim_valid,
                                          bool vec, U out[4]) {
    // entries p[col .. col+3]; entry e exists iff e < lim_valid (the caller
    // folds col's position within the tile into lim_valid)
    if (vec && lim_valid >= 4) {
        const typename Arith<U>::V4 v = *reinterpret_cast<const typename Arith<U>::V4 *>(p + col);
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) out[e] = (e < lim_valid) ? p[col + e] : Arith<U>::inf();
    }
}

// Operands of one k of the current chunk: a[] = A[rows of the patch][k],
// b[] = B[k][columns of the patch].
template <typename U, int NT>
__device__ __forceinline__ void lds_operands(const U (*As)[LDP], const U (*Bs)[LDP], int kk, int tx,
                                             int ty, U a[8], U b[Geo<NT>::cpt]) {
    using V4 = typename Arith<U>::V4;
    const V4 a0 = *reinterpret_cast<const V4 *>(&As[kk][ty * 4]);
    const V4 a1 = *reinterpret_cast<const V4 *>(&As[kk][64 + ty * 4]);
    a[0] = a0.x; a[1] = a0.y; a[2] = a0.z; a[3] = a0.w;
    a[4] = a1.x; a[5] = a1.y; a[6] = a1.z; a[7] = a1.w;
#pragma unroll
    for (int g = 0; g < Geo<NT>::cpt / 4; ++g) {
        const V4 c0 = *reinterpret_cast<const V4 *>(&Bs[kk][g * Geo<NT>::txn * 4 + tx * 4]);
        b[4 * g + 0] = c0.x; b[4 * g + 1] = c0.y; b[4 * g + 2] = c0.z; b[4 * g + 3] = c0.w;
    }
}

template <typename U> __device__ __forceinline__ int as_int(U v) { return __builtin_bit_cast(int, v); }
template <typename U> __device__ __forceinline__ U from_int(int v) { return __builtin_bit_cast(U, v); }

// Orders LDS traffic between lanes of one wave (the LDS executes a wave's
// accesses in issue order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Successor bookkeeping of the min-plus kernel (template argument ARGMIN):
//   0  distances only: two adds and one v_min3 per pair of k's; 256 threads,
//      8 x 8 patches.
//   1  eager reference variant: every relaxation compares, selects the
//      distance and records k (four VALU operations per relaxation).
//   2  deferred (default): 512 threads, 8 x 4 patches.  The k loop keeps the
//      distances-only form on a per-chunk minimum cm; at the end of each chunk
//      the entries with cm < acc (a strict improvement -- rare after the
//      first rounds) are appended, by wave ballot, to a per-wave queue in
//      LDS, and each lane then searches one queued entry over the chunk's
//      k's, still in LDS, for the first k with A[i][k] + B[k][j] == cm.  The
//      winning k is kept in an LDS byte matrix.
// Variants 1 and 2 select the same k: the first one, in increasing order,
// that reaches the final minimum when that minimum beats the old value.
template <typename U, int ARGMIN, int PHASE, bool VEC>
__global__ __launch_bounds__(ARGMIN == 2 ? 512 : 256, ARGMIN == 2 ? 4 : 1) void minplus_kernel(
        U *__restrict__ D, int32_t *__restrict__ NX, int64_t n, int64_t ld, int K, int BS, int nt) {
    constexpr int NT = (ARGMIN == 2) ? 512 : 256;
    using G = Geo<NT>;
    constexpr int CPT = G::cpt;
    constexpr bool NEXT = ARGMIN != 0;
    constexpr int QCAP = 128;                                      // queue entries per wave
    __shared__ __attribute__((aligned(16))) U As[KC][LDP];        // As[k][i] = A[i][k]
    __shared__ __attribute__((aligned(16))) U Bs[KC][LDP];        // Bs[k][j] = B[k][j]
    __shared__ uint32_t kst[ARGMIN == 2 ? kTile * kTile / 4 : 1]; // improving k per entry (bytes)
    __shared__ uint32_t qpos[ARGMIN == 2 ? G::waves * QCAP : 1];  // queued entry: i | j << 8
    __shared__ U qval[ARGMIN == 2 ? G::waves * QCAP : 1];         // its chunk minimum
    __shared__ int qmin[ARGMIN == 2 ? G::waves * 64 : 1];         // per-entry search result

    const int t = threadIdx.x, tx = t % G::txn, ty = t / G::txn;
    const int64_t b0 = (int64_t)K * BS;
    const int bk = (int)imin64((int64_t)BS, n - b0);
    const int64_t b1 = b0 + bk;

    int mode;             // 0 remainder, 1 row band, 2 column band
    int64_t row0, col0;
    if (PHASE == 3) {
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
    constexpr bool use_vec = VEC;

    // ---- load C
    U acc[8][CPT];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int li = G::row_off(ty, r);
        const bool rv = li < rows_valid;
        const U *rowp = D + (row0 + (rv ? li : 0)) * ld + col0;
#pragma unroll
        for (int g = 0; g < CPT / 4; ++g) {
            const int lj = G::col_off(tx, 4 * g);
            U v[4];
            if (rv) {
                load_row4(rowp, lj, cols_valid - lj, use_vec, v);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = Arith<U>::inf();
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[r][4 * g + e] = v[e];
        }
    }
    int32_t idx[8][CPT];    // improving k (-1: none), later the new successor
    if (ARGMIN == 1) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < CPT; ++c) idx[r][c] = -1;
    }
    if (ARGMIN == 2) {
#pragma unroll
        for (int q = t; q < kTile * kTile / 4; q += NT) kst[q] = 0xFFFFFFFFu;
        for (int q = t; q < G::waves * 64; q += NT) qmin[q] = 0xFF;
    }
    const int lane = t & 63;
    const int wq = (t >> 6) * QCAP;     // this wave's queue
    const int wq64 = (t >> 6) * 64;     // this wave's search results

    // ---- k loop: stage KC k's of A and B in LDS, then relax
    constexpr int APT = KC * kTile / NT;          // A entries staged per thread
    constexpr int BPT = KC * kTile / NT;          // B entries staged per thread
    const int a_il = t / (KC / APT), a_kq = (t % (KC / APT)) * APT;
    const int b_kk = t / (kTile / BPT), b_jq = (t % (kTile / BPT)) * BPT;
    for (int kc = 0; kc < bk; kc += KC) {
        if (kc) __syncthreads();
        {   // A: As[kk][il] = D[row0 + il][b0 + kc + kk]
            const bool rv = a_il < rows_valid;
            const U *p = D + (row0 + (rv ? a_il : 0)) * ld + b0 + kc;
#pragma unroll
            for (int q = 0; q < APT / 4; ++q) {
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
            for (int q = 0; q < BPT / 4; ++q) {
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

        if constexpr (ARGMIN == 1) {
#pragma unroll 2
            for (int kk = 0; kk < KC; ++kk) {
                U a[8], b[CPT];
                lds_operands<U, NT>(As, Bs, kk, tx, ty, a, b);
                const int kg = kc + kk;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
#pragma unroll
                    for (int c = 0; c < CPT; ++c) {
                        const U s = a[r] + b[c];
                        const bool lt = s < acc[r][c];
                        acc[r][c] = lt ? s : acc[r][c];
                        idx[r][c] = lt ? kg : idx[r][c];
                    }
                }
            }
        } else if constexpr (ARGMIN == 0) {
#pragma unroll 1
            for (int kk = 0; kk < KC; kk += 2) {
                U a[8], b[CPT], a2[8], b2[CPT];
                lds_operands<U, NT>(As, Bs, kk, tx, ty, a, b);
                lds_operands<U, NT>(As, Bs, kk + 1, tx, ty, a2, b2);
#pragma unroll
                for (int r = 0; r < 8; ++r) {
#pragma unroll
                    for (int c = 0; c < CPT; ++c) {
                        acc[r][c] = Arith<U>::mn(acc[r][c], Arith<U>::mn(a[r] + b[c], a2[r] + b2[c]));
                    }
                }
            }
        } else {
            U cm[8][CPT];   // minimum over this chunk
            {
                U a[8], b[CPT], a2[8], b2[CPT];
                lds_operands<U, NT>(As, Bs, 0, tx, ty, a, b);
                lds_operands<U, NT>(As, Bs, 1, tx, ty, a2, b2);
#pragma unroll
                for (int r = 0; r < 8; ++r)
#pragma unroll
                    for (int c = 0; c < CPT; ++c) cm[r][c] = Arith<U>::mn(a[r] + b[c], a2[r] + b2[c]);
            }
#pragma unroll 1
            for (int kk = 2; kk < KC; kk += 2) {
                U a[8], b[CPT], a2[8], b2[CPT];
                lds_operands<U, NT>(As, Bs, kk, tx, ty, a, b);
                lds_operands<U, NT>(As, Bs, kk + 1, tx, ty, a2, b2);
#pragma unroll
                for (int r = 0; r < 8; ++r) {
#pragma unroll
                    for (int c = 0; c < CPT; ++c) {
                        cm[r][c] = Arith<U>::mn(cm[r][c], Arith<U>::mn(a[r] + b[c], a2[r] + b2[c]));
                    }
                }
            }
            // ---- strict improvements of this chunk (cm < acc): find the first k
            // of each while the chunk is still in LDS.  Scanning k downwards and
            // keeping every hit leaves the smallest one.
            // Opaque copies of tx, ty: addresses derived from them are then
            // computed here, not hoisted out of the chunk loop into registers.
            int txo = tx, tyo = ty;
            asm volatile("" : "+v"(txo), "+v"(tyo));
            // Each pass queues the improved entries of every slot that still fits
            // in the QCAP-entry queue (a slot adds at most 64), folds those slots
            // into acc -- which makes cm < acc false for them, so a later pass
            // skips them -- and then searches the queue with all 64 lanes.  One
            // pass suffices unless more than QCAP entries improved (the first
            // rounds).  A slot with no improvement costs one compare and branch.
            const uint32_t ebase = (uint32_t)(tyo * 4) | ((uint32_t)(txo * 4) << 8);
            bool again;
            do {
                int qcnt = 0;
                again = false;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
#pragma unroll
                    for (int c = 0; c < CPT; ++c) {
                        const bool imp = cm[r][c] < acc[r][c];
                        const uint64_t m = __builtin_amdgcn_ballot_w64(imp);
                        if (m) {                                     // uniform
                            const int cnt = __builtin_popcountll(m);
                            if (qcnt + cnt <= QCAP) {
                                if (imp) {
                                    const int pos = qcnt + (int)__builtin_amdgcn_mbcnt_hi(
                                                               (uint32_t)(m >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                                    qpos[wq + pos] = ebase + (uint32_t)(G::row_off(0, r) | (G::col_off(0, c) << 8));
                                    qval[wq + pos] = cm[r][c];
                                }
                                qcnt += cnt;
                                acc[r][c] = Arith<U>::mn(acc[r][c], cm[r][c]);
                            } else {
                                again = true;
                            }
                        }
                    }
                }
                // m entries per batch; each gets L = 64 / m lanes (a power of two,
                // at most KC); lane o of an entry scans k = o*span .. o*span+span-1
                // and the entry's answer is the smallest hit over its lanes.
                for (int base = 0; base < qcnt; base += 64) {
                    const int m = (qcnt - base < 64) ? qcnt - base : 64;
                    wave_sync();
                    const int cl2 = (m <= 1) ? 0 : 32 - __builtin_clz((uint32_t)(m - 1));   // ceil(log2 m)
                    const int lg = (6 - cl2 < 5) ? 6 - cl2 : 5;                             // log2 L
                    const int span = KC >> lg;
                    const int e = lane >> lg, o = lane & ((1 << lg) - 1);
                    int li = 0, lj = 0, kb = 0xFF;
                    if (e < m) {
                        const uint32_t ent = qpos[wq + base + e];
                        li = (int)(ent & 0xFFu);
                        lj = (int)(ent >> 8);
                        const U tgt = qval[wq + base + e];
                        const int k0 = o * span;
                        int q = span - 1;
                        for (; q >= 3; q -= 4) {
                            const U x0 = As[k0 + q][li] + Bs[k0 + q][lj];
                            const U x1 = As[k0 + q - 1][li] + Bs[k0 + q - 1][lj];
                            const U x2 = As[k0 + q - 2][li] + Bs[k0 + q - 2][lj];
                            const U x3 = As[k0 + q - 3][li] + Bs[k0 + q - 3][lj];
                            kb = (x0 == tgt) ? k0 + q : kb;
                            kb = (x1 == tgt) ? k0 + q - 1 : kb;
                            kb = (x2 == tgt) ? k0 + q - 2 : kb;
                            kb = (x3 == tgt) ? k0 + q - 3 : kb;
                        }
                        for (; q >= 0; --q) kb = (As[k0 + q][li] + Bs[k0 + q][lj] == tgt) ? k0 + q : kb;
                    }
                    if (lg == 0) {
                        if (e < m) reinterpret_cast<uint8_t *>(kst)[li * kTile + lj] = (uint8_t)(kc + kb);
                    } else {
                        if (e < m && kb != 0xFF) atomicMin(&qmin[wq64 + e], kb);
                        wave_sync();
                        if (e < m && o == 0) {
                            reinterpret_cast<uint8_t *>(kst)[li * kTile + lj] = (uint8_t)(kc + qmin[wq64 + e]);
                            qmin[wq64 + e] = 0xFF;
                        }
                    }
                    wave_sync();
                }
            } while (again);
        }
    }

    // The epilogue recomputes its addresses from opaque copies of tx and ty
    // rather than keeping the prologue's live across the k loop.
    int txe = tx, tye = ty;
    asm volatile("" : "+v"(txe), "+v"(tye));

    // ---- successor gather (reads A's NX before anything is written: for the
    // column band A is C itself).  Afterwards idx holds the new successor of
    // an improved entry (>= 0: its A entry is finite) and -1 elsewhere.
    if (NEXT) {
        if (ARGMIN == 2) {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const uint32_t w = kst[(G::row_off(tye, r) * kTile + G::col_off(txe, 0)) >> 2];
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const uint32_t kb = (w >> (8 * c)) & 0xFFu;
                    idx[r][c] = kb == 0xFFu ? -1 : (int32_t)kb;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int li = G::row_off(tye, r);
            const int32_t *nrow = NX + (row0 + (li < rows_valid ? li : 0)) * ld + b0;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                if (idx[r][c] >= 0) idx[r][c] = nrow[idx[r][c]];
            }
        }
        __syncthreads();
    }

    // ---- store (rows / columns of the band itself are not part of phase 3)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int li = G::row_off(tye, r);
        const int64_t gi = row0 + li;
        bool rs = li < rows_valid;
        if (mode != 1) rs = rs && !(gi >= b0 && gi < b1);
        if (!rs) continue;
        U *drow = D + gi * ld + col0;
        int32_t *nrow = NEXT ? NX + gi * ld + col0 : nullptr;
#pragma unroll
        for (int g = 0; g < CPT / 4; ++g) {
            const int lj = G::col_off(txe, 4 * g);
            bool cs[4];
            bool all = true;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gj = col0 + lj + e;
                cs[e] = (lj + e) < cols_valid && (mode == 2 || !(gj >= b0 && gj < b1));
                all = all && cs[e];
            }
            if (NEXT) {
                // only improved entries change
                bool ch[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) ch[e] = cs[e] && idx[r][4 * g + e] >= 0;
                if (use_vec && all) {
                    if (ch[0] || ch[1] || ch[2] || ch[3]) {
                        typename Arith<U>::V4 w;
                        w.x = acc[r][4 * g + 0]; w.y = acc[r][4 * g + 1];
                        w.z = acc[r][4 * g + 2]; w.w = acc[r][4 * g + 3];
                        *reinterpret_cast<typename Arith<U>::V4 *>(drow + lj) = w;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (ch[e]) drow[lj + e] = acc[r][4 * g + e];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (ch[e]) nrow[lj + e] = idx[r][4 * g + e];
            } else {
                if (use_vec && all) {
                    typename Arith<U>::V4 w;
                    w.x = acc[r][4 * g + 0]; w.y = acc[r][4 * g + 1];
                    w.z = acc[r][4 * g + 2]; w.w = acc[r][4 * g + 3];
                    *reinterpret_cast<typename Arith<U>::V4 *>(drow + lj) = w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (cs[e]) drow[lj + e] = acc[r][4 * g + e];
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

template <typename U, int ARGMIN, bool VEC>
hipError_t minplus_t(const Plan &p, int K, int phase) {
    constexpr int NT = (ARGMIN == 2) ? 512 : 256;
    if (phase == 2) {
        hipLaunchKernelGGL((minplus_kernel<U, ARGMIN, 2, VEC>), dim3((unsigned)p.nt, 2), dim3(NT), 0, p.stream,
                           (U *)p.dist, p.next, p.n, p.ld, K, p.bs, p.nt);
    } else {
        const int64_t tiles = (int64_t)p.nt * p.nt;
        hipLaunchKernelGGL((minplus_kernel<U, ARGMIN, 3, VEC>), dim3((unsigned)(8 * ((tiles + 7) / 8))), dim3(NT),
                           0, p.stream, (U *)p.dist, p.next, p.n, p.ld, K, p.bs, p.nt);
    }
    return hipGetLastError();
}

template <typename U, int ARGMIN>
hipError_t minplus_v(const Plan &p, int K, int phase) {
    return p.vec ? minplus_t<U, ARGMIN, true>(p, K, phase) : minplus_t<U, ARGMIN, false>(p, K, phase);
}

}  // namespace

hipError_t launch_init(const Plan &p) {
    return p.dtype == DType::I32 ? init_t<uint32_t>(p) : init_t<float>(p);
}

hipError_t launch_phase1(const Plan &p, int K) {
    if (p.dtype == DType::I32) return p.next ? phase1_t<uint32_t, true>(p, K) : phase1_t<uint32_t, false>(p, K);
    return p.next ? phase1_t<float, true>(p, K) : phase1_t<float, false>(p, K);
}

template <typename U>
hipError_t minplus_dispatch(const Plan &p, int K, int phase) {
    if (!p.next) return minplus_v<U, 0>(p, K, phase);
    return p.eager_argmin ? minplus_v<U, 1>(p, K, phase) : minplus_v<U, 2>(p, K, phase);
}

hipError_t launch_phase2(const Plan &p, int K) {
    return p.dtype == DType::I32 ? minplus_dispatch<uint32_t>(p, K, 2) : minplus_dispatch<float>(p, K, 2);
}

hipError_t launch_phase3(const Plan &p, int K) {
    return p.dtype == DType::I32 ? minplus_dispatch<uint32_t>(p, K, 3) : minplus_dispatch<float>(p, K, 3);
}

}  // namespace fw
