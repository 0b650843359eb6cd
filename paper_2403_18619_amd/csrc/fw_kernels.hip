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
// comparison that choice is the same in every schedule and tile order.  (The
// int32 direct-copy phase 3 records K*BS + k* as a tag instead and looks the
// successor up once the last round is done: resolve_next_kernel.)
//
// Arithmetic: int32 distances run as uint32 (INF = 2^30, INF + INF = 2^31
// does not wrap); float32 and float64 as IEEE single / double.  Every
// relaxation is a single rounded add, so the k order does not change any
// distance.
#include <atomic>
#include <type_traits>

#include "fw_internal.h"

namespace fw {
namespace {

constexpr int KC = 32;            // k-chunk staged in LDS per step
constexpr int LDP = kTile + 4;    // LDS row pitch (elements), keeps 16-byte alignment
constexpr uint32_t kInfU = 1u << 30;
// A successor entry with bits 31..30 = 01 is a tag: "the successor of this
// entry is that of entry (i, v & (kLazyBit - 1))" (direct-copy phase 3 of
// int32 solves; resolve_next_kernel removes every tag before the solve ends).
// Successors proper are -1 or below 2^30.
constexpr int32_t kLazyBit = 1 << 30;

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
template <> struct Arith<double> {
    using V4 = double4;
    static __device__ __forceinline__ double inf() { return __builtin_inf(); }
    static __device__ __forceinline__ double mn(double a, double b) { return __builtin_fmin(a, b); }
};

// One eager relaxation's new value, min(d, s), when the caller also needs
// whether s < d (to move the successor).  Taking the minimum apart from the
// comparison leaves the successor select as the only instruction that waits
// on the comparison's lane mask.  Same bits as s < d ? s : d: distances and
// sums are never NaN or -0, and non-negative floats (+inf included) order as
// their bit patterns do.
__device__ __forceinline__ uint32_t eager_min(uint32_t d, uint32_t s) { return min(d, s); }
__device__ __forceinline__ float eager_min(float d, float s) {
    return __uint_as_float(min(__float_as_uint(d), __float_as_uint(s)));
}
__device__ __forceinline__ double eager_min(double d, double s) { return s < d ? s : d; }

// Launch bounds.  Threads per workgroup of the min-plus code: 512 for the
// successor variants (8 x 4 entries per thread: a value and a chunk minimum,
// or a value and an index, per entry), 256 for distances only (8 x 8).
// Minimum waves per SIMD: 32-bit distances fit 128 VGPRs at four waves;
// 64-bit ones need twice the registers and run two waves.
template <typename U, int ARGMIN> struct Occ {
    static constexpr int threads = ARGMIN == 0 ? 256 : 512;
    // persistent and team kernels (the min-plus tile plus the schedule's own
    // state): the distances-only 8 x 8 patch runs three waves rather than spill
    static constexpr int waves = sizeof(U) == 8 ? 2 : (ARGMIN == 0 ? 3 : 4);
    static constexpr int waves_standalone = sizeof(U) == 8 ? (ARGMIN == 0 ? 1 : 2) : (ARGMIN == 0 ? 1 : 4);
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
__device__ __forceinline__ double norm_weight(double v, bool diag, bool &bad) {
    bad = !diag && (v < 0.0 || v != v);
    if (diag) return 0.0;
    if (v != v) return __builtin_inf();
    return v == 0.0 ? 0.0 : v;
}

// Normalise entries start, start + stride, ... of one graph's n x n
// row-major block (as init_kernel).  Eight loads are in flight per thread
// before any entry is rewritten, and the row and column of the next entry
// are stepped, not divided out, so that the loop costs one memory round trip
// per eight entries.  Returns whether a negative or NaN weight was seen.
template <typename U, bool NEXT>
__device__ __forceinline__ bool normalise_graph(U *__restrict__ Dg, int32_t *__restrict__ NXg, int64_t n,
                                                int64_t start, int64_t stride) {
    constexpr int UNR = 8;
    const int64_t nn = n * n;
    if (start >= nn) return false;
    const int64_t di = stride / n, dj = stride % n;
    int64_t i = start / n, j = start % n;
    bool any_bad = false;
    for (int64_t base = start; base < nn; base += UNR * stride) {
        U w[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t q = base + u * stride;
            w[u] = q < nn ? Dg[q] : U(0);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t q = base + u * stride;
            if (q < nn) {
                bool bad;
                const U v = norm_weight(w[u], i == j, bad);
                any_bad |= bad;
                Dg[q] = v;
                if (NEXT) NXg[q] = (i == j) ? (int32_t)i : (v < Arith<U>::inf() ? (int32_t)j : -1);
            }
            i += di;
            j += dj;
            if (j >= n) {                          // dj < n and j < n: one wrap at most
                j -= n;
                ++i;
            }
        }
    }
    return any_bad;
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
// workgroup of NT threads.  Thread (tx, ty) of a TX x 16 grid keeps an
// MR x MC patch of the block's distances in registers (rows ty*MR + r,
// columns tx*MC + c).  At step k only row k and column k are read, and
// neither they nor successor column k change during step k (D[k][k] = 0,
// strict test), so the owners publish row / column k+1 into a double-buffered
// LDS row / column and one barrier per step suffices.  The k loop is unrolled
// by MR so that every register index is static.  Successors live in the
// patch too (NXLDS = false: fastest, as a workgroup of its own) or in an LDS
// copy of the block (NXLDS = true: fewer registers, inside the persistent
// kernel); both give the same bits.
template <typename U, int BS, bool NXLDS> struct alignas(4 * sizeof(U)) Phase1Smem {
    U rowb[2][BS];
    U colb[2][BS];
    int32_t nxb[NXLDS ? 1 : 2][BS];              // published successor column
    int32_t nx[NXLDS ? BS : 1][BS + 1];          // odd pitch: column reads hit distinct banks
};

// s_max (32-bit entries; may be null): an LDS word that receives, by atomic
// maximum, the largest finite entry of the closed block (the caller zeroes
// it before and reads it after a barrier).
template <typename U, bool NEXT, int BS, int NT, bool NXLDS>
__device__ __forceinline__ void phase1_block(U *__restrict__ D, int32_t *__restrict__ NX, int64_t n,
                                             int64_t ld, int K, Phase1Smem<U, BS, NXLDS> &sm,
                                             uint32_t *s_max = nullptr) {
    constexpr int TX = NT / 16;
    constexpr int MR = BS / 16, MC = BS / TX;
    constexpr bool NXR = NEXT && !NXLDS;         // successors in registers
    constexpr bool NXL = NEXT && NXLDS;          // successors in LDS
    // an opaque thread index: per-thread addresses are derived here, on every
    // call, instead of being hoisted into registers that live across callers
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int tx = t % TX, ty = t / TX;
    const int64_t b0 = (int64_t)K * BS;
    const int bk = (int)imin64((int64_t)BS, n - b0);

    U d[MR][MC];
    int32_t nx[NXR ? MR : 1][NXR ? MC : 1];
#pragma unroll
    for (int r = 0; r < MR; ++r) {
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            const int li = ty * MR + r, lj = tx * MC + c;
            const bool in = li < bk && lj < bk;
            if (in) d[r][c] = D[(b0 + li) * ld + b0 + lj];
            else d[r][c] = (li == lj) ? U(0) : Arith<U>::inf();
            if (NXR) nx[NXR ? r : 0][NXR ? c : 0] = in ? NX[(b0 + li) * ld + b0 + lj] : -1;
        }
    }
    if (NXL) {
        for (int q = t; q < bk * bk; q += NT) {
            const int li = q / bk, lj = q % bk;
            sm.nx[NXL ? li : 0][lj] = NX[(b0 + li) * ld + b0 + lj];
        }
    }
    if (ty == 0) {
#pragma unroll
        for (int c = 0; c < MC; ++c) sm.rowb[0][tx * MC + c] = d[0][c];
    }
    if (tx == 0) {
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            sm.colb[0][ty * MR + r] = d[r][0];
            if (NXR) sm.nxb[0][ty * MR + r] = nx[NXR ? r : 0][0];
        }
    }
    __syncthreads();

    for (int kb = 0; kb * MR < bk; ++kb) {
        // opaque copies: LDS addresses are recomputed here rather than kept
        // for every unrolled step
        int txo = tx, tyo = ty;
        asm volatile("" : "+v"(txo), "+v"(tyo));
#pragma unroll
        for (int u = 0; u < MR; ++u) {
            const int k = kb * MR + u;
            if (k < bk) {                       // uniform across the workgroup
                const int cur = k & 1;
                U a[MR], b[MC];
                int32_t na[MR];
#pragma unroll
                for (int r = 0; r < MR; ++r) {
                    a[r] = sm.colb[cur][tyo * MR + r];
                    if (NXR) na[r] = sm.nxb[NXR ? cur : 0][tyo * MR + r];
                    if (NXL) na[r] = sm.nx[NXL ? tyo * MR + r : 0][k];
                }
#pragma unroll
                for (int c = 0; c < MC; ++c) b[c] = sm.rowb[cur][txo * MC + c];
#pragma unroll
                for (int r = 0; r < MR; ++r) {
#pragma unroll
                    for (int c = 0; c < MC; ++c) {
                        const U s = a[r] + b[c];
                        const bool lt = s < d[r][c];
                        d[r][c] = eager_min(d[r][c], s);
                        if (NXR) nx[NXR ? r : 0][NXR ? c : 0] = lt ? na[r] : nx[NXR ? r : 0][NXR ? c : 0];
                        if (NXL && lt) sm.nx[NXL ? tyo * MR + r : 0][txo * MC + c] = na[r];
                    }
                }
                // publish row / column k+1 for the next step (owners and
                // patch positions are static after unrolling)
                const int k1 = k + 1;
                const int rown = (u + 1 == MR) ? kb + 1 : kb;          // owner ty of row k1
                const int r1 = (u + 1) % MR;
                const int coln = (kb * MR + u + 1) / MC;               // owner tx of column k1
                const int c1 = (u + 1) % MC;
                if (k1 < bk) {
                    if (tyo == rown) {
#pragma unroll
                        for (int c = 0; c < MC; ++c) sm.rowb[cur ^ 1][txo * MC + c] = d[r1][c];
                    }
                    if (txo == coln) {
#pragma unroll
                        for (int r = 0; r < MR; ++r) {
                            sm.colb[cur ^ 1][tyo * MR + r] = d[r][c1];
                            if (NXR) sm.nxb[NXR ? cur ^ 1 : 0][tyo * MR + r] = nx[NXR ? r : 0][NXR ? c1 : 0];
                        }
                    }
                }
                __syncthreads();
            }
        }
    }

    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < MR; ++r) {
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            const int li = ty * MR + r, lj = tx * MC + c;
            if (li < bk && lj < bk) {
                D[(b0 + li) * ld + b0 + lj] = d[r][c];
                if (NXR) NX[(b0 + li) * ld + b0 + lj] = nx[NXR ? r : 0][NXR ? c : 0];
                if constexpr (sizeof(U) == 4 && !std::is_same<U, float>::value) {
                    const uint32_t v = (uint32_t)d[r][c];
                    if (v < kInfU && v > m) m = v;
                }
            }
        }
    }
    if constexpr (sizeof(U) == 4 && !std::is_same<U, float>::value) {
        if (s_max) atomicMax(s_max, m);
    }
    if (NXL) {
        for (int q = t; q < bk * bk; q += NT) {
            const int li = q / bk, lj = q % bk;
            NX[(b0 + li) * ld + b0 + lj] = sm.nx[NXL ? li : 0][lj];
        }
    }
}

// dmax (int32 with successors in the three-launch schedule, else null): the
// closed block's largest finite entry goes to dmax[K & 1], for the band tiles'
// packed-key test.
template <typename U, bool NEXT, int BS>
__global__ __launch_bounds__(256) void phase1_kernel(U *__restrict__ D, int32_t *__restrict__ NX,
                                                     int64_t n, int64_t ld, int K, int *__restrict__ dmax) {
    __shared__ Phase1Smem<U, BS, false> sm;
    __shared__ uint32_t s_max;
    if (threadIdx.x == 0) s_max = 0;               // ordered by phase1_block's first barrier
    phase1_block<U, NEXT, BS, 256, false>(D, NX, n, ld, K, sm, dmax ? &s_max : nullptr);
    if (dmax) {
        __syncthreads();
        if (threadIdx.x == 0) dmax[K & 1] = (int)s_max;
    }
}

// Closure of an n x n block (n <= S) by one workgroup of NT threads: phase 1
// of the batched solve (a diagonal block, or a whole small graph).
// Thread (tx, ty) of an NT/16 x 16 grid keeps an MR x MC patch of the
// distances and successors in registers (rows ty * MR + r, columns tx * MC +
// c; MR = S / 16, MC = S * 16 / NT).  Step k reads row k and column k (and the
// successors of column k) from double-buffered LDS vectors -- they do not
// change during step k -- and the owners of row and column k + 1 publish
// them; one barrier per step.  The k loop is not unrolled: the owners pick
// the published registers through a switch on their static index.  Same
// arithmetic, order and successor choice as phase1_block.
template <typename U, bool NEXT, int S, int NT>
__device__ __forceinline__ void closure_block(U *__restrict__ D, int32_t *__restrict__ NX, int64_t n, int64_t ld,
                                              Phase1Smem<U, S, false> &sm) {
    constexpr int TX = NT / 16, MR = S / 16, MC = S / TX;
    static_assert(MR * 16 == S && MC * TX == S && MR <= 8 && MC <= 8, "patch of at most 8 x 8");
    // The closure is a chain of barrier steps while the workgroup it shares
    // a CU with usually runs tiles: its waves issue first while it lasts.
    __builtin_amdgcn_s_setprio(2);
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int tx = t % TX, ty = t / TX;
    const int nn = (int)n;
    U d[MR][MC];
    int32_t nx[NEXT ? MR : 1][NEXT ? MC : 1];
#pragma unroll
    for (int r = 0; r < MR; ++r) {
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            const int li = ty * MR + r, lj = tx * MC + c;
            const bool in = li < nn && lj < nn;
            d[r][c] = in ? D[(int64_t)li * ld + lj] : ((li == lj) ? U(0) : Arith<U>::inf());
            if (NEXT) nx[NEXT ? r : 0][NEXT ? c : 0] = in ? NX[(int64_t)li * ld + lj] : -1;
        }
    }
    if (ty == 0) {
#pragma unroll
        for (int c = 0; c < MC; ++c) sm.rowb[0][tx * MC + c] = d[0][c];
    }
    if (tx == 0) {
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            sm.colb[0][ty * MR + r] = d[r][0];
            if (NEXT) sm.nxb[0][ty * MR + r] = nx[NEXT ? r : 0][0];
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < nn; ++k) {
        const int cur = k & 1;
        U a[MR], b[MC];
        int32_t na[MR];
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            a[r] = sm.colb[cur][ty * MR + r];
            if (NEXT) na[r] = sm.nxb[cur][ty * MR + r];
        }
#pragma unroll
        for (int c = 0; c < MC; ++c) b[c] = sm.rowb[cur][tx * MC + c];
#pragma unroll
        for (int r = 0; r < MR; ++r) {
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                const U sum = a[r] + b[c];
                const bool lt = sum < d[r][c];
                d[r][c] = eager_min(d[r][c], sum);
                if (NEXT) nx[NEXT ? r : 0][NEXT ? c : 0] = lt ? na[r] : nx[NEXT ? r : 0][NEXT ? c : 0];
            }
        }
        const int k1 = k + 1;
        if (k1 < nn) {
            if (ty == k1 / MR) {                    // owner of row k + 1 (one wave)
                switch (k1 % MR) {
#define FW_PUB_ROW(R)                                                                 \
    case R:                                                                           \
        _Pragma("unroll") for (int c = 0; c < MC; ++c) sm.rowb[cur ^ 1][tx * MC + c] = \
                d[(R) < MR ? (R) : 0][c];                                            \
        break;
                    FW_PUB_ROW(0) FW_PUB_ROW(1) FW_PUB_ROW(2) FW_PUB_ROW(3)
                    FW_PUB_ROW(4) FW_PUB_ROW(5) FW_PUB_ROW(6) FW_PUB_ROW(7)
#undef FW_PUB_ROW
                }
            }
            if (tx == k1 / MC) {                    // owner of column k + 1
                switch (k1 % MC) {
#define FW_PUB_COL(C)                                                                            \
    case C:                                                                                      \
        _Pragma("unroll") for (int r = 0; r < MR; ++r) {                                        \
            sm.colb[cur ^ 1][ty * MR + r] = d[r][(C) < MC ? (C) : 0];                           \
            if (NEXT) sm.nxb[cur ^ 1][ty * MR + r] = nx[NEXT ? r : 0][NEXT && (C) < MC ? (C) : 0]; \
        }                                                                                        \
        break;
                    FW_PUB_COL(0) FW_PUB_COL(1) FW_PUB_COL(2) FW_PUB_COL(3)
                    FW_PUB_COL(4) FW_PUB_COL(5) FW_PUB_COL(6) FW_PUB_COL(7)
#undef FW_PUB_COL
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < MR; ++r) {
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            const int li = ty * MR + r, lj = tx * MC + c;
            if (li < nn && lj < nn) {
                D[(int64_t)li * ld + lj] = d[r][c];
                if (NEXT) NX[(int64_t)li * ld + lj] = nx[NEXT ? r : 0][NEXT ? c : 0];
            }
        }
    }
    __builtin_amdgcn_s_setprio(0);
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
template <typename U, int NT, int P = LDP>
__device__ __forceinline__ void lds_operands(const U (*As)[P], const U (*Bs)[P], int kk, int tx,
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

// Orders LDS traffic between lanes of one wave (the LDS executes a wave's
// accesses in issue order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int ld_flag(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
// Waits until this wave's vector-memory operations (its global stores, a
// cache invalidate) have completed.  A workgroup barrier alone does not: it
// orders the waves but lets their stores still be on the way to L2.
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

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
//
// Packed keys (int32 distances, variant 2, phase 3).  When every finite
// entry of the round's two operand panels is below 2^22, a phase-3 tile runs
// the distances-only loop on 32-bit keys that carry the successor choice:
//   A' = min(a, S) << 8,   B'[k] = (min(b, S) << 8) | (2k + 1),   S = 2^23 - 1
// (k = position in the round, 0..127), the running value starts as
// min(C, S) << 8.  A finite + finite sum stays below S, so its key orders
// exactly like the sum, ties broken by the smaller k; a sum with an "infinite"
// operand clamps to at least S and never beats anything (its true value is
// infinite).  A key below the initial one means a strict improvement, and its
// low bit -- 1 in every candidate, 0 in the initial value -- records that it
// happened; the minimum key also names the first k reaching the minimum, the
// same k as the other variants.  No chunk-end search is needed.  Each row
// and column band tile publishes the largest finite entry it holds (per round
// parity) for the phase-3 tiles to test.
template <typename U, int ARGMIN> struct alignas(4 * sizeof(U)) MinplusSmem {
    static constexpr int NT = (ARGMIN == 0) ? 256 : 512;
    static constexpr int QCAP = 128;                           // queue entries per wave
    static constexpr int Q = (ARGMIN == 2) ? NT / 64 * QCAP : 1;
    // 64-bit entries are read as 32-byte vectors: declare that alignment (for
    // 32-bit ones the struct's own alignment serves 16-byte reads, and a
    // declared member alignment changes the generated code for the worse)
    alignas(sizeof(U) == 8 ? 32 : alignof(U)) U As[KC][LDP];  // As[k][i] = A[i][k]
    alignas(sizeof(U) == 8 ? 32 : alignof(U)) U Bs[KC][LDP];  // Bs[k][j] = B[k][j]
    uint32_t kst[ARGMIN == 2 ? kTile * kTile / 4 : 1];       // improving k per entry (bytes)
    uint32_t qpos[Q];                                         // queued entry: i | j << 8
    U qval[Q];                                                // its chunk minimum
    int qmin[ARGMIN == 2 ? NT : 1];                           // per-entry search result
    uint32_t bmax_s;                                          // band tile: largest finite entry
};

constexpr uint32_t kPackLimit = 1u << 22;     // operand panels below this: packed keys
constexpr uint32_t kPackSat = (1u << 23) - 1; // S: operands clamp here
__device__ __forceinline__ uint32_t pack_a(uint32_t a) { return (a < kPackSat ? a : kPackSat) << 8; }
// 32-bit entries as raw panel words and back (distances-only panels)
__device__ __forceinline__ uint32_t to_bits(uint32_t v) { return v; }
__device__ __forceinline__ uint32_t to_bits(float v) { return __float_as_uint(v); }
template <typename U> __device__ __forceinline__ U from_bits(uint32_t w);
template <> __device__ __forceinline__ uint32_t from_bits<uint32_t>(uint32_t w) { return w; }
template <> __device__ __forceinline__ float from_bits<float>(uint32_t w) { return __uint_as_float(w); }
__device__ __forceinline__ uint32_t pack_b(uint32_t b, int k) {
    return ((b < kPackSat ? b : kPackSat) << 8) | (uint32_t)(2 * k + 1);
}

// Where the tile of a min-plus launch lies.  mode 0: remainder (phase 3),
// 1: row band, 2: column band (phase 2).  Returns false when every row or
// every column of the tile belongs to the band (nothing to update there).
__device__ __forceinline__ bool band_tile(int mode, int64_t idx, int64_t n, int64_t b0, int64_t b1,
                                          int nt, int64_t &row0, int64_t &col0) {
    if (mode == 0) {
        row0 = (idx / nt) * kTile;
        col0 = (idx % nt) * kTile;
    } else if (mode == 1) {
        row0 = b0;
        col0 = idx * kTile;
    } else {
        row0 = idx * kTile;
        col0 = b0;
    }
    if (mode != 1 && row0 >= b0 && imin64(row0 + kTile, n) <= b1) return false;
    if (mode != 2 && col0 >= b0 && imin64(col0 + kTile, n) <= b1) return false;
    return true;
}

// One 128 x 128 tile of C <- min(C, A (x) B) over the round's band.
// bmax (may be null): per-round-parity band maxima, 2 x 2 x nt ints
// (row band tiles, then column band tiles), read by phase-3 tiles and written
// by band tiles when packed keys apply (int32, variant 2).
template <typename U, int ARGMIN, bool VEC, bool PACKED>
__device__ __forceinline__ void minplus_tile_impl(U *__restrict__ D, int32_t *__restrict__ NX, int64_t n,
                                                  int64_t ld, int K, int BS, int mode, int64_t row0,
                                                  int64_t col0, MinplusSmem<U, ARGMIN> &sm,
                                                  int *__restrict__ bmax, int nt,
                                                  uint32_t *__restrict__ panel, int64_t ppitch) {
    constexpr int NT = MinplusSmem<U, ARGMIN>::NT;
    using G = Geo<NT>;
    constexpr int CPT = G::cpt;
    constexpr bool NEXT = ARGMIN != 0;
    constexpr int QCAP = MinplusSmem<U, ARGMIN>::QCAP;
    // chunks of 32 k (64 for the packed form measured slower: more staging
    // registers per thread outweigh the halved barriers)
    constexpr int KCT = KC;
    auto &As = sm.As;
    auto &Bs = sm.Bs;
    auto &kst = sm.kst;
    auto &qpos = sm.qpos;
    auto &qval = sm.qval;
    auto &qmin = sm.qmin;

    // an opaque thread index (see phase1_block)
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int64_t b0 = (int64_t)K * BS;
    const int bk = (int)imin64((int64_t)BS, n - b0);
    const int64_t b1 = b0 + bk;
    // number of valid rows / columns of C (and of A's rows, B's columns)
    const int rows_valid = (mode == 1) ? bk : (int)imin64(kTile, n - row0);
    const int cols_valid = (mode == 2) ? bk : (int)imin64(kTile, n - col0);
    // Thread -> patch.  The eager variant gives each wave a block of the tile
    // so that a wave whose columns, or rows, all lie past a ragged tile's edge
    // has nothing to relax (it stages operands and joins the barriers, and
    // skips the relaxations).  Of two layouts the tile takes the one with
    // fewer waves left working: 16 x 4 threads per wave (a 64-column half,
    // 16 rows of each 64-row half) or 8 x 8 (a 32-column quarter, 32 rows of
    // each half).  The other variants keep 32 x 2 threads per wave.
    int tx, ty;
    bool idle_wave = false;
    if constexpr (ARGMIN == 1 && NT == 512) {
        const int ca = min(2, (cols_valid + 63) / 64), ra = min(4, (rows_valid + 15) / 16);
        const int cb = min(4, (cols_valid + 31) / 32), rb = min(2, (rows_valid + 31) / 32);
        const bool quarters = cb * rb < ca * ra;      // uniform
        const int w = t >> 6, l = t & 63;
        const int ws = __builtin_amdgcn_readfirstlane(w);
        if (quarters) {
            tx = (w & 3) * 8 + (l & 7);
            ty = (w >> 2) * 8 + (l >> 3);
            idle_wave = (ws & 3) * 32 >= cols_valid || (ws >> 2) * 32 >= rows_valid;
        } else {
            tx = (w & 1) * 16 + (l & 15);
            ty = (w >> 1) * 4 + (l >> 4);
            idle_wave = (ws & 1) * 64 >= cols_valid || (ws >> 1) * 16 >= rows_valid;
        }
    } else {
        tx = t % G::txn;
        ty = t / G::txn;
    }
    constexpr bool use_vec = VEC;
    constexpr bool PACKABLE = ARGMIN == 2 && std::is_same<U, uint32_t>::value;
    constexpr bool fast = PACKABLE && PACKED;       // packed keys for this tile
    int *const bm = PACKABLE && bmax ? bmax + (K & 1) * 2 * nt : nullptr;
    if constexpr (PACKABLE) {
        if (t == 0) sm.bmax_s = 0;
    }

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
    if constexpr (fast) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < CPT; ++c) acc[r][c] = pack_a((uint32_t)acc[r][c]);
    }
    int32_t idx[8][CPT];    // improving k (-1: none), later the new successor
    if (ARGMIN == 1) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < CPT; ++c) idx[r][c] = -1;
    }
    if (ARGMIN == 2 && !fast) {
        for (int q = t; q < kTile * kTile / 4; q += NT) kst[q] = 0xFFFFFFFFu;
        for (int q = t; q < G::waves * 64; q += NT) qmin[q] = 0xFF;
    }
    const int lane = t & 63;
    const int wq = (t >> 6) * QCAP;     // this wave's queue
    const int wq64 = (t >> 6) * 64;     // this wave's search results

    // ---- k loop: stage KCT k's of A and B in LDS, then relax
    constexpr int APT = KCT * kTile / NT;         // A entries staged per thread
    constexpr int BPT = KCT * kTile / NT;         // B entries staged per thread
    const int a_il = t / (KCT / APT), a_kq = (t % (KCT / APT)) * APT;
    const int b_kk = t / (kTile / BPT), b_jq = (t % (kTile / BPT)) * BPT;
    for (int kc = 0; kc < bk; kc += KCT) {
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
                if constexpr (fast) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = pack_a(v[e]);
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
                if constexpr (fast) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = pack_b(v[e], kc + b_kk);
                }
                typename Arith<U>::V4 w;
                w.x = v[0]; w.y = v[1]; w.z = v[2]; w.w = v[3];
                *reinterpret_cast<typename Arith<U>::V4 *>(&Bs[b_kk][jl]) = w;
            }
        }
        __syncthreads();

        if constexpr (fast) {
#pragma unroll 1
            for (int kk = 0; kk < KCT; kk += 2) {
                U a[8], b[CPT], a2[8], b2[CPT];
                lds_operands<U, NT>(As, Bs, kk, tx, ty, a, b);
                lds_operands<U, NT>(As, Bs, kk + 1, tx, ty, a2, b2);
#pragma unroll
                for (int r = 0; r < 8; ++r) {
#pragma unroll
                    for (int c = 0; c < CPT; ++c)
                        acc[r][c] = Arith<U>::mn(acc[r][c], Arith<U>::mn(a[r] + b[c], a2[r] + b2[c]));
                }
            }
        } else if constexpr (ARGMIN == 1) {
            // rows 64.. of the patch (r >= 4) exist only when the tile has
            // more than 64 valid rows; a ragged tile (a small graph's last
            // band) skips that half, uniformly across the workgroup (the k's
            // past the band's end are INF operands and change nothing)
            auto eager = [&](auto rows_t) {
                constexpr int RR = decltype(rows_t)::value;
                const int klim = (bk - kc < KC) ? bk - kc : KC;   // a short last band stops early
#pragma unroll 2
                for (int kk = 0; kk < klim; ++kk) {
                    U a[8], b[CPT];
                    lds_operands<U, NT>(As, Bs, kk, tx, ty, a, b);
                    const int kg = kc + kk;
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
#pragma unroll
                        for (int c = 0; c < CPT; ++c) {
                            const U s = a[r] + b[c];
                            const bool lt = s < acc[r][c];
                            acc[r][c] = eager_min(acc[r][c], s);
                            idx[r][c] = lt ? kg : idx[r][c];
                        }
                    }
                }
            };
            if (!idle_wave) {
                if (rows_valid > 64) eager(std::integral_constant<int, 8>{});
                else eager(std::integral_constant<int, 4>{});
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
        if constexpr (fast) {
            // packed keys: bit 0 = improved, bits 1..7 = k, bits 8.. = value
#pragma unroll
            for (int r = 0; r < 8; ++r) {
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const uint32_t key = (uint32_t)acc[r][c];
                    idx[r][c] = (key & 1u) ? (int32_t)((key >> 1) & 127u) : -1;
                    acc[r][c] = (U)(key >> 8);
                }
            }
        } else if (ARGMIN == 2) {
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

    // ---- a band tile publishes its largest finite entry (packed keys).  In
    // the packed form an entry that stayed infinite holds the clamped value
    // S (every finite result there is a sum below S), so S counts as infinite.
    if constexpr (PACKABLE) {
        if (mode != 0 && bm) {
            constexpr uint32_t fin = PACKED ? kPackSat : kInfU;
            uint32_t m = 0;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const bool rv = G::row_off(tye, r) < rows_valid;
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const uint32_t v = (uint32_t)acc[r][c];
                    if (rv && G::col_off(txe, c) < cols_valid && v < fin) m = v > m ? v : m;
                }
            }
            atomicMax(&sm.bmax_s, m);
            __syncthreads();
            if (t == 0) bm[(mode == 1 ? 0 : nt) + (int)((mode == 1 ? col0 : row0) / kTile)] = (int)sm.bmax_s;
        }
        // ... and its packed operand panel for the direct-copy phase 3 (block
        // size 128; round parity K & 1): a row band tile writes
        // B'[k][j] = pack_b(D[b0 + k][j], k), a column band tile
        // A'[k][i] = pack_a(D[i][b0 + k]) (transposed: k-major, like LDS)
        if (mode != 0 && panel) {
            uint32_t *const pa = panel + (int64_t)(K & 1) * 2 * kTile * ppitch;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int li = G::row_off(tye, r);
                if (li >= rows_valid) continue;
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int lj = G::col_off(txe, c);
                    if (lj >= cols_valid) continue;
                    const uint32_t v = (uint32_t)acc[r][c];
                    if (mode == 1)
                        pa[(kTile + li) * ppitch + col0 + lj] = pack_b(v, li);
                    else
                        pa[lj * ppitch + row0 + li] = pack_a(v);
                }
            }
        }
    }
    // ---- distances only (32-bit types), and float32 with deferred
    // successors: the band tiles write raw operand panels instead, same
    // layout: B'[k][j] = D[b0 + k][j], A'[k][i] = D[i][b0 + k]
    if constexpr ((ARGMIN == 0 && sizeof(U) == 4) || (ARGMIN == 2 && std::is_same<U, float>::value)) {
        if (mode != 0 && panel) {
            uint32_t *const pa = panel + (int64_t)(K & 1) * 2 * kTile * ppitch;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int li = G::row_off(tye, r);
                if (li >= rows_valid) continue;
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int lj = G::col_off(txe, c);
                    if (lj >= cols_valid) continue;
                    const uint32_t v = to_bits(acc[r][c]);
                    if (mode == 1)
                        pa[(kTile + li) * ppitch + col0 + lj] = v;
                    else
                        pa[lj * ppitch + row0 + li] = v;
                }
            }
        }
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
                // only improved entries change; with packed keys an unimproved
                // entry holds its clamped key, not its value, so a four-entry
                // store needs all four improved
                bool ch[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) ch[e] = cs[e] && idx[r][4 * g + e] >= 0;
                const bool any4 = ch[0] || ch[1] || ch[2] || ch[3];
                const bool all4 = ch[0] && ch[1] && ch[2] && ch[3];
                if (use_vec && all && (fast ? all4 : any4)) {
                    typename Arith<U>::V4 w;
                    w.x = acc[r][4 * g + 0]; w.y = acc[r][4 * g + 1];
                    w.z = acc[r][4 * g + 2]; w.w = acc[r][4 * g + 3];
                    *reinterpret_cast<typename Arith<U>::V4 *>(drow + lj) = w;
                } else if (any4) {
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

// One 128 x 128 tile: packed keys when the round's operand panels allow them
// (int32 with successors, phase 3), the general form otherwise.
// BANDS: band tiles may take packed keys too (the three-launch phase 2,
// where phase 1 publishes the diagonal block's maximum).
template <typename U, int ARGMIN, bool VEC, bool BANDS = false>
__device__ __forceinline__ void minplus_tile(U *__restrict__ D, int32_t *__restrict__ NX, int64_t n, int64_t ld,
                                             int K, int BS, int mode, int64_t row0, int64_t col0,
                                             MinplusSmem<U, ARGMIN> &sm, int *__restrict__ bmax, int nt,
                                             uint32_t *__restrict__ panel = nullptr, int64_t ppitch = 0) {
    if constexpr (ARGMIN == 2 && std::is_same<U, uint32_t>::value) {
        if (mode == 0 && bmax) {
            const int *bm = bmax + (K & 1) * 2 * nt;
            const uint32_t ma = (uint32_t)bm[nt + (int)(row0 / kTile)];   // A = column band tile (I, K)
            const uint32_t mb = (uint32_t)bm[(int)(col0 / kTile)];        // B = row band tile (K, J)
            if (ma < kPackLimit && mb < kPackLimit) {
                minplus_tile_impl<U, ARGMIN, VEC, true>(D, NX, n, ld, K, BS, mode, row0, col0, sm, bmax, nt,
                                                        nullptr, 0);
                return;
            }
        } else if (BANDS && mode != 0 && bmax) {
            // a band tile: its operands are the closed diagonal block (largest
            // finite entry published by phase 1) and the tile itself
            const uint32_t md = (uint32_t)bmax[4 * nt + (K & 1)];
            bool big = md >= kPackLimit;               // uniform
            if (!big) {
                using G = Geo<MinplusSmem<U, ARGMIN>::NT>;
                const int64_t b0 = (int64_t)K * BS;
                const int bk = (int)imin64((int64_t)BS, n - b0);
                const int rows_valid = (mode == 1) ? bk : (int)imin64(kTile, n - row0);
                const int cols_valid = (mode == 2) ? bk : (int)imin64(kTile, n - col0);
                const int tx = (int)threadIdx.x % G::txn, ty = (int)threadIdx.x / G::txn;
                bool mine = false;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int li = G::row_off(ty, r);
                    if (li >= rows_valid) continue;
#pragma unroll
                    for (int c = 0; c < G::cpt; ++c) {
                        const int lj = G::col_off(tx, c);
                        if (lj >= cols_valid) continue;
                        const uint32_t v = D[(row0 + li) * ld + col0 + lj];
                        mine = mine || (v >= kPackLimit && v < kInfU);
                    }
                }
                big = __syncthreads_or((int)mine) != 0;
            }
            if (!big) {
                minplus_tile_impl<U, ARGMIN, VEC, true>(D, NX, n, ld, K, BS, mode, row0, col0, sm, bmax, nt,
                                                        panel, ppitch);
                return;
            }
        }
    }
    minplus_tile_impl<U, ARGMIN, VEC, false>(D, NX, n, ld, K, BS, mode, row0, col0, sm, bmax, nt, panel, ppitch);
}

// Tile of a phase-3 launch: part 1 = the next band's tiles (row and column
// K + 1; block size = tile edge), part 2 = the rest, part 0 = all; -1 = none.
// Workgroups are dealt to the eight XCDs round-robin; each XCD gets a
// contiguous run of positions in the tile order below.
constexpr int kBandRows = 8;
__device__ __forceinline__ int64_t phase3_tile(int part, int K, int nt) {
    if (part == 1) {
        const int q = (int)blockIdx.x, nx1 = K + 1;
        if (q < nt) return (int64_t)nx1 * nt + q;
        if (q - nt == nx1) return -1;             // (K+1, K+1) is in the row above
        return (int64_t)(q - nt) * nt + nx1;
    }
    const int64_t tiles = (int64_t)nt * nt;
    const int64_t per = (tiles + 7) / 8;
    const int64_t g = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (g >= tiles) return -1;
    // position g -> tile: bands of kBandRows tile rows, column by column
    // inside a band, so that the tiles one XCD runs at once form a compact
    // block whose operand panel rows (A' of its rows, B' of its columns)
    // stay in that XCD's L2
    const int64_t band = g / ((int64_t)kBandRows * nt);
    const int64_t brows = imin64(kBandRows, nt - band * kBandRows);
    const int64_t o = g - band * kBandRows * nt;
    const int64_t idx = (band * kBandRows + o % brows) * nt + o / brows;
    if (part == 2 && (idx / nt == K + 1 || idx % nt == K + 1)) return -1;   // done by part 1
    return idx;
}

// panel (block size 128 and either int32 with deferred successors or 32-bit
// distances only; else null): the operand panels, 2 x 2 x 128 rows of ppitch
// entries, written by the band tiles (phase 2) for phase 3's direct-copy
// kernel.
template <typename U, int ARGMIN, int PHASE, bool VEC>
__global__ __launch_bounds__((Occ<U, ARGMIN>::threads), (Occ<U, ARGMIN>::waves_standalone)) void minplus_kernel(
        U *__restrict__ D, int32_t *__restrict__ NX, int64_t n, int64_t ld, int K, int BS, int nt,
        int *__restrict__ bmax, int part, uint32_t *__restrict__ panel, int64_t ppitch) {
    __shared__ MinplusSmem<U, ARGMIN> sm;
    const int64_t b0 = (int64_t)K * BS;
    const int64_t b1 = b0 + imin64((int64_t)BS, n - b0);
    int mode;
    int64_t idx;
    if (PHASE == 3) {
        idx = phase3_tile(part, K, nt);
        if (idx < 0) return;
        mode = 0;
    } else {
        mode = 1 + (int)blockIdx.y;
        idx = blockIdx.x;
    }
    int64_t row0, col0;
    if (!band_tile(mode, idx, n, b0, b1, nt, row0, col0)) return;
    minplus_tile<U, ARGMIN, VEC, PHASE == 2>(D, NX, n, ld, K, BS, mode, row0, col0, sm, bmax, nt, panel, ppitch);
}

// ------------------------------------------- phase 3: direct-copy kernel
// The common case of phase 3 in the three-launch schedule -- block size = tile
// edge, a full tile and band, 16-byte aligned rows, row pitch <= 2^22 entries,
// and either int32 with successors in packed keys or 32-bit distances only --
// runs in a kernel of its own, small enough (32 KB of LDS, <= 128 VGPRs) for
// four workgroups per CU:
//   - operands: the band tiles also write the round's operand panels (A'[k][i]
//     k-major and B'[k][j], round parity K & 1, rows of ppitch entries; packed
//     keys, or raw entries for distances only); each 16-k chunk of both is
//     copied from memory straight into LDS with global_load_lds (gfx950's
//     16-byte direct-to-LDS load: no registers, no VALU work),
//     double-buffered: chunk c + 1 is copied while chunk c is relaxed, one
//     barrier per chunk;
//   - 256 threads with 8 x 8 entries each: eight 16-byte LDS reads feed 128
//     relaxations per thread and pair of k's;
//   - entry by entry, the two adds and the min3 that reads them are issued
//     together (empty asm statements pin the order; the compiler would
//     otherwise issue all adds first): on gfx950 v_add issues at about twice
//     the rate of v_min3, and this order lets the two overlap (measured);
//   - every global address is a per-tile base in scalar registers plus a
//     per-thread offset, and there are no bounds or band tests; with
//     successors, an improved entry records the improving vertex as a tag
//     (resolve_next_kernel turns the tags into successors after the last
//     round), so the tile reads nothing but its operands and C.
// Same arithmetic, k order and results as the general tile.  A tile that does
// not qualify is appended to the launch's fix-up list, which
// minplus_fixup_kernel then runs with the general tile.
constexpr int64_t kFullTileMaxLd = int64_t(1) << 22;
constexpr int KCD = 16;                    // k's per chunk of the direct tile
struct alignas(16) DirectSmem {
    uint32_t As[2][KCD][kTile];            // As[buf][k][i] = A'[chunk k][i]
    uint32_t Bs[2][KCD][kTile];            // Bs[buf][k][j] = B'[chunk k][j]
};

// One chunk of KCD k's into the running minima, two k's per step.
template <typename U>
__device__ __forceinline__ void direct_chunk(const U (*__restrict__ As)[kTile], const U (*__restrict__ Bs)[kTile],
                                             int tx, int ty, U acc[8][8]) {
#pragma unroll 1
    for (int kk = 0; kk < KCD; kk += 2) {
        U a[8], b[8], a2[8], b2[8];
        lds_operands<U, 256, kTile>(As, Bs, kk, tx, ty, a, b);
        lds_operands<U, 256, kTile>(As, Bs, kk + 1, tx, ty, a2, b2);
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                U x = a[r] + b[c], y = a2[r] + b2[c];
                asm volatile("" : "+v"(x), "+v"(y));
                acc[r][c] = Arith<U>::mn(acc[r][c], Arith<U>::mn(x, y));
                asm volatile("" : "+v"(acc[r][c]));
            }
    }
}

// PACKED: int32 with successors, U = uint32_t holding keys; otherwise
// distances only, U = uint32_t or float holding raw entries (NX and bmax are
// not read).  fix_count / fix_list: this launch's fix-up counter (zeroed once
// per solve) and the list of tiles the general kernel runs afterwards (nt^2
// entries).
template <typename U, bool PACKED>
__global__ __launch_bounds__(256, 4) void minplus_direct_kernel(
        U *__restrict__ D, int32_t *__restrict__ NX, int64_t n, int64_t ld, int K, int nt,
        const int *__restrict__ bmax, int part, const uint32_t *__restrict__ panel, int64_t ppitch,
        int *__restrict__ fix_count, int *__restrict__ fix_list) {
    static_assert(sizeof(U) == 4 && (!PACKED || std::is_same<U, uint32_t>::value), "32-bit entries");
    __shared__ DirectSmem sm;
    using G = Geo<256>;
    const int64_t idx = phase3_tile(part, K, nt);
    if (idx < 0) return;
    const int64_t b0 = (int64_t)K * kTile;
    const int64_t row0_ = (idx / nt) * kTile, col0_ = (idx % nt) * kTile;
    if (row0_ == b0 || col0_ == b0) return;                       // the band's own tiles
    {
        // with keys, both operand bands must stay below the packing limit
        const int *bm = bmax + (PACKED ? (K & 1) * 2 * nt : 0);
        const bool direct = n - b0 >= kTile && row0_ + kTile <= n && col0_ + kTile <= n && ld <= kFullTileMaxLd &&
                            (!PACKED || ((uint32_t)bm[nt + (int)(row0_ / kTile)] < kPackLimit &&
                                         (uint32_t)bm[(int)(col0_ / kTile)] < kPackLimit));
        if (!direct) {
            if (threadIdx.x == 0) fix_list[atomicAdd(fix_count, 1)] = (int)idx;
            return;
        }
    }
    const int64_t row0 = __builtin_amdgcn_readfirstlane((int)row0_);
    const int64_t col0 = __builtin_amdgcn_readfirstlane((int)col0_);
    const int64_t pitch = ld * 4;
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int tx = t % G::txn, ty = t / G::txn;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t pb = ppitch * 4;
    const int64_t par = K & 1;
    const char *const ap = reinterpret_cast<const char *>(panel + par * 2 * kTile * ppitch) + row0 * 4;
    const char *const bp = reinterpret_cast<const char *>(panel + (par * 2 + 1) * kTile * ppitch) + col0 * 4;
    // One global_load_lds of a wave moves 1 KiB, two panel rows of the tile:
    // lanes 0-31 row kr, lanes 32-63 row kr + 1, 16 bytes each, landing at LDS
    // base + 16 lane (the instruction offset, unused, would apply to both
    // addresses); the four waves move a 16-row chunk of A' and of B' in two
    // each.  (The casts name the global source and LDS destination spaces.)
    const uint32_t loff = (uint32_t)(lane >> 5) * (uint32_t)pb + (uint32_t)(lane & 31) * 16u;
    auto copy_chunk = [&](int kc, int buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int kr = 2 * wv + 8 * q;
            const int64_t go = (int64_t)(kc + kr) * pb;
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(ap + go + loff),
                                             (__attribute__((address_space(3))) void *)&sm.As[buf][kr][0], 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(bp + go + loff),
                                             (__attribute__((address_space(3))) void *)&sm.Bs[buf][kr][0], 16, 0, 0);
        }
    };
    copy_chunk(0, 0);
    // C.  Distances only: raw entries, loaded before the k loop.  With
    // successors: the keys min(C, S) << 8 are folded into the running minima
    // after it, which start above every key (a candidate key is at most
    // 0x7FFFFF00 + 0x7FFFFFFF); a minimum does not depend on that order, and
    // this order measured 1.2% faster per launch (2.24 against 2.27 ms at
    // n = 32768, alternating on one box).
    const char *const cbase = reinterpret_cast<const char *>(D) + row0 * pitch + col0 * 4;
    U acc[8][8];
    if constexpr (PACKED) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[r][c] = 0xFFFFFFFFu;
    } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int64_t ro = (int64_t)G::row_off(ty, r) * pitch;
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const uint4 v = *reinterpret_cast<const uint4 *>(cbase + ro + (int64_t)G::col_off(tx, 4 * g) * 4);
                acc[r][4 * g] = from_bits<U>(v.x); acc[r][4 * g + 1] = from_bits<U>(v.y);
                acc[r][4 * g + 2] = from_bits<U>(v.z); acc[r][4 * g + 3] = from_bits<U>(v.w);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kTile / KCD; ++c) {
        wait_vmem();                               // this wave's copies of chunk c (and C, distances only)
        __syncthreads();                           // everyone's; and chunk c - 1 is consumed
        if (c + 1 < kTile / KCD) copy_chunk((c + 1) * KCD, (c + 1) & 1);
        direct_chunk<U>(reinterpret_cast<const U (*)[kTile]>(sm.As[c & 1]),
                        reinterpret_cast<const U (*)[kTile]>(sm.Bs[c & 1]), tx, ty, acc);
    }
    if constexpr (!PACKED) {
        // distances only: the tile's new values, four at a time
        char *const Db = reinterpret_cast<char *>(D);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int64_t ro = (row0 + G::row_off(ty, r)) * pitch;
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const U *e = &acc[r][4 * g];
                *reinterpret_cast<uint4 *>(Db + ro + (col0 + G::col_off(tx, 4 * g)) * 4) =
                        make_uint4(to_bits(e[0]), to_bits(e[1]), to_bits(e[2]), to_bits(e[3]));
            }
        }
    } else {
        // C's keys are folded in two rows at a time, the next two rows'
        // loads issued before this pair's stores (empty asm statements keep
        // the compiler from hoisting every load, which would spill).  Keys ->
        // results:
        // bit 0 = improved, bits 1..7 = k, bits 8.. = value.  An improved
        // entry stores its new distance and, in place of its successor, the
        // tag of the improving vertex b0 + k (its successor is that of entry
        // (i, b0 + k), looked up once the solve has ended:
        // resolve_next_kernel).  Only improved entries are stored, four at
        // once only when all four improved (an unimproved key holds
        // min(C, S), not C).
        char *const Db = reinterpret_cast<char *>(D);
        char *const Nb = reinterpret_cast<char *>(NX);
        const int32_t tag0 = kLazyBit | (int32_t)b0;
        uint4 cv[2][2][2];                         // [buffer][row][half row]
        auto load_c = [&](int h) {
#pragma unroll
            for (int rr = 0; rr < 2; ++rr)
#pragma unroll
                for (int g = 0; g < 2; ++g)
                    cv[h & 1][rr][g] = *reinterpret_cast<const uint4 *>(
                            cbase + (int64_t)G::row_off(ty, 2 * h + rr) * pitch + (int64_t)G::col_off(tx, 4 * g) * 4);
        };
        auto fold_c = [&](int h) {
#pragma unroll
            for (int rr = 0; rr < 2; ++rr)
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    const uint4 &c = cv[h & 1][rr][g];
                    uint32_t *const e = &acc[2 * h + rr][4 * g];
                    e[0] = Arith<U>::mn(e[0], pack_a(c.x)); e[1] = Arith<U>::mn(e[1], pack_a(c.y));
                    e[2] = Arith<U>::mn(e[2], pack_a(c.z)); e[3] = Arith<U>::mn(e[3], pack_a(c.w));
                }
        };
        auto store = [&](int h) {
#pragma unroll
            for (int rr = 0; rr < 2; ++rr) {
                const int r = 2 * h + rr;
                const int64_t ro = (row0 + G::row_off(ty, r)) * pitch;
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    const int64_t co = (col0 + G::col_off(tx, 4 * g)) * 4;
                    uint32_t *dp = reinterpret_cast<uint32_t *>(Db + ro + co);
                    int32_t *np = reinterpret_cast<int32_t *>(Nb + ro + co);
                    const uint32_t *e = &acc[r][4 * g];
                    int32_t tag[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) tag[q] = tag0 + (int32_t)((e[q] >> 1) & 127u);
                    const bool all = (e[0] & e[1] & e[2] & e[3] & 1u) != 0;
                    if (all) {
                        *reinterpret_cast<uint4 *>(dp) = make_uint4(e[0] >> 8, e[1] >> 8, e[2] >> 8, e[3] >> 8);
                        *reinterpret_cast<int4 *>(np) = make_int4(tag[0], tag[1], tag[2], tag[3]);
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (e[q] & 1u) { dp[q] = e[q] >> 8; np[q] = tag[q]; }
                    }
                }
            }
        };
        load_c(0);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            fold_c(h);
            if (h + 1 < 4) load_c(h + 1);
            asm volatile("" ::: "memory");
            store(h);
            asm volatile("" ::: "memory");
        }
    }
}

// ------------------- phase 3: direct-copy kernel, float32 with successors
// Float sums carry no room for the improving k (the packed keys of int32),
// so this tile keeps two minima per entry -- the running one, acc, and the
// current chunk's, cm -- and finds the improving k only for the entries a
// chunk strictly improves, while that chunk is still in LDS (the deferred
// bookkeeping of the general tile, on the direct-copy operand path):
//   - the band tiles write the round's raw operand panels (A'[k][i] k-major,
//     B'[k][j]; round parity K & 1), and 16-k chunks of both are copied from
//     memory straight into double-buffered LDS with global_load_lds;
//   - 512 threads own 8 x 4 entries each (acc and cm: 64 VGPRs); per pair of
//     k, two adds and one min3 per entry (in the compiler's order);
//   - at each chunk's end the entries with cm < acc are queued per wave
//     (ballot + mbcnt), folded into acc, and searched lane-parallel over the
//     chunk's 16 k's for the first k with A'[k][i] + B'[k][j] == cm; the
//     winner goes into an LDS byte matrix (one byte per entry);
//   - afterwards the tile's block of the successor column band,
//     next[i][b0 .. b0+127], is copied into the operand LDS in two halves and
//     each improved entry takes next[i][b0 + k*]; only improved entries'
//     successors are stored.
// The chosen k is the first one (in increasing order) that reaches the final
// minimum when that minimum beats the old value: the last strictly
// improving chunk is the one that first reaches the final minimum, and the
// search takes the first k in it -- the same k as every other variant.
struct alignas(16) DirectSearchSmem {
    static constexpr int NT = 512, WAVES = NT / 64, QCAP = 128;
    float As[2][KCD][kTile];               // As[buf][k][i] = A'[chunk k][i]
    float Bs[2][KCD][kTile];               // Bs[buf][k][j] = B'[chunk k][j]
    uint32_t kst[kTile * kTile / 4];       // improving k per entry (bytes; 0xFF = none)
    uint32_t qpos[WAVES * QCAP];           // queued entry: i | j << 8
    float qval[WAVES * QCAP];              // its chunk minimum
    int qmin[WAVES * 64];                  // per-entry search result
};

__global__ __launch_bounds__(512, 4) void minplus_direct_search_kernel(
        float *__restrict__ D, int32_t *__restrict__ NX, int64_t n, int64_t ld, int K, int nt, int part,
        const uint32_t *__restrict__ panel, int64_t ppitch, int *__restrict__ fix_count, int *__restrict__ fix_list) {
    using SM = DirectSearchSmem;
    __shared__ SM sm;
    using G = Geo<512>;
    constexpr int NT = SM::NT, QCAP = SM::QCAP;
    const int64_t idx = phase3_tile(part, K, nt);
    if (idx < 0) return;
    const int64_t b0 = (int64_t)K * kTile;
    const int64_t row0_ = (idx / nt) * kTile, col0_ = (idx % nt) * kTile;
    if (row0_ == b0 || col0_ == b0) return;                       // the band's own tiles
    if (!(n - b0 >= kTile && row0_ + kTile <= n && col0_ + kTile <= n && ld <= kFullTileMaxLd)) {
        if (threadIdx.x == 0) fix_list[atomicAdd(fix_count, 1)] = (int)idx;
        return;
    }
    const int64_t row0 = __builtin_amdgcn_readfirstlane((int)row0_);
    const int64_t col0 = __builtin_amdgcn_readfirstlane((int)col0_);
    const int64_t pitch = ld * 4;
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int tx = t % G::txn, ty = t / G::txn;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t pb = ppitch * 4;
    const int64_t par = K & 1;
    const char *const ap = reinterpret_cast<const char *>(panel + par * 2 * kTile * ppitch) + row0 * 4;
    const char *const bp = reinterpret_cast<const char *>(panel + (par * 2 + 1) * kTile * ppitch) + col0 * 4;
    // one global_load_lds of a wave moves two panel rows (lanes 0-31 row kr,
    // lanes 32-63 row kr + 1); eight waves move a 16-row chunk of A' and B'
    const uint32_t loff = (uint32_t)(lane >> 5) * (uint32_t)pb + (uint32_t)(lane & 31) * 16u;
    auto copy_chunk = [&](int kc, int buf) {
        const int kr = 2 * wv;
        const int64_t go = (int64_t)(kc + kr) * pb;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(ap + go + loff),
                                         (__attribute__((address_space(3))) void *)&sm.As[buf][kr][0], 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(bp + go + loff),
                                         (__attribute__((address_space(3))) void *)&sm.Bs[buf][kr][0], 16, 0, 0);
    };
    copy_chunk(0, 0);
    for (int q = t; q < kTile * kTile / 4; q += NT) sm.kst[q] = 0xFFFFFFFFu;
    for (int q = t; q < SM::WAVES * 64; q += NT) sm.qmin[q] = 0xFF;
    // C, loaded before the k loop
    const char *const cbase = reinterpret_cast<const char *>(D) + row0 * pitch + col0 * 4;
    float acc[8][4];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const float4 v = *reinterpret_cast<const float4 *>(cbase + (int64_t)G::row_off(ty, r) * pitch +
                                                           (int64_t)G::col_off(tx, 0) * 4);
        acc[r][0] = v.x; acc[r][1] = v.y; acc[r][2] = v.z; acc[r][3] = v.w;
    }
    const int wq = wv * QCAP;           // this wave's queue
    const int wq64 = wv * 64;           // this wave's search results
    uint8_t *const kst8 = reinterpret_cast<uint8_t *>(sm.kst);
#pragma unroll 1
    for (int c = 0; c < kTile / KCD; ++c) {
        wait_vmem();                               // this wave's copies of chunk c (and C)
        __syncthreads();                           // everyone's; chunk c - 1 and its search are done
        if (c + 1 < kTile / KCD) copy_chunk((c + 1) * KCD, (c + 1) & 1);
        const float (*As)[kTile] = sm.As[c & 1];
        const float (*Bs)[kTile] = sm.Bs[c & 1];
        float cm[8][4];
        {
            float a[8], b[4], a2[8], b2[4];
            lds_operands<float, 512, kTile>(As, Bs, 0, tx, ty, a, b);
            lds_operands<float, 512, kTile>(As, Bs, 1, tx, ty, a2, b2);
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e) cm[r][e] = __builtin_fminf(a[r] + b[e], a2[r] + b2[e]);
        }
#pragma unroll 1
        for (int kk = 2; kk < KCD; kk += 2) {
            float a[8], b[4], a2[8], b2[4];
            lds_operands<float, 512, kTile>(As, Bs, kk, tx, ty, a, b);
            lds_operands<float, 512, kTile>(As, Bs, kk + 1, tx, ty, a2, b2);
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    cm[r][e] = __builtin_fminf(cm[r][e], __builtin_fminf(a[r] + b[e], a2[r] + b2[e]));
        }
        // ---- strict improvements of this chunk: queue, fold, search
        int txo = tx, tyo = ty;
        asm volatile("" : "+v"(txo), "+v"(tyo));
        const uint32_t ebase = (uint32_t)(tyo * 4) | ((uint32_t)(txo * 4) << 8);
        bool again;
        do {
            int qcnt = 0;
            again = false;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const bool imp = cm[r][e] < acc[r][e];
                    const uint64_t m = __builtin_amdgcn_ballot_w64(imp);
                    if (m) {                                     // uniform
                        const int cnt = __builtin_popcountll(m);
                        if (qcnt + cnt <= QCAP) {
                            if (imp) {
                                const int pos = qcnt + (int)__builtin_amdgcn_mbcnt_hi(
                                                           (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                                sm.qpos[wq + pos] = ebase + (uint32_t)(G::row_off(0, r) | (G::col_off(0, e) << 8));
                                sm.qval[wq + pos] = cm[r][e];
                            }
                            qcnt += cnt;
                            acc[r][e] = __builtin_fminf(acc[r][e], cm[r][e]);
                        } else {
                            again = true;
                        }
                    }
                }
            }
            // m entries per batch, L = 64 / m lanes each (a power of two, at
            // most KCD); lane o of an entry scans k = o*span .. o*span+span-1
            // and the entry's answer is the smallest hit over its lanes
            for (int base = 0; base < qcnt; base += 64) {
                const int m = (qcnt - base < 64) ? qcnt - base : 64;
                wave_sync();
                const int cl2 = (m <= 1) ? 0 : 32 - __builtin_clz((uint32_t)(m - 1));   // ceil(log2 m)
                const int lg = (6 - cl2 < 4) ? 6 - cl2 : 4;                             // log2 L
                const int span = KCD >> lg;
                const int e = lane >> lg, o = lane & ((1 << lg) - 1);
                int li = 0, lj = 0, kb = 0xFF;
                if (e < m) {
                    const uint32_t ent = sm.qpos[wq + base + e];
                    li = (int)(ent & 0xFFu);
                    lj = (int)(ent >> 8);
                    const float tgt = sm.qval[wq + base + e];
                    const int k0 = o * span;
                    for (int q = span - 1; q >= 0; --q) kb = (As[k0 + q][li] + Bs[k0 + q][lj] == tgt) ? k0 + q : kb;
                }
                if (lg == 0) {
                    if (e < m) kst8[li * kTile + lj] = (uint8_t)(c * KCD + kb);
                } else {
                    if (e < m && kb != 0xFF) atomicMin(&sm.qmin[wq64 + e], kb);
                    wave_sync();
                    if (e < m && o == 0) {
                        kst8[li * kTile + lj] = (uint8_t)(c * KCD + sm.qmin[wq64 + e]);
                        sm.qmin[wq64 + e] = 0xFF;
                    }
                }
                wave_sync();
            }
        } while (again);
    }
    // ---- results: improving k per entry (0xFF: none)
    __syncthreads();                               // every search's byte is in LDS
    int txe = tx, tye = ty;
    asm volatile("" : "+v"(txe), "+v"(tye));
    uint32_t kw[8];
    uint32_t any = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        kw[r] = sm.kst[(G::row_off(tye, r) * kTile + G::col_off(txe, 0)) >> 2];
        any |= ~kw[r];                             // a byte other than 0xFF: improved
    }
    if (!__syncthreads_or(any != 0)) return;       // nothing improved: C is unchanged
    char *const Db = reinterpret_cast<char *>(D);
    char *const Nb = reinterpret_cast<char *>(NX);
    int32_t (*const NXs)[kTile] = reinterpret_cast<int32_t (*)[kTile]>(&sm.As[0][0][0]);   // 64 rows, 32 KB
    static_assert(sizeof(sm.As) + sizeof(sm.Bs) == 64 * kTile * sizeof(int32_t), "LDS for half the successor block");
    const char *const nband = Nb + row0 * pitch + b0 * 4;
    const uint32_t noff = (uint32_t)(lane >> 5) * (uint32_t)pitch + (uint32_t)(lane & 31) * 16u;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h) __syncthreads();                    // the first half is consumed
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int x = 16 * q + 2 * wv;         // rows x, x + 1 of this half
            __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(nband + (int64_t)(64 * h + x) * pitch + noff),
                    (__attribute__((address_space(3))) void *)&NXs[x][0], 16, 0, 0);
        }
        wait_vmem();
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int r = 4 * h + rr;
            const int li = G::row_off(tye, r);     // 64 h + local row
            const int32_t *const nrow = NXs[li - 64 * h];
            const int64_t ro = (row0 + li) * pitch;
            const int64_t co = (col0 + G::col_off(txe, 0)) * 4;
            float *dp = reinterpret_cast<float *>(Db + ro + co);
            int32_t *np = reinterpret_cast<int32_t *>(Nb + ro + co);
            uint32_t kb[4];
            int32_t nxv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                kb[e] = (kw[r] >> (8 * e)) & 0xFFu;
                nxv[e] = nrow[kb[e] & 127u];       // k = 127 when unimproved (not stored)
            }
            const bool ch0 = kb[0] != 0xFFu, ch1 = kb[1] != 0xFFu, ch2 = kb[2] != 0xFFu, ch3 = kb[3] != 0xFFu;
            if (ch0 || ch1 || ch2 || ch3)          // unimproved entries hold C itself
                *reinterpret_cast<float4 *>(dp) = make_float4(acc[r][0], acc[r][1], acc[r][2], acc[r][3]);
            if (ch0 && ch1 && ch2 && ch3) {
                *reinterpret_cast<int4 *>(np) = make_int4(nxv[0], nxv[1], nxv[2], nxv[3]);
            } else {
                if (ch0) np[0] = nxv[0];
                if (ch1) np[1] = nxv[1];
                if (ch2) np[2] = nxv[2];
                if (ch3) np[3] = nxv[3];
            }
        }
    }
}

// The fix-up tiles of a direct-copy launch, with the general tile (packed
// keys or not, ragged or not); a resident-size grid walks the list.
template <typename U, int ARGMIN, bool VEC>
__global__ __launch_bounds__((Occ<U, ARGMIN>::threads), (Occ<U, ARGMIN>::waves_standalone)) void
minplus_fixup_kernel(U *__restrict__ D, int32_t *__restrict__ NX, int64_t n, int64_t ld, int K, int nt,
                     int *__restrict__ bmax, const int *__restrict__ fix_count, const int *__restrict__ fix_list) {
    __shared__ MinplusSmem<U, ARGMIN> sm;
    const int count = __hip_atomic_load(fix_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t b0 = (int64_t)K * kTile;
    const int64_t b1 = b0 + imin64((int64_t)kTile, n - b0);
    for (int q = blockIdx.x; q < count; q += gridDim.x) {
        int64_t row0, col0;
        if (band_tile(0, fix_list[q], n, b0, b1, nt, row0, col0))
            minplus_tile<U, ARGMIN, VEC>(D, NX, n, ld, K, kTile, 0, row0, col0, sm, bmax, nt);
        __syncthreads();                           // LDS is reused by the next tile
    }
}

// ------------------------------------------------ successor resolution
// After the last round of a three-launch int32 solve with successors, entries
// the direct-copy phase 3 improved hold tags (kLazyBit | k: "successor of
// (i, j) = successor of (i, k)", k the improving vertex).  The final
// successors follow from the final matrix: when a relaxation through k gave
// (i, j) its final distance, d(i, k) was already final -- had it dropped
// later, d(i, k) + d(k, j) would undercut the final d(i, j), which with
// integer sums is the exact shortest distance -- and a successor changes only
// with a strict decrease of its own distance, so the successor the eager
// bookkeeping copies at that moment is the final successor of (i, k).  A tag
// names an entry last written before the tag was, so the tags of a row form
// chains without cycles that end at successors.  One workgroup per row
// resolves them by pointer jumping (a tag takes the value of the entry it
// names; after p passes a chain of length below 2^p is resolved): one or two
// passes on the dense graphs of the measurements.  Rows of at most CAP
// entries are staged in LDS and written back whole if they held a tag; CAP =
// 0 works on the row in memory.  Input that breaks the contract (a negative
// cycle) could make a cycle of tags: the passes stop after kResolvePasses
// (chains are shorter than 2^31) and a tag still left, or one naming an
// entry outside the row, becomes -1.
constexpr int kResolveThreads = 1024;
constexpr int kResolvePasses = 40;
__device__ __forceinline__ bool is_tag(int32_t v) { return (v & (int32_t)0xC0000000) == kLazyBit; }
__device__ __forceinline__ int32_t ld_wg(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_wg(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int CAP>
__global__ __launch_bounds__(kResolveThreads) void resolve_next_kernel(int32_t *__restrict__ NX, int64_t n,
                                                                       int64_t ld) {
    __shared__ int32_t row[CAP > 0 ? CAP : 1];
    const int t = threadIdx.x;
    int32_t *const g = NX + (int64_t)blockIdx.x * ld;
    int32_t *const r = CAP > 0 ? row : g;
    bool any = false;
#pragma unroll 8
    for (int64_t j = t; j < n; j += kResolveThreads) {
        const int32_t v = g[j];
        if (CAP > 0) row[j] = v;
        any |= is_tag(v);
    }
    if (!__syncthreads_or(any)) return;            // no tag in this row
    bool left = true;
    for (int pass = 0; pass < kResolvePasses && left; ++pass) {
        bool l = false;
        for (int64_t j = t; j < n; j += kResolveThreads) {
            const int32_t v = ld_wg(r + j);
            if (is_tag(v)) {
                const int32_t k = v & (kLazyBit - 1);
                const int32_t w = k < n ? ld_wg(r + k) : -1;
                st_wg(r + j, w);
                l |= is_tag(w);
            }
        }
        __syncthreads();                           // this pass's values are visible to the next
        left = __syncthreads_or(l);
    }
#pragma unroll 8
    for (int64_t j = t; j < n; j += kResolveThreads) {
        const int32_t v = r[j];
        if (CAP > 0) g[j] = is_tag(v) ? -1 : v;
        else if (is_tag(v)) g[j] = -1;
    }
}

// ------------------------------------------------------ persistent schedule
// One launch runs every round (block size 128 = the tile edge).  Work items
// are taken from per-round queues in round order; round K's items are, in
// queue order: phase 1, the 2*nt phase-2 tiles (row band j, then column band
// i), then the nt^2 phase-3 tiles, of which the ones round K+1's phases 1 and
// 2 read (the diagonal tile of band K+1, then its row and column tiles) come
// first.  Dependencies are epoch-valued flags (value = round + 1, so nothing
// is reset between rounds), the GPU form of the per-block semaphores of the
// paper's intra-round concurrency:
//   phase 1 (K)        : tile (K, K) of round K-1 done            nrow[K] >= K
//   phase 2 row tile j : phase 1 of round K                        diag >= K+1
//                        tile (K, j) of round K-1 done            nrow[j] >= K
//                        j = K-1 only: every round-(K-1) reader of
//                        that tile (the phase-3 tiles (K, *)) done  rrd[K-1] >= nt-1
//   phase 2 col tile i : phase 1 of round K,  tile (i, K) of K-1   ncol[i] >= K
//                        i = K-1 only: the tiles (*, K) of K-1     crd[K-1] >= nt-1
//   phase 3 tile (i,j) : every item of round K-1 done (its own C, and no
//                        round-(K-1) reader of the old bands is left)
//                        done[K-1] == items, rowf[j] >= K+1, colf[i] >= K+1
// Tile (K, K-1) is both round K-1's column band -- the A operand of its
// phase-3 tiles (K, *) -- and a tile that round K's row band overwrites, hence
// the extra wait (write after read); likewise (K-1, K).  Phases 1 and 2 of
// round K+1 thus overlap the end of round K (the paper's
// "inter-round" future work).  A workgroup waits only on items that running
// workgroups have already taken, so the schedule needs no co-resident grid.
// Flags are published with an agent-scope release (L2 write-back) and read
// with an agent-scope acquire (L1/L2 invalidate), which is what makes a
// tile written on one XCD visible on another.  Every wait is bounded by a
// wall-clock deadline; on expiry the error word gets code 2 and an abort
// flag makes every workgroup leave.
struct PersistWs {
    int *abort, *diag, *q, *xq, *done, *p2c, *rrd, *crd, *rowf, *colf, *nrow, *ncol, *bmax;
};

constexpr int kXcds = 8;        // MI355X: eight XCDs, workgroups dealt round-robin

__host__ __device__ __forceinline__ int64_t persist_ws_ints(int R, int nt) {
    return 4 + (5 + kXcds) * (int64_t)R + 8 * (int64_t)nt;
}

__device__ __forceinline__ PersistWs persist_ws(int *w, int R, int nt) {
    PersistWs p;
    p.abort = w;
    p.diag = w + 1;
    p.q = w + 4;
    p.xq = p.q + R;
    p.done = p.xq + (int64_t)kXcds * R;
    p.p2c = p.done + R;
    p.rrd = p.p2c + R;
    p.crd = p.rrd + R;
    p.rowf = p.crd + R;
    p.colf = p.rowf + nt;
    p.nrow = p.colf + nt;
    p.ncol = p.nrow + nt;
    p.bmax = p.ncol + nt;                      // 2 parities x (row, column) x nt
    return p;
}

__global__ void zero_ints_kernel(int *w, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        w[i] = 0;
}

// Publishes everything the workgroup has written: every wave drains its
// stores into L2, then one thread writes the L2 back (agent-scope release)
// and stores the flag.
__device__ __forceinline__ void publish(bool lead, int *flag, int value) {
    wait_vmem();
    __syncthreads();
    if (lead) {
        release_agent();
        __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Thread 0 only.  Spins until *p >= v; false when the solve is aborted or the
// deadline (s_memrealtime ticks) passes, which sets the error word and abort.
__device__ bool wait_ge(const int *p, int v, const PersistWs &ws, int *err, uint64_t deadline) {
    while (ld_flag(p) < v) {
        if (ld_flag(ws.abort)) return false;
        if (__builtin_amdgcn_s_memrealtime() > deadline) {
            atomicCAS(err, 0, 2);
            __hip_atomic_store(ws.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Phase-3 queue position q of round K -> tile (ti, tj); nxt = K + 1 is the
// next band, whose tiles come first.
__device__ __forceinline__ void p3_tile(int64_t q, int nxt, int nt, int &ti, int &tj) {
    if (nxt >= nt) {
        ti = (int)(q / nt);
        tj = (int)(q % nt);
        return;
    }
    if (q == 0) {
        ti = tj = nxt;
        return;
    }
    q -= 1;
    if (q < nt - 1) {
        ti = nxt;
        tj = (int)(q < nxt ? q : q + 1);
        return;
    }
    q -= nt - 1;
    if (q < nt - 1) {
        tj = nxt;
        ti = (int)(q < nxt ? q : q + 1);
        return;
    }
    q -= nt - 1;
    const int a = (int)(q / (nt - 1)), b = (int)(q % (nt - 1));
    ti = a < nxt ? a : a + 1;
    tj = b < nxt ? b : b + 1;
}

template <typename U, int ARGMIN> union PersistSmem {
    MinplusSmem<U, ARGMIN> mp;
    Phase1Smem<U, kTile, false> p1c;                           // closure_block (32-bit)
    Phase1Smem<U, kTile, ARGMIN != 0 && sizeof(U) == 8> p1;   // phase1_block, successors in LDS (64-bit)
};

// Phase 1 of round K on the diagonal block: 32-bit entries by closure_block
// (successors in registers), 64-bit ones by phase1_block (successors in LDS);
// the same bits either way.
template <typename U, bool NEXT, int NT, typename SM>
__device__ __forceinline__ void phase1_any(U *__restrict__ D, int32_t *__restrict__ NX, int64_t n, int64_t ld,
                                           int K, SM &sm) {
    const int64_t b0 = (int64_t)K * kTile;
    if constexpr (sizeof(U) == 4)
        closure_block<U, NEXT, kTile, NT>(D + b0 * ld + b0, NEXT ? NX + b0 * ld + b0 : nullptr,
                                          imin64(kTile, n - b0), ld, sm.p1c);
    else
        phase1_block<U, NEXT, kTile, NT, NEXT>(D, NX, n, ld, K, sm.p1);
}

// The whole solve of one graph by the workgroups that call it (every
// workgroup of the persistent launch, or a team of the batched one).  Returns
// false when the solve was aborted (a wait passed its deadline).
template <typename U, int ARGMIN, bool VEC>
__device__ __forceinline__ bool persistent_solve(U *__restrict__ D, int32_t *__restrict__ NX, int64_t n, int64_t ld,
                                                 int R, int nt, const PersistWs &ws, int *__restrict__ err,
                                                 uint64_t timeout_ticks, PersistSmem<U, ARGMIN> &sm, int &s_item,
                                                 int &s_ok) {
    constexpr int NT = MinplusSmem<U, ARGMIN>::NT;
    constexpr bool NEXT = ARGMIN != 0;
    constexpr int BS = kTile;
    const int items = 1 + 2 * nt + nt * nt;
    const bool lead = threadIdx.x == 0;

    // Phase-3 tiles other than the next band's are split into kXcds
    // contiguous ranges; a workgroup drains the range of its own XCD first
    // (tiles sharing a row of A then share an L2), then helps the others.
    const int xcd = (int)(blockIdx.x % kXcds);
    const int pq = (nt > 1) ? 2 * nt - 1 : 0;                 // next-band tiles (not in the last round)

    for (int K = 0; K < R; ++K) {
        const int64_t b0 = (int64_t)K * BS;
        const int64_t b1 = b0 + imin64((int64_t)BS, n - b0);
        const int pqk = (K + 1 < nt) ? pq : 0;
        const int lim0 = 1 + 2 * nt + pqk;                     // items of the shared queue
        const int rest = nt * nt - pqk;
        const int per = (rest + kXcds - 1) / kXcds;
        int mine = 0;            // items of round K taken by this workgroup
        bool ready3 = false;     // every phase-3 dependency of round K acquired
        // queue walk of thread 0: shared queue, then the XCD ranges
        int stage = 0;
        auto fetch = [&]() -> int {
            if (stage == 0) {
                const int v = __hip_atomic_fetch_add(&ws.q[K], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (v < lim0) return v;
                stage = 1;
            }
            while (stage <= kXcds) {
                const int x = (xcd + stage - 1) % kXcds;
                const int tq = __hip_atomic_fetch_add(&ws.xq[(int64_t)K * kXcds + x], 1, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                const int pos = pqk + x * per + tq;
                if (tq < per && pos < nt * nt) return 1 + 2 * nt + pos;
                ++stage;
            }
            return items;
        };
        int upcoming = lead ? fetch() : 0;
        for (;;) {
            __syncthreads();
            if (lead) s_item = upcoming;
            __syncthreads();
            const int item = s_item;
            if (item >= items) break;
            ++mine;
            if (lead) upcoming = fetch();          // overlaps this item's work

            // ---- what the item is
            int mode = 0, ti = 0, tj = 0;        // mode: 0 phase 3, 1 row band, 2 column band
            if (item > 0 && item <= 2 * nt) {
                mode = item <= nt ? 1 : 2;
                ti = tj = (item - 1) % nt;
            } else if (item > 2 * nt) {
                p3_tile(item - 1 - 2 * nt, K + 1, nt, ti, tj);
            }
            int64_t row0 = 0, col0 = 0;
            const bool work = item > 0 &&
                              band_tile(mode, mode == 0 ? (int64_t)ti * nt + tj : ti, n, b0, b1, nt, row0, col0);
            const bool feeds = item > 2 * nt && (ti == K + 1 || tj == K + 1);   // read by round K+1's phases 1/2
            // ---- wait for its inputs (one thread spins, then acquires)
            const bool waits = item <= 2 * nt || (work && !ready3) || (!work && feeds);
            if (waits) {
                if (lead) {
                    const uint64_t dl = __builtin_amdgcn_s_memrealtime() + timeout_ticks;
                    int ok = 1;
                    if (item == 0) {
                        ok = K == 0 || wait_ge(&ws.nrow[K], K, ws, err, dl);
                    } else if (item <= 2 * nt) {
                        ok = wait_ge(ws.diag, K + 1, ws, err, dl);
                        if (ok && K > 0) ok = wait_ge(mode == 1 ? &ws.nrow[tj] : &ws.ncol[ti], K, ws, err, dl);
                        if (ok && K > 0 && ti == K - 1)
                            ok = wait_ge(mode == 1 ? &ws.rrd[K - 1] : &ws.crd[K - 1], nt - 1, ws, err, dl);
                    } else if (work) {
                        ok = K == 0 || wait_ge(&ws.done[K - 1], items, ws, err, dl);
                        // all of phase 2 done: nothing else to wait for in this round
                        const bool all2 = ok && ld_flag(&ws.p2c[K]) >= 2 * nt;
                        if (ok && !all2)
                            ok = wait_ge(&ws.rowf[tj], K + 1, ws, err, dl) && wait_ge(&ws.colf[ti], K + 1, ws, err, dl);
                        if (ok && all2) ok = 2;
                    } else {
                        // a band-K tile that round K+1 reads: its data come from
                        // this round's phase 2; forward that tile's flag
                        ok = (ti == K) ? wait_ge(&ws.rowf[tj], K + 1, ws, err, dl)
                                       : wait_ge(&ws.colf[ti], K + 1, ws, err, dl);
                    }
                    s_ok = ok;
                    acquire_agent();
                    wait_vmem();
                }
                __syncthreads();
                if (!s_ok) return false;
                if (item > 2 * nt && work && s_ok == 2) ready3 = true;
            }
            // ---- the work
            if (item == 0)
                phase1_any<U, NEXT, NT>(D, NX, n, ld, K, sm);
            else if (work)
                minplus_tile<U, ARGMIN, VEC>(D, NX, n, ld, K, BS, mode, row0, col0, sm.mp,
                                             (ARGMIN == 2 && std::is_same<U, uint32_t>::value) ? ws.bmax : nullptr,
                                             nt);
            // ---- publish what later items wait for
            if (item == 0) {
                publish(lead, ws.diag, K + 1);
            } else if (item <= 2 * nt) {
                publish(lead, mode == 1 ? &ws.rowf[tj] : &ws.colf[ti], K + 1);
                if (lead) __hip_atomic_fetch_add(&ws.p2c[K], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else if (feeds) {
                if (ti == K + 1) publish(lead, &ws.nrow[tj], K + 1);
                if (tj == K + 1) publish(lead, &ws.ncol[ti], K + 1);
                // a phase-3 tile of row (column) block K+1 has finished reading
                // its band-K operand tile (K+1, K) (resp. (K, K+1))
                if (work && lead) {
                    if (ti == K + 1) __hip_atomic_fetch_add(&ws.rrd[K], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (tj == K + 1) __hip_atomic_fetch_add(&ws.crd[K], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        // this workgroup's share of round K is finished
        wait_vmem();
        __syncthreads();
        if (lead) {
            release_agent();
            __hip_atomic_fetch_add(&ws.done[K], mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (ld_flag(ws.abort)) return false;
    }
    return true;
}

template <typename U, int ARGMIN, bool VEC>
__global__ __launch_bounds__((Occ<U, ARGMIN>::threads), (Occ<U, ARGMIN>::waves)) void persistent_kernel(
        U *__restrict__ D, int32_t *__restrict__ NX, int64_t n, int64_t ld, int R, int nt,
        int *__restrict__ wsp, int *__restrict__ err, uint64_t timeout_ticks) {
    __shared__ PersistSmem<U, ARGMIN> sm;
    __shared__ int s_item, s_ok;
    persistent_solve<U, ARGMIN, VEC>(D, NX, n, ld, R, nt, persist_ws(wsp, R, nt), err, timeout_ticks, sm, s_item,
                                     s_ok);
}

// ------------------------------------------------------------- batched solve
// Many independent graphs in one launch.  Graph g occupies an n_g x n_g
// row-major block at dist + off[g] (and next + off[g]).  One workgroup solves
// one graph: it normalises the input, then runs the blocked rounds itself --
// phase 1 (phase1_block), the row and column bands and the remaining tiles
// (minplus_tile) -- with workgroup barriers between the phases.  A graph of
// at most 128 vertices is a single phase-1 closure.  Workgroups take graphs
// in the order perm[] (largest first, from batch_order_kernel) so that the
// largest graphs do not form the tail of the launch.
template <typename U, int ARGMIN> union BatchSmem {
    MinplusSmem<U, ARGMIN> mp;
    Phase1Smem<U, kTile, false> p1c;           // closure_block of a diagonal block (32-bit)
    Phase1Smem<U, kTile, ARGMIN != 0 && sizeof(U) == 8> p1;   // phase1_block, successors in LDS (64-bit)
    Phase1Smem<U, 64, false> small;            // graphs of at most 64 vertices
};

// Workgroups that may share one graph in the team schedule: every tile of
// a round at most, capped by the caller's limit; a one-tile graph is a single
// phase-1 closure.
__host__ __device__ __forceinline__ int team_size(int64_t n, int team_cap) {
    const int64_t nt = (n + kTile - 1) / kTile;
    if (nt <= 1) return 1;
    const int64_t t = nt * nt;
    return (int)(t < team_cap ? t : team_cap);
}

// Counting sort of graph indices by decreasing n (one workgroup).  cnt must
// hold n_max + 2 ints of scratch.  With cum != nullptr it also writes the
// team schedule's ticket ranges: sorted graph s owns tickets
// [cum[s], cum[s+1]), and resets the ticket counter.
__global__ __launch_bounds__(1024) void batch_order_kernel(const int32_t *__restrict__ nv, int batch, int n_max,
                                                          int *__restrict__ cnt, int *__restrict__ perm,
                                                          int *__restrict__ err, int team_cap,
                                                          int *__restrict__ cum, int *__restrict__ ticket) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    for (int v = t; v <= n_max + 1; v += blockDim.x) cnt[v] = 0;
    __syncthreads();
    for (int g = t; g < batch; g += blockDim.x) {
        int m = nv[g];
        if (m < 0 || m > n_max) {
            atomicCAS(err, 0, 3);
            m = 0;
        }
        atomicAdd(&cnt[n_max - m], 1);            // bucket 0 = largest n
    }
    __syncthreads();
    if (t == 0) {                                 // exclusive prefix sum (n_max is small)
        int acc = 0;
        for (int v = 0; v <= n_max; ++v) {
            const int c = cnt[v];
            cnt[v] = acc;
            acc += c;
        }
    }
    __syncthreads();
    for (int g = t; g < batch; g += blockDim.x) {
        int m = nv[g];
        if (m < 0 || m > n_max) m = 0;
        perm[atomicAdd(&cnt[n_max - m], 1)] = g;
    }
    if (!cum) return;
    __syncthreads();
    // ticket ranges: each thread scans a contiguous run of sorted positions
    const int per = (batch + 1023) / 1024;
    const int lo = (int)imin64((int64_t)t * per, batch), hi = (int)imin64((int64_t)lo + per, batch);
    int acc = 0;
    for (int q = lo; q < hi; ++q) {
        const int m = nv[perm[q]];
        acc += (m < 0 || m > n_max) ? 0 : team_size(m, team_cap);
    }
    part[t] = acc;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int v = 0; v < 1024; ++v) {
            const int c = part[v];
            part[v] = run;
            run += c;
        }
        cum[batch] = run;
        *ticket = 0;
    }
    __syncthreads();
    acc = part[t];
    for (int q = lo; q < hi; ++q) {
        cum[q] = acc;
        const int m = nv[perm[q]];
        acc += (m < 0 || m > n_max) ? 0 : team_size(m, team_cap);
    }
}

// Input normalisation of every graph of a batch (as init_kernel);
// grid.y = graph.
template <typename U>
__global__ __launch_bounds__(256) void batch_init_kernel(U *__restrict__ D, int32_t *__restrict__ NX,
                                                         const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ nv, int n_max, int validate,
                                                         int *__restrict__ err) {
    const int g = blockIdx.y;
    const int64_t n = nv[g];
    if (n <= 0 || n > n_max) return;
    U *Dg = D + off[g];
    int32_t *NXg = NX ? NX + off[g] : nullptr;
    const int64_t start = (int64_t)blockIdx.x * 256 + threadIdx.x, stride = (int64_t)gridDim.x * 256;
    const bool any_bad = NXg ? normalise_graph<U, true>(Dg, NXg, n, start, stride)
                             : normalise_graph<U, false>(Dg, NXg, n, start, stride);
    if (validate && any_bad) atomicCAS(err, 0, 1);
}

// Team schedule: a resident grid; each workgroup takes a ticket, which names
// a graph (largest first) and makes it one member of that graph's team; the
// team runs the persistent schedule of that graph with the graph's own flag
// workspace, then each member takes another ticket.  Teams only wait on
// items of their own graph that running members have taken, so the launch
// needs no co-resident grid.  A one-tile graph is one phase-1 closure.
template <typename U, int ARGMIN>
__global__ __launch_bounds__((Occ<U, ARGMIN>::threads), (Occ<U, ARGMIN>::waves)) void batched_team_kernel(
        U *__restrict__ D, int32_t *__restrict__ NX, const int64_t *__restrict__ off,
        const int32_t *__restrict__ nv, const int *__restrict__ perm, const int *__restrict__ cum, int batch,
        int n_max, int *__restrict__ ticket, int *__restrict__ wsbase, int64_t ws_stride, int *__restrict__ err,
        uint64_t timeout_ticks) {
    constexpr int NT = MinplusSmem<U, ARGMIN>::NT;
    constexpr bool NEXT = ARGMIN != 0;
    __shared__ PersistSmem<U, ARGMIN> sm;
    __shared__ int s_item, s_ok, s_graph;
    for (;;) {
        __syncthreads();                           // s_graph of the previous graph is consumed
        if (threadIdx.x == 0) {
            const int tk = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int sg = -1;
            if (tk < cum[batch]) {                 // largest s with cum[s] <= tk
                int lo = 0, hi = batch;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (cum[mid] <= tk) lo = mid;
                    else hi = mid;
                }
                sg = lo;
            }
            s_graph = sg;
        }
        __syncthreads();
        const int sg = s_graph;
        if (sg < 0) return;
        const int g = perm[sg];
        const int64_t n = nv[g];
        if (n <= 0 || n > n_max) continue;
        U *Dg = D + off[g];
        int32_t *NXg = NEXT ? NX + off[g] : nullptr;
        const int nt = (int)((n + kTile - 1) / kTile);
        if (nt == 1) {
            phase1_any<U, NEXT, NT>(Dg, NXg, n, n, 0, sm);
            continue;
        }
        const PersistWs ws = persist_ws(wsbase + (int64_t)sg * ws_stride, nt, nt);
        if (!persistent_solve<U, ARGMIN, false>(Dg, NXg, n, n, nt, nt, ws, err, timeout_ticks, sm, s_item, s_ok))
            return;
    }
}

template <typename U, int ARGMIN>
__global__ __launch_bounds__((Occ<U, ARGMIN>::threads), (sizeof(U) == 4 && ARGMIN != 0 ? 4 : 1)) void batched_kernel(
        U *__restrict__ D, int32_t *__restrict__ NX, const int64_t *__restrict__ off,
        const int32_t *__restrict__ nv, const int *__restrict__ perm, int n_max, int validate,
        int *__restrict__ err) {
    constexpr int NT = MinplusSmem<U, ARGMIN>::NT;
    constexpr bool NEXT = ARGMIN != 0;
    constexpr int BS = kTile;
    __shared__ BatchSmem<U, ARGMIN> sm;
    const int g = perm[blockIdx.x];
    const int64_t n = nv[g];
    if (n <= 0 || n > n_max) return;               // reported by the ordering kernel
    U *Dg = D + off[g];
    int32_t *NXg = NEXT ? NX + off[g] : nullptr;
    // normalise the input (as init_kernel), entries of this graph only
    const bool any_bad = normalise_graph<U, NEXT>(Dg, NXg, n, threadIdx.x, NT);
    if (validate && any_bad) atomicCAS(err, 0, 1);
    __syncthreads();
    // at most 64 vertices (32-bit entries): the one-round solve by
    // closure_block -- NT / 16 x 4 threads over a 64 x 64 block, 8 (or 16)
    // entries each -- instead of phase1_block's 128 x 128 patch; same
    // arithmetic, order and successor choice
    if constexpr (sizeof(U) == 4) {
        if (n <= 64) {
            closure_block<U, NEXT, 64, NT>(Dg, NXg, n, n, sm.small);
            return;
        }
    }
    const int R = (int)((n + BS - 1) / BS);
    const int nt = R;
    for (int K = 0; K < R; ++K) {
        const int64_t b0 = (int64_t)K * BS;
        const int64_t b1 = b0 + imin64((int64_t)BS, n - b0);
        // a last diagonal block of at most 64 vertices (32-bit entries) is
        // closed by the 64 x 64 patch (same arithmetic, order and successor
        // choice), not by the 128 x 128 one
        bool short_block = false;
        if constexpr (sizeof(U) == 4) {
            if (b1 - b0 <= 64) {
                closure_block<U, NEXT, 64, NT>(Dg + b0 * n + b0, NEXT ? NXg + b0 * n + b0 : nullptr, b1 - b0, n,
                                               sm.small);
                short_block = true;
            }
        }
        if (!short_block) phase1_any<U, NEXT, NT>(Dg, NXg, n, n, K, sm);
        __syncthreads();
        if (R == 1) break;
        for (int q = 0; q < 2 * nt; ++q) {          // row band, then column band
            const int mode = q < nt ? 1 : 2;
            int64_t row0, col0;
            if (band_tile(mode, q % nt, n, b0, b1, nt, row0, col0)) {
                minplus_tile<U, ARGMIN, false>(Dg, NXg, n, n, K, BS, mode, row0, col0, sm.mp, nullptr, nt);
                __syncthreads();
            }
        }
        for (int q = 0; q < nt * nt; ++q) {
            int64_t row0, col0;
            if (band_tile(0, q, n, b0, b1, nt, row0, col0)) {
                minplus_tile<U, ARGMIN, false>(Dg, NXg, n, n, K, BS, 0, row0, col0, sm.mp, nullptr, nt);
                __syncthreads();
            }
        }
    }
}

// Resident grid of a persistent-style kernel: workgroups per CU (the
// kernel's occupancy, computed once per kernel; a relaxed atomic keeps
// concurrent first calls from different host threads well defined) times CUs.
hipError_t resident_grid(const void *kern, int threads, std::atomic<int> &per_cu, int *grid) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int pc = per_cu.load(std::memory_order_relaxed);
    if (pc <= 0) {
        int nb = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, threads, 0);
        if (e != hipSuccess) return e;
        pc = nb > 0 ? nb : 1;
        per_cu.store(pc, std::memory_order_relaxed);
    }
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    *grid = pc * cus;
    return hipSuccess;
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
    // the block maximum for packed band tiles: int32 with deferred successors
    int *dmax = (std::is_same<U, uint32_t>::value && NEXT && !p.eager_argmin && p.work->bmax)
                        ? p.work->bmax + 4 * (int64_t)p.nt : nullptr;
    switch (p.bs) {
    case 32: hipLaunchKernelGGL((phase1_kernel<U, NEXT, 32>), dim3(1), dim3(256), 0, p.stream, (U *)p.dist, p.next, p.n, p.ld, K, dmax); break;
    case 64: hipLaunchKernelGGL((phase1_kernel<U, NEXT, 64>), dim3(1), dim3(256), 0, p.stream, (U *)p.dist, p.next, p.n, p.ld, K, dmax); break;
    case 128: hipLaunchKernelGGL((phase1_kernel<U, NEXT, 128>), dim3(1), dim3(256), 0, p.stream, (U *)p.dist, p.next, p.n, p.ld, K, dmax); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// phase 2: the band tiles; phase 3: every remaining tile (part 0), only the
// next band's tiles (part 1) or all but those (part 2).
template <typename U, int ARGMIN, bool VEC>
hipError_t minplus_t(const Plan &p, int K, int phase, int part) {
    constexpr int NT = Occ<U, ARGMIN>::threads;
    // the direct-copy phase 3 (block 128, aligned rows): int32 with
    // successors in packed keys, or 32-bit distances only
    constexpr bool PACKED = ARGMIN == 2 && std::is_same<U, uint32_t>::value;
    constexpr bool SEARCH = ARGMIN == 2 && std::is_same<U, float>::value;   // float32 with successors
    constexpr bool DIRECT = VEC && (PACKED || SEARCH || (ARGMIN == 0 && sizeof(U) == 4));
    int *bmax = PACKED ? p.work->bmax : nullptr;
    uint32_t *panel = (DIRECT && p.bs == kTile && !p.general_tile) ? reinterpret_cast<uint32_t *>(p.work->panel)
                                                                   : nullptr;
    const int64_t ppitch = (int64_t)p.nt * kTile;
    if constexpr (DIRECT) {
        if (phase == 3 && panel) {
            // direct-copy tiles, then the general tile on the ones that did not qualify
            const int64_t tiles = (int64_t)p.nt * p.nt;
            const unsigned grid = part == 1 ? (unsigned)(2 * p.nt) : (unsigned)(8 * ((tiles + 7) / 8));
            int *cnt = p.work->fix + 2 * K + (part == 2 ? 1 : 0);
            int *list = p.work->fix + 2 * (int64_t)p.rounds;
            if constexpr (SEARCH) {
                hipLaunchKernelGGL(minplus_direct_search_kernel, dim3(grid), dim3(512), 0, p.stream, (float *)p.dist,
                                   p.next, p.n, p.ld, K, p.nt, part, panel, ppitch, cnt, list);
            } else {
                hipLaunchKernelGGL((minplus_direct_kernel<U, PACKED>), dim3(grid), dim3(256), 0, p.stream,
                                   (U *)p.dist, p.next, p.n, p.ld, K, p.nt, bmax, part, panel, ppitch, cnt, list);
            }
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            const unsigned fgrid = (unsigned)imin64(part == 1 ? 2 * (int64_t)p.nt : tiles, 512);
            hipLaunchKernelGGL((minplus_fixup_kernel<U, ARGMIN, VEC>), dim3(fgrid), dim3(NT), 0, p.stream, (U *)p.dist,
                               p.next, p.n, p.ld, K, p.nt, bmax, cnt, list);
            return hipGetLastError();
        }
    }
    if (phase == 2) {
        hipLaunchKernelGGL((minplus_kernel<U, ARGMIN, 2, VEC>), dim3((unsigned)p.nt, 2), dim3(NT), 0, p.stream,
                           (U *)p.dist, p.next, p.n, p.ld, K, p.bs, p.nt, bmax, 0, panel, ppitch);
    } else if (part == 1) {
        hipLaunchKernelGGL((minplus_kernel<U, ARGMIN, 3, VEC>), dim3((unsigned)(2 * p.nt)), dim3(NT), 0, p.stream,
                           (U *)p.dist, p.next, p.n, p.ld, K, p.bs, p.nt, bmax, 1, panel, ppitch);
    } else {
        const int64_t tiles = (int64_t)p.nt * p.nt;
        hipLaunchKernelGGL((minplus_kernel<U, ARGMIN, 3, VEC>), dim3((unsigned)(8 * ((tiles + 7) / 8))), dim3(NT),
                           0, p.stream, (U *)p.dist, p.next, p.n, p.ld, K, p.bs, p.nt, bmax, part, panel, ppitch);
    }
    return hipGetLastError();
}

template <typename U, int ARGMIN>
hipError_t minplus_v(const Plan &p, int K, int phase, int part) {
    return p.vec ? minplus_t<U, ARGMIN, true>(p, K, phase, part) : minplus_t<U, ARGMIN, false>(p, K, phase, part);
}

template <typename U, int ARGMIN, bool VEC>
hipError_t persistent_t(const Plan &p) {
    constexpr int NT = Occ<U, ARGMIN>::threads;
    auto kern = persistent_kernel<U, ARGMIN, VEC>;
    static std::atomic<int> per_cu{0};
    int resident = 0;
    hipError_t e = resident_grid(reinterpret_cast<const void *>(kern), NT, per_cu, &resident);
    if (e != hipSuccess) return e;
    const int64_t count = persist_ws_ints(p.rounds, p.nt);
    hipLaunchKernelGGL(zero_ints_kernel, dim3(8), dim3(256), 0, p.stream, p.work->persist, count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t items = 1 + 2 * (int64_t)p.nt + (int64_t)p.nt * p.nt;
    const int grid = (int)imin64(resident, items);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, p.stream, (U *)p.dist, p.next, p.n, p.ld, p.rounds, p.nt,
                       p.work->persist, p.work->err, p.timeout_ticks);
    return hipGetLastError();
}

template <typename U>
hipError_t persistent_dispatch(const Plan &p) {
    if (!p.next) return p.vec ? persistent_t<U, 0, true>(p) : persistent_t<U, 0, false>(p);
    if (p.eager_argmin) return p.vec ? persistent_t<U, 1, true>(p) : persistent_t<U, 1, false>(p);
    return p.vec ? persistent_t<U, 2, true>(p) : persistent_t<U, 2, false>(p);
}

// Batched scratch (ints): cnt[n_max + 2] | perm[batch] | cum[batch + 1] |
// ticket, padded to 64 | team flag workspaces, ws_stride per sorted graph.
struct BatchLayout {
    int64_t cnt, perm, cum, ticket, ws, total, ws_stride;
};
BatchLayout batch_layout(int batch, int n_max, bool team) {
    BatchLayout L;
    L.cnt = 0;
    L.perm = L.cnt + n_max + 2;
    L.cum = L.perm + batch;
    L.ticket = L.cum + batch + 1;
    L.ws = ((L.ticket + 1 + 63) / 64) * 64;
    const int nt = (n_max + kTile - 1) / kTile;
    L.ws_stride = team && nt > 1 ? ((persist_ws_ints(nt, nt) + 15) / 16) * 16 : 0;
    L.total = L.ws + (int64_t)batch * L.ws_stride;
    return L;
}

template <typename U, int ARGMIN>
hipError_t batched_t(const BatchPlan &b) {
    constexpr int NT = Occ<U, ARGMIN>::threads;
    const bool team = b.team_cap != 1;
    const BatchLayout L = batch_layout(b.batch, b.n_max, team);
    int *sc = b.scratch;
    hipLaunchKernelGGL(batch_order_kernel, dim3(1), dim3(1024), 0, b.stream, b.nv, b.batch, b.n_max, sc + L.cnt,
                       sc + L.perm, b.err, b.team_cap, team ? sc + L.cum : nullptr, sc + L.ticket);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!team) {
        hipLaunchKernelGGL((batched_kernel<U, ARGMIN>), dim3((unsigned)b.batch), dim3(NT), 0, b.stream,
                           (U *)b.dist, b.next, b.off, b.nv, sc + L.perm, b.n_max, b.validate ? 1 : 0, b.err);
        return hipGetLastError();
    }
    if (L.ws_stride > 0) {
        const int64_t cnt = (int64_t)b.batch * L.ws_stride;
        const unsigned zg = (unsigned)imin64((cnt + 255) / 256, 1024);
        hipLaunchKernelGGL(zero_ints_kernel, dim3(zg), dim3(256), 0, b.stream, sc + L.ws, cnt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int64_t nn = (int64_t)b.n_max * b.n_max;
    const unsigned ix = (unsigned)imin64((nn + 255) / 256, 64);
    hipLaunchKernelGGL(batch_init_kernel<U>, dim3(ix, (unsigned)b.batch), dim3(256), 0, b.stream, (U *)b.dist,
                       b.next, b.off, b.nv, b.n_max, b.validate ? 1 : 0, b.err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    auto kern = batched_team_kernel<U, ARGMIN>;
    static std::atomic<int> per_cu{0};
    int resident = 0;
    if ((e = resident_grid(reinterpret_cast<const void *>(kern), NT, per_cu, &resident)) != hipSuccess) return e;
    const int64_t tickets = (int64_t)b.batch * team_size(b.n_max, b.team_cap);
    const int grid = (int)imin64(resident, tickets);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, b.stream, (U *)b.dist, b.next, b.off, b.nv, sc + L.perm,
                       sc + L.cum, b.batch, b.n_max, sc + L.ticket, sc + L.ws, L.ws_stride, b.err, b.timeout_ticks);
    return hipGetLastError();
}

// Successor bookkeeping per schedule (measured on MI355X, float32, same
// bits either way): with one workgroup per graph (n <= 256 in practice) most
// entries improve in most k chunks, so the eager variant's fixed four
// operations beat the deferred search (4096 graphs of n ~ U{16..256}: 4.5 vs
// 6.8 ms); team schedules on larger graphs keep the deferred one.
template <typename U>
hipError_t batched_dispatch(const BatchPlan &b) {
    if (!b.next) return batched_t<U, 0>(b);
    return (b.eager_argmin || b.team_cap == 1) ? batched_t<U, 1>(b) : batched_t<U, 2>(b);
}

}  // namespace

int64_t batched_workspace_ints(int batch, int n_max, int team_cap) {
    return batch_layout(batch, n_max, team_cap != 1).total;
}

hipError_t launch_batched(const BatchPlan &b) {
    switch (b.dtype) {
    case DType::I32: return batched_dispatch<uint32_t>(b);
    case DType::F32: return batched_dispatch<float>(b);
    default: return batched_dispatch<double>(b);
    }
}

int64_t persistent_workspace_ints(int rounds, int nt) { return persist_ws_ints(rounds, nt); }

hipError_t launch_persistent(const Plan &p) {
    switch (p.dtype) {
    case DType::I32: return persistent_dispatch<uint32_t>(p);
    case DType::F32: return persistent_dispatch<float>(p);
    default: return persistent_dispatch<double>(p);
    }
}

hipError_t launch_fix_reset(const Plan &p) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(256), 0, p.stream, p.work->fix, 2 * (int64_t)p.rounds);
    return hipGetLastError();
}

hipError_t launch_init(const Plan &p) {
    switch (p.dtype) {
    case DType::I32: return init_t<uint32_t>(p);
    case DType::F32: return init_t<float>(p);
    default: return init_t<double>(p);
    }
}

hipError_t launch_phase1(const Plan &p, int K) {
    if (p.dtype == DType::I32) return p.next ? phase1_t<uint32_t, true>(p, K) : phase1_t<uint32_t, false>(p, K);
    if (p.dtype == DType::F32) return p.next ? phase1_t<float, true>(p, K) : phase1_t<float, false>(p, K);
    return p.next ? phase1_t<double, true>(p, K) : phase1_t<double, false>(p, K);
}

template <typename U>
hipError_t minplus_dispatch(const Plan &p, int K, int phase, int part) {
    if (!p.next) return minplus_v<U, 0>(p, K, phase, part);
    return p.eager_argmin ? minplus_v<U, 1>(p, K, phase, part) : minplus_v<U, 2>(p, K, phase, part);
}

hipError_t launch_phase2(const Plan &p, int K) {
    switch (p.dtype) {
    case DType::I32: return minplus_dispatch<uint32_t>(p, K, 2, 0);
    case DType::F32: return minplus_dispatch<float>(p, K, 2, 0);
    default: return minplus_dispatch<double>(p, K, 2, 0);
    }
}

hipError_t launch_resolve(const Plan &p) {
    if (!p.next || p.n == 0) return hipSuccess;
    const dim3 grid((unsigned)p.n), block(kResolveThreads);
    if (!p.resolve_in_memory && p.n <= 4096)
        hipLaunchKernelGGL(resolve_next_kernel<4096>, grid, block, 0, p.stream, p.next, p.n, p.ld);
    else if (!p.resolve_in_memory && p.n <= kResolveLdsMaxN)
        hipLaunchKernelGGL(resolve_next_kernel<kResolveLdsMaxN>, grid, block, 0, p.stream, p.next, p.n, p.ld);
    else
        hipLaunchKernelGGL(resolve_next_kernel<0>, grid, block, 0, p.stream, p.next, p.n, p.ld);
    return hipGetLastError();
}

hipError_t launch_phase3(const Plan &p, int K, int part) {
    switch (p.dtype) {
    case DType::I32: return minplus_dispatch<uint32_t>(p, K, 3, part);
    case DType::F32: return minplus_dispatch<float>(p, K, 3, part);
    default: return minplus_dispatch<double>(p, K, 3, part);
    }
}

}  // namespace fw
