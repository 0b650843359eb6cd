// Measured ceilings of the phase-3 min-plus tile on the GPU it runs on: a
// standalone program (not part of libfwgpu.so) that times register-only and
// LDS-only loops with the tile's instruction mix and prints one line each.
//
//   valu <op>   : one 32-bit VALU instruction repeated on 32 independent
//                 accumulators (v_add_u32, v_min_u32, v_min3_u32)
//   mix <order> : the packed-key relaxation of the tile, two v_add_u32 and one
//                 v_min3_u32 per pair of k's and entry, operands in registers
//                 (8 x 4 entries per thread); "compiler" = the compiler's own
//                 order, "pinned" = add, add, min3 entry by entry
//   eager f32   : the eager float32 relaxation with a successor (the batched
//                 solve's closures and tiles), one k per step, operands in
//                 registers (8 x 4 entries per thread): v_add_f32,
//                 v_cmp_lt_f32, a minimum on the bit patterns and the
//                 successor select -- four VALU instructions per relaxation
//   min f32     : the float32 distances-only relaxation of the same tile, two
//                 k's per step (two v_add_f32 and one three-way minimum)
//   lds <form>  : ds_read_b128 of the tile's operand patterns, as in the
//                 tile's k loop: "A" (32 lanes share an address), "B" (two
//                 lanes share an address) and "distinct"
//
// Occupancy is pinned with dynamic LDS (k workgroups of 256 threads per CU).
// The work per launch is fixed, so rates are whole-launch averages over all
// CUs, including launch and tail time.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kThreads = 256;

template <int OP>
__global__ __launch_bounds__(kThreads) void valu_kernel(uint32_t *out, int iters, uint32_t seed) {
    extern __shared__ uint32_t pad[];
    const uint32_t t = threadIdx.x + blockIdx.x * kThreads + seed;
    uint32_t acc[32];
    for (int i = 0; i < 32; ++i) acc[i] = t * 2654435761u + i;
    uint32_t s = t * 7u, s2 = t * 13u;
    for (int it = 0; it < iters; ++it) {
        asm volatile("" : "+v"(s), "+v"(s2));
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                if constexpr (OP == 0) acc[i] += s;
                else if constexpr (OP == 1) acc[i] = min(acc[i], s);
                else acc[i] = min(min(acc[i], s), s2);
                asm volatile("" : "+v"(acc[i]));   // keeps the 96 instructions as written
            }
    }
    uint32_t x = 0;
    for (int i = 0; i < 32; ++i) x ^= acc[i];
    if (threadIdx.x == 0) pad[0] = x;
    out[blockIdx.x * kThreads + threadIdx.x] = x;
}

template <bool PINNED>
__global__ __launch_bounds__(kThreads) void mix_kernel(uint32_t *out, int iters, uint32_t seed) {
    extern __shared__ uint32_t pad[];
    const uint32_t t = threadIdx.x + blockIdx.x * kThreads + seed;
    uint32_t acc[8][4], a[8], b[4], a2[8], b2[4];
    for (int r = 0; r < 8; ++r) { a[r] = t * 3u + r; a2[r] = t * 5u + r; }
    for (int c = 0; c < 4; ++c) { b[c] = t * 7u + c; b2[c] = t * 11u + c; }
    for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 4; ++c) acc[r][c] = 0xFFFFFFFFu - r - c;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 8; ++r) asm volatile("" : "+v"(a[r]), "+v"(a2[r]));
#pragma unroll
        for (int c = 0; c < 4; ++c) asm volatile("" : "+v"(b[c]), "+v"(b2[c]));
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if constexpr (PINNED) {
                    uint32_t x = a[r] + b[c], y = a2[r] + b2[c];
                    asm volatile("" : "+v"(x), "+v"(y));
                    acc[r][c] = min(acc[r][c], min(x, y));
                    asm volatile("" : "+v"(acc[r][c]));
                } else {
                    acc[r][c] = min(acc[r][c], min(a[r] + b[c], a2[r] + b2[c]));
                }
            }
    }
    uint32_t x = 0;
    for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 4; ++c) x ^= acc[r][c];
    if (threadIdx.x == 0) pad[0] = x;
    out[blockIdx.x * kThreads + threadIdx.x] = x;
}

// The float32 relaxations of the batched solve, operands in registers.
// EAGER: d <- min(d, a + b) and the successor select, one k per step; else
// distances only, two k's per step.  Values are non-negative, so the minimum
// is taken on bit patterns, as the solve does.
template <bool EAGER>
__global__ __launch_bounds__(kThreads) void f32_kernel(uint32_t *out, int iters, uint32_t seed) {
    extern __shared__ uint32_t pad[];
    const uint32_t t = threadIdx.x + blockIdx.x * kThreads + seed;
    float acc[8][4], a[8], b[4], a2[8], b2[4];
    int32_t idx[8][4], na[8];
    for (int r = 0; r < 8; ++r) {
        a[r] = (float)((t + r) % 97) * 0.25f;
        a2[r] = (float)((t + 3 * r) % 89) * 0.25f;
        na[r] = (int32_t)(t + r);
    }
    for (int c = 0; c < 4; ++c) {
        b[c] = (float)((t >> 3) % 61 + c) * 0.125f;
        b2[c] = (float)((t >> 5) % 53 + c) * 0.125f;
    }
    for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 4; ++c) {
            acc[r][c] = 1e30f;
            idx[r][c] = -1;
        }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 8; ++r) asm volatile("" : "+v"(a[r]), "+v"(a2[r]), "+v"(na[r]));
#pragma unroll
        for (int c = 0; c < 4; ++c) asm volatile("" : "+v"(b[c]), "+v"(b2[c]));
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if constexpr (EAGER) {
                    const float x = a[r] + b[c];
                    const bool lt = x < acc[r][c];
                    acc[r][c] = __uint_as_float(min(__float_as_uint(acc[r][c]), __float_as_uint(x)));
                    idx[r][c] = lt ? na[r] : idx[r][c];
                } else {
                    const uint32_t x = __float_as_uint(a[r] + b[c]), y = __float_as_uint(a2[r] + b2[c]);
                    acc[r][c] = __uint_as_float(min(min(__float_as_uint(acc[r][c]), x), y));
                }
            }
    }
    uint32_t x = 0;
    for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 4; ++c) x ^= __float_as_uint(acc[r][c]) ^ (uint32_t)idx[r][c];
    if (threadIdx.x == 0) pad[0] = x;
    out[blockIdx.x * kThreads + threadIdx.x] = x;
}

// 34 rows of 128 words of LDS (the launch gives at least that); each step
// reads 4 x 16 bytes per lane from rows kk .. kk + 3 (kk < 32).
constexpr int kLdsWords = 34 * 128;
template <int FORM>
__global__ __launch_bounds__(kThreads) void lds_kernel(uint32_t *out, int iters, uint32_t seed) {
    extern __shared__ __attribute__((aligned(16))) uint32_t buf[];
    for (int q = threadIdx.x; q < kLdsWords; q += kThreads) buf[q] = q * 2654435761u + seed;
    __syncthreads();
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int lane = t & 63, w = t >> 6;
    // word offset of this lane's 16 bytes in row 0
    int off;
    if constexpr (FORM == 0) off = (w * 2 + (lane >> 5)) * 4;      // A: 32 lanes per address
    else if constexpr (FORM == 1) off = (lane & 31) * 4;           // B: 2 lanes per address
    else off = lane * 4;                                           // distinct: 1 KiB over two rows
    const uint32_t *p = buf + off;
    uint4 x = make_uint4(0, 0, 0, 0);
    for (int it = 0; it < iters; ++it) {
#pragma unroll 1
        for (int kk = 0; kk < 32; kk += 4) {
            const uint4 v0 = *reinterpret_cast<const uint4 *>(p + (kk + 0) * 128);
            const uint4 v1 = *reinterpret_cast<const uint4 *>(p + (kk + 1) * 128);
            const uint4 v2 = *reinterpret_cast<const uint4 *>(p + (kk + 2) * 128);
            const uint4 v3 = *reinterpret_cast<const uint4 *>(p + (kk + 3) * 128);
            x.x ^= v0.x ^ v1.x ^ v2.x ^ v3.x;       // every word used: four full 16-byte reads
            x.y ^= v0.y ^ v1.y ^ v2.y ^ v3.y;
            x.z ^= v0.z ^ v1.z ^ v2.z ^ v3.z;
            x.w ^= v0.w ^ v1.w ^ v2.w ^ v3.w;
        }
    }
    out[blockIdx.x * kThreads + threadIdx.x] = x.x ^ x.y ^ x.z ^ x.w;
}

struct Timer {
    hipEvent_t a, b;
    Timer() { (void)hipEventCreate(&a); (void)hipEventCreate(&b); }
    ~Timer() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
};

template <typename K>
bool launch_timed(K kern, int grid, size_t lds, uint32_t *out, int iters, float *ms) {
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            150 * 1024) != hipSuccess)
        return false;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, 0, out, 2, 1u);   // warm-up
    if (hipDeviceSynchronize() != hipSuccess) return false;
    Timer tm;
    if (hipEventRecord(tm.a) != hipSuccess) return false;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, 0, out, iters, 2u);
    if (hipEventRecord(tm.b) != hipSuccess || hipEventSynchronize(tm.b) != hipSuccess) return false;
    return hipEventElapsedTime(ms, tm.a, tm.b) == hipSuccess;
}

}  // namespace

int main() {
    int dev = 0, cus = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev) != hipSuccess) {
        std::printf("no HIP device\n");
        return 2;
    }
    const double ghz = khz / 1e6;
    const int k = 8;                                  // workgroups (of 4 waves) per CU: 8 waves per SIMD
    const int grid = cus * k;
    const size_t lds = (size_t)(150 * 1024) / k;      // at most k workgroups fit per CU
    static_assert((150 * 1024) / 8 >= kLdsWords * 4, "LDS of the lds kernels");
    uint32_t *out = nullptr;
    if (hipMalloc(&out, (size_t)grid * kThreads * sizeof(uint32_t)) != hipSuccess) return 2;
    std::printf("%d CUs, peak engine clock %.2f GHz, %d workgroups of %d threads per CU\n", cus, ghz, k, kThreads);
    const double simds = cus * 4.0;
    float ms = 0;
    int rc = 0;
    const char *valu_names[3] = {"v_add_u32", "v_min_u32", "v_min3_u32"};
    void (*valu[3])(uint32_t *, int, uint32_t) = {valu_kernel<0>, valu_kernel<1>, valu_kernel<2>};
    for (int i = 0; i < 3; ++i) {
        const int iters = 20000;
        if (!launch_timed(valu[i], grid, lds, out, iters, &ms)) { rc = 1; break; }
        const double inst = (double)grid * 4 * iters * 96.0;                 // wave instructions
        const double per_clk = inst / simds / (ms * 1e-3 * ghz * 1e9);
        std::printf("valu %-10s %8.3f ms  %.2f cycles per wave64 instruction per SIMD (%.1f lanes/clock)\n",
                    valu_names[i], ms, 1.0 / per_clk, 64.0 * per_clk);
    }
    for (int pinned = 0; pinned < 2 && !rc; ++pinned) {
        const int iters = 20000;
        if (!launch_timed(pinned ? mix_kernel<true> : mix_kernel<false>, grid, lds, out, iters, &ms)) { rc = 1; break; }
        const double relax = (double)grid * kThreads * iters * 64.0;
        std::printf("mix  %-10s %8.3f ms  %.4e relaxations/s (2 x v_add_u32 + v_min3_u32 per pair of k's)\n",
                    pinned ? "pinned" : "compiler", ms, relax / (ms * 1e-3));
    }
    // float32 relaxations; the fraction is of the 2-operation-per-relaxation
    // rate (128 lanes per clock per CU)
    const double peak_relax = cus * ghz * 1e9 * 128.0 / 2.0;
    for (int eager = 1; eager >= 0 && !rc; --eager) {
        const int iters = 20000;
        if (!launch_timed(eager ? f32_kernel<true> : f32_kernel<false>, grid, lds, out, iters, &ms)) { rc = 1; break; }
        const double relax = (double)grid * kThreads * iters * (eager ? 32.0 : 64.0);
        const double rate = relax / (ms * 1e-3);
        std::printf("%-15s %8.3f ms  %.4e relaxations/s (%.3f of 2 operations per relaxation at 128 lanes/clock)\n",
                    eager ? "eager f32" : "min f32", ms, rate, rate / peak_relax);
    }
    const char *lds_names[3] = {"A", "B", "distinct"};
    void (*ldsk[3])(uint32_t *, int, uint32_t) = {lds_kernel<0>, lds_kernel<1>, lds_kernel<2>};
    for (int i = 0; i < 3 && !rc; ++i) {
        const int iters = 4000;
        if (!launch_timed(ldsk[i], grid, lds, out, iters, &ms)) { rc = 1; break; }
        const double inst = (double)grid * 4 * iters * 32.0;                  // wave ds_read_b128
        const double per_cu_clk = inst / cus / (ms * 1e-3 * ghz * 1e9);
        std::printf("lds  %-10s %8.3f ms  %.2f cycles per wave ds_read_b128 per CU (%.0f bytes/clock per CU)\n",
                    lds_names[i], ms, 1.0 / per_cu_clk, 1024.0 * per_cu_clk);
    }
    if (rc) std::printf("launch failed\n");
    (void)hipFree(out);
    return rc;
}
