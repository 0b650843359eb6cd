// Gradient of the distances with respect to the edge weights (gfx950).
//
// A distance the solver returns is the sum of the edge weights along the path
// its successor matrix selects, i -> NX[i][j] -> ... -> j (the paths the
// blocked rounds of Section 2.3 build, one relaxation at a time).  For a loss
// with upstream gradient G = dL/dD, dL/dW[u][v] is the sum of G[i][j] over
// the pairs (i, j), i != j, whose selected path uses the edge (u, v); the
// diagonal and unreachable pairs are constants.
//
// For one destination j the selected paths form an in-tree: every vertex u
// that reaches j points at parent(u) = NX[u][j].  The edge (u, parent(u)) is
// on path(i, j) exactly when i lies in u's subtree, so it receives the
// subtree sum S_j(u) = G[u][j] + the sum of S_j(c) over u's children c.  One
// workgroup handles one destination (one column of G and NX):
//   1. load the column: parent and S_j(u) = G[u][j] per vertex;
//   2. count each vertex's children (LDS atomics);
//   3. queue the leaves, then process the queue level by level: a vertex
//      adds S_j(u) to dW[u][parent(u)] (a global float atomic, since other
//      destinations use the same edge) and to S_j(parent); the parent joins
//      the queue when its last child is done.
// Work and traffic are O(n) per destination; a step of the level loop is one
// tree level.  A successor entry outside [0, n) counts as "no path"; a vertex
// on a successor cycle never becomes ready and is skipped, so malformed
// input cannot fault or hang.  The float atomics make the summation order,
// and so the last bits, vary from run to run.
#include "fw_internal.h"

namespace fw {
namespace {

constexpr int kBwdThreads = 256;

__device__ __forceinline__ void wait_vmem_bwd() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Per-destination working arrays live in LDS (SH = true) or in a global
// scratch slice of the workgroup; the global form bypasses the per-CU cache
// (agent-scope atomics) so that the waves of the workgroup see each other's
// updates, and drains its stores before every barrier.
template <bool SH, typename T> __device__ __forceinline__ T sld(const T *p) {
    if constexpr (SH) return *p;
    else return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool SH, typename T> __device__ __forceinline__ void sst(T *p, T v) {
    if constexpr (SH) *p = v;
    else __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool SH> __device__ __forceinline__ void bsync() {
    if (!SH) wait_vmem_bwd();
    __syncthreads();
}

template <bool SH>
__device__ void backward_column(const float *__restrict__ G, const int32_t *__restrict__ NX,
                                float *__restrict__ dW, int64_t ld, int n, int j, int *par, int *cnt,
                                float *S, int *q, int &tail) {
    const int t = threadIdx.x;
    bsync<SH>();                               // the previous column is finished
    if (t == 0) tail = 0;
    for (int u = t; u < n; u += kBwdThreads) {
        const int64_t o = (int64_t)u * ld + j;
        const int v = NX[o];
        const bool on = u != j && v >= 0 && v < n;
        sst<SH>(&par[u], on ? v : -1);
        sst<SH>(&S[u], on ? G[o] : 0.0f);
        sst<SH>(&cnt[u], 0);
    }
    bsync<SH>();
    for (int u = t; u < n; u += kBwdThreads) {
        const int v = sld<SH>(&par[u]);
        if (v >= 0 && v != j) atomicAdd(&cnt[v], 1);
    }
    bsync<SH>();
    for (int u = t; u < n; u += kBwdThreads)
        if (sld<SH>(&par[u]) >= 0 && sld<SH>(&cnt[u]) == 0) sst<SH>(&q[atomicAdd(&tail, 1)], u);
    int head = 0;
    for (;;) {
        bsync<SH>();
        const int end = tail;                  // the same value in every thread
        if (head >= end) break;
        __syncthreads();                       // read before the level appends more
        for (int x = head + t; x < end; x += kBwdThreads) {
            const int u = sld<SH>(&q[x]);
            const int v = sld<SH>(&par[u]);
            const float s = sld<SH>(&S[u]);
            unsafeAtomicAdd(&dW[(int64_t)u * ld + v], s);
            if (v != j) {
                if (SH) atomicAdd(&S[v], s);
                else unsafeAtomicAdd(&S[v], s);
                if (atomicSub(&cnt[v], 1) == 1) sst<SH>(&q[atomicAdd(&tail, 1)], v);
            }
        }
        head = end;
    }
}

// grid.x = 8 * ceil(columns / 8) workgroups (or fewer for the global form,
// which then loops), grid.y = graphs.  Workgroups are dealt to the eight XCDs
// round-robin; the mapping gives each XCD a contiguous run of destinations,
// so neighbouring columns share cache lines in one L2.
template <bool SH>
__global__ __launch_bounds__(kBwdThreads) void backward_kernel(
        const float *__restrict__ G, const int32_t *__restrict__ NX, float *__restrict__ dW, int64_t n1,
        int64_t ld1, const int64_t *__restrict__ off, const int32_t *__restrict__ nv, int n_cap,
        int *__restrict__ scratch, int *__restrict__ err) {
    extern __shared__ int bwd_lds[];
    __shared__ int s_tail;
    int64_t base = 0, ld = ld1;
    int n = (int)n1;
    if (off) {
        n = nv[blockIdx.y];
        base = off[blockIdx.y];
        ld = n;
        if (n < 0 || n > n_cap) {
            if (threadIdx.x == 0 && blockIdx.x == 0) atomicCAS(err, 0, 3);
            return;
        }
    }
    if (n <= 1) return;
    const int per = (int)(gridDim.x / 8);
    const int jb = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    int *par, *cnt, *q;
    float *S;
    if (SH) {
        par = bwd_lds;
        cnt = par + n_cap;
        S = reinterpret_cast<float *>(cnt + n_cap);
        q = reinterpret_cast<int *>(S + n_cap);
    } else {
        par = scratch + (int64_t)blockIdx.x * 4 * n_cap;
        cnt = par + n_cap;
        S = reinterpret_cast<float *>(cnt + n_cap);
        q = reinterpret_cast<int *>(S + n_cap);
    }
    for (int64_t j = jb; j < n; j += gridDim.x)
        backward_column<SH>(G + base, NX + base, dW + base, ld, n, (int)j, par, cnt, S, q, s_tail);
}

// dW = 0 over each graph's n x n block (rows of length n at stride ld).
__global__ __launch_bounds__(256) void zero_grad_kernel(float *__restrict__ dW, int64_t n1, int64_t ld1,
                                                         const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ nv, int n_cap) {
    int64_t base = 0, ld = ld1, n = n1;
    if (off) {
        n = nv[blockIdx.y];
        base = off[blockIdx.y];
        ld = n;
        if (n < 0 || n > n_cap) return;
    }
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x)
        for (int64_t c = threadIdx.x; c < n; c += 256) dW[base + i * ld + c] = 0.0f;
}

}  // namespace

int64_t backward_scratch_ints(const BackwardPlan &b) {
    if (b.n_cap <= kBackwardLdsMaxN) return 0;
    return (int64_t)backward_global_workgroups(b) * 4 * b.n_cap;
}

int backward_global_workgroups(const BackwardPlan &b) {
    const int64_t cols = 8 * (((int64_t)b.n_cap + 7) / 8);
    return (int)(cols < 1024 ? cols : 1024);
}

hipError_t launch_backward(const BackwardPlan &b) {
    const unsigned graphs = b.off ? (unsigned)b.batch : 1u;
    const unsigned zx = (unsigned)(b.n_cap < 4096 ? b.n_cap : 4096);
    hipLaunchKernelGGL(zero_grad_kernel, dim3(zx, graphs), dim3(256), 0, b.stream, b.dW, b.n, b.ld, b.off, b.nv,
                       b.n_cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b.n_cap <= kBackwardLdsMaxN) {
        const unsigned gx = (unsigned)(8 * ((b.n_cap + 7) / 8));
        const size_t lds = (size_t)16 * b.n_cap;
        hipLaunchKernelGGL(backward_kernel<true>, dim3(gx, graphs), dim3(kBwdThreads), lds, b.stream, b.G, b.NX,
                           b.dW, b.n, b.ld, b.off, b.nv, b.n_cap, nullptr, b.err);
    } else {
        const unsigned gx = (unsigned)backward_global_workgroups(b);
        hipLaunchKernelGGL(backward_kernel<false>, dim3(gx, graphs), dim3(kBwdThreads), 0, b.stream, b.G, b.NX,
                           b.dW, b.n, b.ld, b.off, b.nv, b.n_cap, b.scratch, b.err);
    }
    return hipGetLastError();
}

}  // namespace fw
