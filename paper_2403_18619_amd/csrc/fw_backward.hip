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
// wave (graphs of up to 1024 vertices) or one workgroup handles one
// destination (one column of G and NX):
//   1. load the column: parent and S_j(u) = G[u][j] per vertex;
//   2. count each vertex's children (LDS atomics);
//   3. queue the leaves, then process the queue level by level: a vertex
//      adds S_j(u) to S_j(parent); the parent joins the queue when its last
//      child is done;
//   4. write S_j(u) into dW[u][j], used as scratch (0 for the root, for
//      unreachable vertices and for vertices never processed).
// A second pass then works per source row u: the edge (u, v) collects
// S_j(u) over the destinations j with next[u][j] = v, a scatter-add of the
// row's sums into an LDS histogram indexed by successor, which then
// overwrites the row.  Both passes read rows or columns once and the second
// writes each gradient row once, with no global atomics (a column's float
// atomics into dW touched one cache line per lane and dominated the time).
// Graphs above 32768 vertices, whose histogram row does not fit in LDS, add
// into dW with global atomics instead.
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

template <bool SH, bool ROWS>
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
            if (ROWS) sst<SH>(&cnt[u], -1);                  // processed
            else unsafeAtomicAdd(&dW[(int64_t)u * ld + v], s);
            if (v != j) {
                if (SH) atomicAdd(&S[v], s);
                else unsafeAtomicAdd(&S[v], s);
                if (atomicSub(&cnt[v], 1) == 1) sst<SH>(&q[atomicAdd(&tail, 1)], v);
            }
        }
        head = end;
    }
    if (ROWS) {
        for (int u = t; u < n; u += kBwdThreads)
            dW[(int64_t)u * ld + j] = sld<SH>(&cnt[u]) == -1 ? sld<SH>(&S[u]) : 0.0f;
    }
}

// grid.x = 8 * ceil(columns / 8) workgroups (or fewer for the global form,
// which then loops), grid.y = graphs.  Workgroups are dealt to the eight XCDs
// round-robin; the mapping gives each XCD a contiguous run of destinations,
// so neighbouring columns share cache lines in one L2.
template <bool SH, bool ROWS>
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
        backward_column<SH, ROWS>(G + base, NX + base, dW + base, ld, n, (int)j, par, cnt, S, q, s_tail);
}

// Graphs of at most kBwdWaveMaxN vertices: one wave per destination, four
// neighbouring destinations j0 .. j0+3 per workgroup, wave-level ordering
// instead of workgroup barriers while the trees are processed (a
// destination's tree has few levels and few vertices per lane, so barriers
// and idle lanes dominated the workgroup form).  Per vertex and destination
// the wave keeps 12 bytes of LDS -- child count and subtree sum (32-bit,
// updated with LDS atomics), parent and queue slot (16-bit, n <= 1024) -- so
// that three workgroups share a CU.  The workgroup reads and writes its four
// columns together: four lanes take the four entries of one row, so that one
// access of a wave touches 16 rows (cache lines) rather than 64, and each
// entry goes to, or comes from, its destination wave's arrays (eight rows per
// lane in flight before the first LDS store).
constexpr int kBwdWaveMaxN = 1024;
constexpr int kBwdWaveBytes = 12;           // LDS bytes per vertex and destination
constexpr int kBwdWavePad = 16;             // words between two waves' arrays (LDS banks)

__device__ __forceinline__ void wave_sync_bwd() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ __forceinline__ int64_t bwd_wave_stride_words(int n_cap) {
    return (int64_t)(kBwdWaveBytes / 4) * n_cap + kBwdWavePad;
}

__global__ __launch_bounds__(256) void backward_wave_kernel(
        const float *__restrict__ G, const int32_t *__restrict__ NX, float *__restrict__ dW, int64_t n1,
        int64_t ld1, const int64_t *__restrict__ off, const int32_t *__restrict__ nv, int n_cap,
        int *__restrict__ err) {
    extern __shared__ int bwd_lds[];
    __shared__ int s_tail[4];
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
    const int t = (int)threadIdx.x, w = t >> 6, lane = t & 63;
    // workgroups are dealt to the XCDs round-robin: each XCD gets a run of
    // neighbouring destinations, whose columns share cache lines
    const int per = (int)(gridDim.x / 8);
    const int grp = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    const int j0 = grp * 4;
    if (j0 >= n) return;                    // the whole workgroup; no barrier follows
    const int64_t stride = bwd_wave_stride_words(n_cap);
    const float *Gg = G + base;
    const int32_t *Ng = NX + base;
    float *dWg = dW + base;

    // ---- columns j0 .. j0+3 into the four waves' arrays: thread t takes
    // column c = t % 4 of rows r, r + 64, ... (r = t / 4)
    const int c = t & 3, r = t >> 2, jc = j0 + c;
    int *cnt_c = bwd_lds + c * stride;
    float *S_c = reinterpret_cast<float *>(cnt_c + n_cap);
    int16_t *par_c = reinterpret_cast<int16_t *>(S_c + n_cap);
    if (t < 4) s_tail[t] = 0;
    for (int u0 = 0; u0 < n; u0 += 8 * 64) {
        int v[8];
        float g[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int u = u0 + 64 * m + r;
            const int64_t o = (u < n && jc < n) ? (int64_t)u * ld + jc : 0;
            v[m] = Ng[o];
            g[m] = Gg[o];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int u = u0 + 64 * m + r;
            if (u < n && jc < n) {
                const bool on = u != jc && v[m] >= 0 && v[m] < n;
                par_c[u] = (int16_t)(on ? v[m] : -1);
                S_c[u] = on ? g[m] : 0.0f;
                cnt_c[u] = 0;
            }
        }
    }
    __syncthreads();

    // ---- this wave's tree (destination j)
    const int j = j0 + w;
    if (j < n) {
        int *cnt = bwd_lds + w * stride;
        float *S = reinterpret_cast<float *>(cnt + n_cap);
        int16_t *par = reinterpret_cast<int16_t *>(S + n_cap);
        int16_t *q = par + n_cap;
        int &tail = s_tail[w];
        for (int u = lane; u < n; u += 64) {
            const int v = par[u];
            if (v >= 0 && v != j) atomicAdd(&cnt[v], 1);
        }
        wave_sync_bwd();
        for (int u = lane; u < n; u += 64)
            if (par[u] >= 0 && cnt[u] == 0) q[atomicAdd(&tail, 1)] = (int16_t)u;
        int head = 0;
        for (;;) {
            wave_sync_bwd();
            const int end = tail;
            if (head >= end) break;
            for (int x = head + lane; x < end; x += 64) {
                const int u = q[x];
                const int v = par[u];
                const float sv = S[u];
                cnt[u] = -1;                                      // processed
                if (v != j) {
                    atomicAdd(&S[v], sv);
                    if (atomicSub(&cnt[v], 1) == 1) q[atomicAdd(&tail, 1)] = (int16_t)v;
                }
            }
            head = end;
        }
    }
    __syncthreads();

    // ---- the four columns of subtree sums back, row segments together
    if (jc < n) {
        for (int u = r; u < n; u += 64) dWg[(int64_t)u * ld + jc] = cnt_c[u] == -1 ? S_c[u] : 0.0f;
    }
}

// Second pass: row u of every graph.  T[u][j] = S_j(u) (the first pass's
// sums, stored in dW) is scatter-added into bins[next[u][j]], then the row
// becomes the gradient.  j == u and successors outside [0, n) add nothing.
constexpr int kBwdRowsMaxN = 32768;     // 4 bytes of LDS per vertex

__global__ __launch_bounds__(256) void backward_rows_kernel(const int32_t *__restrict__ NX, float *__restrict__ dW,
                                                            int64_t n1, int64_t ld1, const int64_t *__restrict__ off,
                                                            const int32_t *__restrict__ nv, int n_cap) {
    extern __shared__ float bins[];
    int64_t base = 0, ld = ld1;
    int n = (int)n1;
    if (off) {
        n = nv[blockIdx.y];
        base = off[blockIdx.y];
        ld = n;
        if (n < 0 || n > n_cap) return;                      // reported by the first pass
    }
    const int t = threadIdx.x;
    for (int64_t u = blockIdx.x; u < n; u += gridDim.x) {
        const int32_t *nrow = NX + base + u * ld;
        float *drow = dW + base + u * ld;
        for (int v = t; v < n; v += 256) bins[v] = 0.0f;
        __syncthreads();
        for (int jj = t; jj < n; jj += 256) {
            const int v = nrow[jj];
            const float sv = drow[jj];
            if (jj != (int)u && v >= 0 && v < n && sv != 0.0f) atomicAdd(&bins[v], sv);
        }
        __syncthreads();
        for (int v = t; v < n; v += 256) drow[v] = bins[v];
        __syncthreads();
    }
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
    const bool rows = b.n_cap <= kBwdRowsMaxN;
    hipError_t e;
    if (!rows) {                                      // global atomics need a zeroed dW
        const unsigned zx = (unsigned)(b.n_cap < 4096 ? b.n_cap : 4096);
        hipLaunchKernelGGL(zero_grad_kernel, dim3(zx, graphs), dim3(256), 0, b.stream, b.dW, b.n, b.ld, b.off, b.nv,
                           b.n_cap);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (b.n_cap <= kBwdWaveMaxN) {
        const int groups = (b.n_cap + 3) / 4;
        const unsigned gx = (unsigned)(8 * ((groups + 7) / 8));
        const size_t lds = (size_t)4 * 4 * bwd_wave_stride_words(b.n_cap);
        hipLaunchKernelGGL(backward_wave_kernel, dim3(gx, graphs), dim3(256), lds, b.stream, b.G, b.NX, b.dW, b.n,
                           b.ld, b.off, b.nv, b.n_cap, b.err);
    } else if (b.n_cap <= kBackwardLdsMaxN) {
        const unsigned gx = (unsigned)(8 * ((b.n_cap + 7) / 8));
        const size_t lds = (size_t)16 * b.n_cap;
        hipLaunchKernelGGL((backward_kernel<true, true>), dim3(gx, graphs), dim3(kBwdThreads), lds, b.stream, b.G,
                           b.NX, b.dW, b.n, b.ld, b.off, b.nv, b.n_cap, nullptr, b.err);
    } else {
        const unsigned gx = (unsigned)backward_global_workgroups(b);
        if (rows)
            hipLaunchKernelGGL((backward_kernel<false, true>), dim3(gx, graphs), dim3(kBwdThreads), 0, b.stream, b.G,
                               b.NX, b.dW, b.n, b.ld, b.off, b.nv, b.n_cap, b.scratch, b.err);
        else
            hipLaunchKernelGGL((backward_kernel<false, false>), dim3(gx, graphs), dim3(kBwdThreads), 0, b.stream, b.G,
                               b.NX, b.dW, b.n, b.ld, b.off, b.nv, b.n_cap, b.scratch, b.err);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (rows) {
        const unsigned rx = (unsigned)(b.n_cap < 8192 ? b.n_cap : 8192);
        hipLaunchKernelGGL(backward_rows_kernel, dim3(rx, graphs), dim3(256), (size_t)4 * b.n_cap, b.stream, b.NX,
                           b.dW, b.n, b.ld, b.off, b.nv, b.n_cap);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace fw
