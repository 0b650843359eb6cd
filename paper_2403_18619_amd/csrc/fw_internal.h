// Internal interface between the host dispatcher and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

constexpr int kTile = 128;     // output tile edge of the min-plus kernel
constexpr int kThreads = 256;  // threads per workgroup (four wave64s)

enum class DType { I32, F32, F64 };
inline int dtype_bytes(DType d) { return d == DType::F64 ? 8 : 4; }

// Per-device scratch owned by the library (a few words).
struct DeviceWork {
    int *err = nullptr;        // device error word (0 = none)
    int *persist = nullptr;    // persistent-schedule flags and counters
    int64_t persist_ints = 0;  // their capacity
    int *batch = nullptr;      // batched solve: graph order and counts
    int64_t batch_ints = 0;    // its capacity
    int *bwd = nullptr;        // backward, large n: per-workgroup vertex arrays
    int64_t bwd_ints = 0;      // its capacity
    int *bmax = nullptr;       // three-launch schedule: band maxima, 4 nt ints, then 2 block maxima
    int64_t bmax_ints = 0;     // its capacity
    int *panel = nullptr;      // three-launch, block 128: packed operand panels, 4 x 128 x 128 nt
    int64_t panel_ints = 0;    // its capacity
    int *fix = nullptr;        // direct-copy phase 3: 2 R fix-up counters, then an nt^2 tile list
    int64_t fix_ints = 0;      // its capacity
    hipStream_t aux = nullptr; // three-launch lookahead: the next round's phases 1-2
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
};

struct Plan {
    DType dtype;
    void *dist;
    int32_t *next;             // may be null
    int64_t n, ld;
    int bs;                    // block size (k-depth of a round)
    int rounds;                // ceil(n / bs)
    int nt;                    // ceil(n / kTile)
    bool vec;                  // 16-byte global accesses are legal
    bool validate;
    bool eager_argmin;         // successor variant: per-relaxation tracking
    bool general_tile;         // three launches: phase 3 without the direct-copy tile
    bool resolve_in_memory;    // tests: successor resolution without the LDS row copy
    uint64_t timeout_ticks;    // persistent schedule: wait bound (100 MHz ticks)
    hipStream_t stream;
    DeviceWork *work;
};

// A batch of independent graphs (fw_solve_batched_*).
struct BatchPlan {
    DType dtype;
    void *dist;
    int32_t *next;             // may be null
    const int64_t *off;        // device: first element of graph g
    const int32_t *nv;         // device: vertices of graph g
    int batch, n_max;
    bool validate, eager_argmin;
    int team_cap;              // 1: one workgroup per graph; else team schedule
    uint64_t timeout_ticks;    // team schedule: wait bound
    int *scratch;              // batched_workspace_ints(batch, n_max, team_cap) ints
    int *err;
    hipStream_t stream;
};

// Gradient pass (fw_backward.hip): one graph (off == nullptr: n x n at
// stride ld) or a batch packed like the batched solve (row stride n).
constexpr int kBackwardLdsMaxN = 4096;   // per-destination arrays in LDS (16 bytes per vertex)
struct BackwardPlan {
    const float *G;
    const int32_t *NX;
    float *dW;
    int64_t n, ld;             // single graph
    const int64_t *off;        // batch: device offsets (nullptr for one graph)
    const int32_t *nv;         // batch: device sizes
    int batch;
    int n_cap;                 // largest n (single graph: n)
    int *scratch;              // n_cap > kBackwardLdsMaxN: backward_scratch_ints ints
    int *err;
    hipStream_t stream;
};
hipError_t launch_backward(const BackwardPlan &b);
int64_t backward_scratch_ints(const BackwardPlan &b);
int backward_global_workgroups(const BackwardPlan &b);

// Enqueue helpers (fw_kernels.hip).  Each returns the launch's hipError_t.
hipError_t launch_init(const Plan &p);
// zeroes the direct-copy phase 3's fix-up counters (work->fix, 2 R ints)
hipError_t launch_fix_reset(const Plan &p);
hipError_t launch_phase1(const Plan &p, int K);
hipError_t launch_phase2(const Plan &p, int K);
// part 0: every phase-3 tile of round K; 1: the tiles of band K+1 only;
// 2: all but those (block size 128)
hipError_t launch_phase3(const Plan &p, int K, int part = 0);
// after the last round of a solve whose direct-copy phase 3 stored
// successor tags (int32 with successors): one workgroup per row turns them
// into successors; rows of up to kResolveLdsMaxN entries are staged in LDS
constexpr int kResolveLdsMaxN = 32768;
hipError_t launch_resolve(const Plan &p);
hipError_t launch_persistent(const Plan &p);
int64_t persistent_workspace_ints(int rounds, int nt);
hipError_t launch_batched(const BatchPlan &b);
int64_t batched_workspace_ints(int batch, int n_max, int team_cap);

}  // namespace fw
