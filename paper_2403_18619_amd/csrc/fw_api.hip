// C ABI of the blocked Floyd-Warshall solver: argument checks, the plan
// (block size, schedule), the per-device workspace and the launch sequence.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <unordered_map>
#include <vector>

#include "fw.h"
#include "fw_internal.h"

namespace {

thread_local char g_err[512];

fw_status fail(fw_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

fw_status hip_fail(hipError_t e, const char *what) {
    return fail(FW_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

std::mutex g_mu;
std::unordered_map<int, fw::DeviceWork> g_work;

// The per-device workspace is allocated on first use and kept until exit.
fw_status get_work(fw::DeviceWork **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    fw::DeviceWork &w = g_work[dev];
    if (!w.err) {
        e = hipMalloc(&w.err, 256);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
        e = hipMemset(w.err, 0, 256);
        if (e != hipSuccess) return hip_fail(e, "hipMemset(workspace)");
    }
    *out = &w;
    return FW_OK;
}

fw_status check_args(const void *dist, int64_t n, int64_t ld, const fw_options *opt) {
    if (n < 0) return fail(FW_ERR_INVALID_ARG, "n = %lld is negative", (long long)n);
    if (n >= (int64_t)INT32_MAX) return fail(FW_ERR_INVALID_ARG, "n = %lld does not fit the int32 successor matrix", (long long)n);
    if (n == 0) return FW_OK;
    if (!dist) return fail(FW_ERR_INVALID_ARG, "dist is NULL");
    if (ld < n) return fail(FW_ERR_INVALID_ARG, "ld = %lld < n = %lld", (long long)ld, (long long)n);
    if (ld > INT64_MAX / 4 / n) return fail(FW_ERR_INVALID_ARG, "n * ld overflows");
    if (opt) {
        if (opt->block != 0 && opt->block != 32 && opt->block != 64 && opt->block != 128)
            return fail(FW_ERR_INVALID_ARG, "block = %d (allowed: 0, 32, 64, 128)", opt->block);
        if (opt->schedule < FW_SCHED_AUTO || opt->schedule > FW_SCHED_PERSISTENT)
            return fail(FW_ERR_INVALID_ARG, "schedule = %d", opt->schedule);
        if (opt->flags & ~(FW_FLAG_TIME_PHASES | FW_FLAG_EAGER_ARGMIN | FW_FLAG_TEST_TIMEOUT)) return fail(FW_ERR_INVALID_ARG, "flags = %d (unknown bits)", opt->flags);
    }
    return FW_OK;
}

// ---- optional per-phase timing (FW_FLAG_TIME_PHASES)
constexpr int kKinds = 5;
struct Timing {
    std::mutex mu;
    std::vector<hipEvent_t> free_events;
    struct Pending { int kind; hipEvent_t a, b; };
    std::vector<Pending> pending;
};
Timing g_timing;

hipError_t take_event(hipEvent_t *ev) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (!g_timing.free_events.empty()) {
        *ev = g_timing.free_events.back();
        g_timing.free_events.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

// Launch `fn` between two events when timing is on.
template <typename F>
hipError_t timed(bool on, int kind, hipStream_t st, F fn) {
    if (!on) return fn();
    hipEvent_t a, b;
    hipError_t e = take_event(&a);
    if (e != hipSuccess) return e;
    e = take_event(&b);
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(a, st)) != hipSuccess) return e;
    if ((e = fn()) != hipSuccess) return e;
    if ((e = hipEventRecord(b, st)) != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.pending.push_back({kind, a, b});
    return hipSuccess;
}

// Grows a per-device int buffer to at least `need` entries (the old one is
// freed, which waits for the device).
fw_status grow_ints(int **buf, int64_t *cap, int64_t need, const char *what) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (*cap >= need) return FW_OK;
    hipError_t e;
    if (*buf) {
        e = hipFree(*buf);
        if (e != hipSuccess) return hip_fail(e, what);
        *buf = nullptr;
        *cap = 0;
    }
    e = hipMalloc(buf, need * sizeof(int));
    if (e != hipSuccess) return hip_fail(e, what);
    *cap = need;
    return FW_OK;
}

// Persistent schedule: flag workspace of the right size (grown on demand;
// the old one is freed, which waits for the device) and the wait bound.
fw_status persistent_plan(fw::Plan &p, bool test_timeout) {
    const int64_t need = fw::persistent_workspace_ints(p.rounds, p.nt);
    fw_status s = grow_ints(&p.work->persist, &p.work->persist_ints, need, "persistent workspace");
    if (s != FW_OK) return s;
    hipError_t e;
    int dev = 0, khz = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return hip_fail(e, "wall clock rate");
    if (khz <= 0) khz = 100000;
    // a wait never legitimately lasts longer than a few rounds; 20 s is far
    // beyond that and still ends a stuck solve
    p.timeout_ticks = test_timeout ? 0 : (uint64_t)khz * 1000ull * 20ull;
    return FW_OK;
}

int auto_block(int64_t n) {
    if (n <= 32) return 32;
    if (n <= 64) return 64;
    return 128;
}

fw_status solve(fw::DType dt, void *dist, int32_t *next, int64_t n, int64_t ld,
                const fw_options *opt, void *stream) {
    g_err[0] = 0;
    fw_status s = check_args(dist, n, ld, opt);
    if (s != FW_OK || n == 0) return s;
    fw_options o = {0, FW_SCHED_AUTO, 0, 0};
    if (opt) o = *opt;
    // Automatic schedule (measured on MI355X): one persistent launch hides
    // phase 1 and 2 behind the previous round and removes launch gaps; only
    // large solves with successors run slightly faster as three launches.
    bool persistent = o.schedule == FW_SCHED_PERSISTENT;
    if (o.schedule == FW_SCHED_AUTO)
        persistent = (o.block == 0 || o.block == fw::kTile) && n > fw::kTile && !(next && n >= 16384);
    if (persistent && o.block != 0 && o.block != fw::kTile)
        return fail(FW_ERR_UNSUPPORTED, "the persistent schedule runs block size %d only", fw::kTile);

    fw::Plan p;
    p.dtype = dt;
    p.dist = dist;
    p.next = next;
    p.n = n;
    p.ld = ld;
    p.bs = persistent ? fw::kTile : (o.block ? o.block : auto_block(n));
    p.rounds = (int)((n + p.bs - 1) / p.bs);
    p.nt = (int)((n + fw::kTile - 1) / fw::kTile);
    p.vec = (ld % 4 == 0) && ((uintptr_t)dist % 16 == 0);
    p.validate = o.validate != 0;
    p.eager_argmin = (o.flags & FW_FLAG_EAGER_ARGMIN) != 0;
    p.timeout_ticks = 0;
    p.stream = (hipStream_t)stream;
    s = get_work(&p.work);
    if (s != FW_OK) return s;

    const bool tm = (o.flags & FW_FLAG_TIME_PHASES) != 0;
    if (persistent) {
        s = persistent_plan(p, (o.flags & FW_FLAG_TEST_TIMEOUT) != 0);
        if (s != FW_OK) return s;
    }
    hipError_t e = timed(tm, 0, p.stream, [&] { return fw::launch_init(p); });
    if (e != hipSuccess) return hip_fail(e, "init launch");
    if (persistent) {
        e = timed(tm, 4, p.stream, [&] { return fw::launch_persistent(p); });
        if (e != hipSuccess) return hip_fail(e, "persistent launch");
        return FW_OK;
    }
    for (int K = 0; K < p.rounds; ++K) {
        e = timed(tm, 1, p.stream, [&] { return fw::launch_phase1(p, K); });
        if (e != hipSuccess) return hip_fail(e, "phase 1 launch");
        if (p.rounds == 1) break;
        e = timed(tm, 2, p.stream, [&] { return fw::launch_phase2(p, K); });
        if (e != hipSuccess) return hip_fail(e, "phase 2 launch");
        e = timed(tm, 3, p.stream, [&] { return fw::launch_phase3(p, K); });
        if (e != hipSuccess) return hip_fail(e, "phase 3 launch");
    }
    return FW_OK;
}

fw_status solve_batched(fw::DType dt, void *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                        int32_t batch, int32_t n_max, const fw_options *opt, void *stream) {
    g_err[0] = 0;
    if (batch < 0) return fail(FW_ERR_INVALID_ARG, "batch = %d is negative", batch);
    if (batch == 0) return FW_OK;
    if (!dist || !d_offset || !d_n) return fail(FW_ERR_INVALID_ARG, "dist, d_offset and d_n must not be NULL");
    if (n_max < 1 || n_max > 65536)
        return fail(FW_ERR_INVALID_ARG, "n_max = %d (allowed: 1 .. 65536)", n_max);
    fw_options o = {0, FW_SCHED_AUTO, 0, 0};
    if (opt) {
        if (opt->flags & ~(FW_FLAG_EAGER_ARGMIN)) return fail(FW_ERR_INVALID_ARG, "flags = %d", opt->flags);
        if (opt->block != 0 && opt->block != fw::kTile)
            return fail(FW_ERR_UNSUPPORTED, "batched solves run block size %d only", fw::kTile);
        o = *opt;
    }
    fw::DeviceWork *work = nullptr;
    fw_status s = get_work(&work);
    if (s != FW_OK) return s;
    s = grow_ints(&work->batch, &work->batch_ints, (int64_t)n_max + 2 + batch, "batch workspace");
    if (s != FW_OK) return s;
    fw::BatchPlan b;
    b.dtype = dt;
    b.dist = dist;
    b.next = next;
    b.off = d_offset;
    b.nv = d_n;
    b.batch = batch;
    b.n_max = n_max;
    b.validate = o.validate != 0;
    b.eager_argmin = (o.flags & FW_FLAG_EAGER_ARGMIN) != 0;
    b.scratch = work->batch;
    b.err = work->err;
    b.stream = (hipStream_t)stream;
    hipError_t e = fw::launch_batched(b);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return FW_OK;
}

fw_status backward(const float *G, const int32_t *next, float *dW, int64_t n, int64_t ld, const int64_t *d_offset,
                   const int32_t *d_n, int32_t batch, int32_t n_max, void *stream) {
    g_err[0] = 0;
    fw::BackwardPlan b;
    b.G = G;
    b.NX = next;
    b.dW = dW;
    b.n = n;
    b.ld = ld;
    b.off = d_offset;
    b.nv = d_n;
    b.batch = batch;
    b.scratch = nullptr;
    b.stream = (hipStream_t)stream;
    if (!d_offset) {                           // one graph
        fw_status s = check_args(G, n, ld, nullptr);
        if (s != FW_OK || n == 0) return s;
        if (!next || !dW) return fail(FW_ERR_INVALID_ARG, "next and grad_w must not be NULL");
        b.n_cap = (int)n;
    } else {
        if (batch < 0) return fail(FW_ERR_INVALID_ARG, "batch = %d is negative", batch);
        if (batch == 0) return FW_OK;
        if (batch > 65535) return fail(FW_ERR_UNSUPPORTED, "batch = %d (at most 65535 graphs per call)", batch);
        if (!G || !next || !dW || !d_n) return fail(FW_ERR_INVALID_ARG, "pointer arguments must not be NULL");
        if (n_max < 1 || n_max > fw::kBackwardLdsMaxN)
            return fail(n_max < 1 ? FW_ERR_INVALID_ARG : FW_ERR_UNSUPPORTED,
                        "n_max = %d (batched gradients: 1 .. %d)", n_max, fw::kBackwardLdsMaxN);
        b.n_cap = n_max;
    }
    fw::DeviceWork *work = nullptr;
    fw_status s = get_work(&work);
    if (s != FW_OK) return s;
    b.err = work->err;
    const int64_t need = fw::backward_scratch_ints(b);
    if (need > 0) {
        s = grow_ints(&work->bwd, &work->bwd_ints, need, "backward workspace");
        if (s != FW_OK) return s;
        b.scratch = work->bwd;
    }
    hipError_t e = fw::launch_backward(b);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return FW_OK;
}

}  // namespace

extern "C" {

fw_status fw_backward_f32(const float *grad_dist, const int32_t *next, float *grad_w, int64_t n, int64_t ld,
                          void *stream) {
    return backward(grad_dist, next, grad_w, n, ld, nullptr, nullptr, 0, 0, stream);
}

fw_status fw_backward_batched_f32(const float *grad_dist, const int32_t *next, float *grad_w,
                                  const int64_t *d_offset, const int32_t *d_n, int32_t batch, int32_t n_max,
                                  void *stream) {
    if (!d_offset && batch > 0) return fail(FW_ERR_INVALID_ARG, "d_offset must not be NULL");
    return backward(grad_dist, next, grad_w, 0, 0, d_offset, d_n, batch, n_max, stream);
}

fw_status fw_solve_batched_i32(int32_t *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                               int32_t batch, int32_t n_max, const fw_options *opt, void *stream) {
    return solve_batched(fw::DType::I32, dist, next, d_offset, d_n, batch, n_max, opt, stream);
}

fw_status fw_solve_batched_f32(float *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                               int32_t batch, int32_t n_max, const fw_options *opt, void *stream) {
    return solve_batched(fw::DType::F32, dist, next, d_offset, d_n, batch, n_max, opt, stream);
}

fw_status fw_solve_i32(int32_t *dist, int32_t *next, int64_t n, int64_t ld, void *stream) {
    return solve(fw::DType::I32, dist, next, n, ld, nullptr, stream);
}

fw_status fw_solve_f32(float *dist, int32_t *next, int64_t n, int64_t ld, void *stream) {
    return solve(fw::DType::F32, dist, next, n, ld, nullptr, stream);
}

fw_status fw_solve_ex_i32(int32_t *dist, int32_t *next, int64_t n, int64_t ld,
                          const fw_options *opt, void *stream) {
    return solve(fw::DType::I32, dist, next, n, ld, opt, stream);
}

fw_status fw_solve_ex_f32(float *dist, int32_t *next, int64_t n, int64_t ld,
                          const fw_options *opt, void *stream) {
    return solve(fw::DType::F32, dist, next, n, ld, opt, stream);
}

fw_status fw_check(void *stream) {
    g_err[0] = 0;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    fw::DeviceWork *w = nullptr;
    fw_status s = get_work(&w);
    if (s != FW_OK) return s;
    int code = 0;
    e = hipMemcpy(&code, w->err, sizeof code, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(error word)");
    if (code == 0) return FW_OK;
    e = hipMemset(w->err, 0, sizeof code);
    if (e != hipSuccess) return hip_fail(e, "hipMemset(error word)");
    if (code == 1) return fail(FW_ERR_NEGATIVE, "a weight is negative or NaN");
    if (code == 2) return fail(FW_ERR_TIMEOUT, "a dependency wait exceeded its bound");
    if (code == 3) return fail(FW_ERR_INVALID_ARG, "a batched graph has n < 0 or n > n_max");
    return fail(FW_ERR_HIP, "device error word %d", code);
}

fw_status fw_phase_times(double *ms, int64_t *launches) {
    g_err[0] = 0;
    std::vector<Timing::Pending> todo;
    {
        std::lock_guard<std::mutex> lk(g_timing.mu);
        todo.swap(g_timing.pending);
    }
    double acc[kKinds] = {0, 0, 0, 0, 0};
    int64_t cnt[kKinds] = {0, 0, 0, 0, 0};
    fw_status st = FW_OK;
    for (auto &pe : todo) {
        if (st == FW_OK) {
            hipError_t e = hipEventSynchronize(pe.b);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, pe.a, pe.b);
            if (e != hipSuccess) {
                st = hip_fail(e, "phase timing events");
            } else {
                acc[pe.kind] += t;
                cnt[pe.kind] += 1;
            }
        }
        std::lock_guard<std::mutex> lk(g_timing.mu);
        g_timing.free_events.push_back(pe.a);
        g_timing.free_events.push_back(pe.b);
    }
    for (int k = 0; k < kKinds; ++k) {
        if (ms) ms[k] = acc[k];
        if (launches) launches[k] = cnt[k];
    }
    return st;
}

const char *fw_status_string(int status) {
    switch (status) {
    case FW_OK: return "FW_OK";
    case FW_ERR_INVALID_ARG: return "FW_ERR_INVALID_ARG: invalid argument";
    case FW_ERR_UNSUPPORTED: return "FW_ERR_UNSUPPORTED: unsupported request";
    case FW_ERR_HIP: return "FW_ERR_HIP: HIP runtime error";
    case FW_ERR_NEGATIVE: return "FW_ERR_NEGATIVE: negative or NaN weight";
    case FW_ERR_TIMEOUT: return "FW_ERR_TIMEOUT: dependency wait timed out";
    default: return "unknown status";
    }
}

const char *fw_last_error(void) { return g_err; }

int32_t fw_version(void) { return (1 << 16) | 0; }

}  // extern "C"
