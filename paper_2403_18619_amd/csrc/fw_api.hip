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

fw_status check_args(const void *dist, int64_t n, int64_t ld, const fw_options *opt, int elem = 4) {
    if (n < 0) return fail(FW_ERR_INVALID_ARG, "n = %lld is negative", (long long)n);
    if (n >= (int64_t)INT32_MAX) return fail(FW_ERR_INVALID_ARG, "n = %lld does not fit the int32 successor matrix", (long long)n);
    if (n == 0) return FW_OK;
    if (!dist) return fail(FW_ERR_INVALID_ARG, "dist is NULL");
    if (ld < n) return fail(FW_ERR_INVALID_ARG, "ld = %lld < n = %lld", (long long)ld, (long long)n);
    if (ld > INT64_MAX / elem / n) return fail(FW_ERR_INVALID_ARG, "n * ld overflows");
    if (opt) {
        if (opt->block != 0 && opt->block != 32 && opt->block != 64 && opt->block != 128)
            return fail(FW_ERR_INVALID_ARG, "block = %d (allowed: 0, 32, 64, 128)", opt->block);
        if (opt->schedule < FW_SCHED_AUTO || opt->schedule > FW_SCHED_PERSISTENT)
            return fail(FW_ERR_INVALID_ARG, "schedule = %d", opt->schedule);
        if (opt->flags & ~(FW_FLAG_TIME_PHASES | FW_FLAG_EAGER_ARGMIN | FW_FLAG_TEST_TIMEOUT | FW_FLAG_GENERAL_TILE |
                           FW_FLAG_TEST_RESOLVE_MEMORY))
            return fail(FW_ERR_INVALID_ARG, "flags = %d (unknown bits)", opt->flags);
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

// The three-launch lookahead's auxiliary stream and its two events (per
// device, default priority, created on first use and kept until exit).
fw_status get_aux(fw::DeviceWork *w) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (w->aux) return FW_OK;
    hipError_t e = hipStreamCreateWithFlags(&w->aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w->ev_a, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w->ev_b, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "lookahead stream");
    return FW_OK;
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
fw_status wait_bound(bool test_timeout, uint64_t *ticks);

fw_status persistent_plan(fw::Plan &p, bool test_timeout) {
    const int64_t need = fw::persistent_workspace_ints(p.rounds, p.nt);
    fw_status s = grow_ints(&p.work->persist, &p.work->persist_ints, need, "persistent workspace");
    if (s != FW_OK) return s;
    return wait_bound(test_timeout, &p.timeout_ticks);
}

// ---- tuned team limits for batched solves (fw_tune_batched)
std::mutex g_tune_mu;
std::unordered_map<int64_t, int> g_tuned;
int64_t tune_key(fw::DType dt, bool next, int nt) {
    return ((int64_t)nt << 3) | ((int64_t)dt << 1) | (int64_t)next;
}
int tuned_team(fw::DType dt, bool next, int nt) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(tune_key(dt, next, nt));
    return it == g_tuned.end() ? 0 : it->second;
}
// single solves: (block << 8) | schedule per (dtype, successors, n)
std::unordered_map<int64_t, int> g_tuned_solve;
int64_t solve_key(fw::DType dt, bool next, int64_t n) {
    return (n << 3) | ((int64_t)dt << 1) | (int64_t)next;
}
int tuned_solve(fw::DType dt, bool next, int64_t n) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned_solve.find(solve_key(dt, next, n));
    return it == g_tuned_solve.end() ? 0 : it->second;
}

// Automatic block size (no tuned entry).  Up to a few thousand vertices the
// rounds are latency-bound -- each one's phase 1 is a chain of BS dependent
// steps and its band tiles are few -- and block 64 halves that chain for
// twice the rounds; beyond, block 128's longer tiles (and the direct-copy
// phase 3) win.  Measured on MI355X, three launches, ms per solve at block 64
// against 128: int32 with successors n = 512: 1.06 / 1.55, 2048: 3.94 /
// 5.39, 4096: 10.3 / 10.9, 5120: 16.4 / 14.9; float32 with successors 4096:
// 13.2 / 13.8, 6144: 29.9 / 25.6; int32 distances only 2048: 2.94 / 3.45,
// 3072: 5.60 / 5.49; float32 distances only 4096: 7.75 / 8.88; float64 with
// successors 2048: 6.41 / 9.10, 4096: 23.6 / 22.5.
int auto_block(fw::DType dt, int64_t n) {
    if (n <= 32) return 32;
    if (n <= 64) return 64;
    if (n <= (dt == fw::DType::F64 ? 3072 : 4096)) return 64;
    return 128;
}

fw_status solve(fw::DType dt, void *dist, int32_t *next, int64_t n, int64_t ld,
                const fw_options *opt, void *stream) {
    g_err[0] = 0;
    fw_status s = check_args(dist, n, ld, opt, fw::dtype_bytes(dt));
    if (s != FW_OK || n == 0) return s;
    fw_options o = {0, FW_SCHED_AUTO, 0, 0, 0};
    if (opt) o = *opt;
    // Automatic schedule: a tuned choice for this size if there is one, else
    // three launches per round with lookahead.  Measured on MI355X over
    // n = 512 .. 32768, int32 / float32 / float64, with and without
    // successors, three launches beat the persistent schedule in 30 of 36
    // cases and trail it by at most 4% in the others.
    if (o.schedule == FW_SCHED_AUTO && o.block == 0) {
        const int t = tuned_solve(dt, next != nullptr, n);
        if (t) {
            o.block = t >> 8;
            o.schedule = t & 0xff;
        }
    }
    const bool persistent = o.schedule == FW_SCHED_PERSISTENT;
    if (persistent && o.block != 0 && o.block != fw::kTile)
        return fail(FW_ERR_UNSUPPORTED, "the persistent schedule runs block size %d only", fw::kTile);

    fw::Plan p;
    p.dtype = dt;
    p.dist = dist;
    p.next = next;
    p.n = n;
    p.ld = ld;
    p.bs = persistent ? fw::kTile : (o.block ? o.block : auto_block(dt, n));
    p.rounds = (int)((n + p.bs - 1) / p.bs);
    p.nt = (int)((n + fw::kTile - 1) / fw::kTile);
    p.vec = (ld % 4 == 0) && ((uintptr_t)dist % (4 * fw::dtype_bytes(dt)) == 0);   // 4-element vector accesses
    p.validate = o.validate != 0;
    p.eager_argmin = (o.flags & FW_FLAG_EAGER_ARGMIN) != 0;
    p.general_tile = (o.flags & FW_FLAG_GENERAL_TILE) != 0;
    p.resolve_in_memory = (o.flags & FW_FLAG_TEST_RESOLVE_MEMORY) != 0;
    p.timeout_ticks = 0;
    p.stream = (hipStream_t)stream;
    s = get_work(&p.work);
    if (s != FW_OK) return s;

    const bool tm = (o.flags & FW_FLAG_TIME_PHASES) != 0;
    if (persistent) {
        s = persistent_plan(p, (o.flags & FW_FLAG_TEST_TIMEOUT) != 0);
        if (s != FW_OK) return s;
    }
    const bool packed = !persistent && dt == fw::DType::I32 && next && !p.eager_argmin;
    if (packed) {
        // band maxima for the packed-key phase 3 (two round parities)
        s = grow_ints(&p.work->bmax, &p.work->bmax_ints, 4 * (int64_t)p.nt + 2, "band maxima");
        if (s != FW_OK) return s;
    }
    // the direct-copy phase 3 (block 128, aligned rows): int32 with successors
    // in packed keys, float32 with successors (chunk-end search), or 32-bit
    // distances only
    const bool direct = !persistent && !p.general_tile && p.bs == fw::kTile && p.vec &&
                        (packed || (!next && dt != fw::DType::F64) ||
                         (next && dt == fw::DType::F32 && !p.eager_argmin));
    if (direct) {
        // operand panels (two parities, A' and B', 128 rows of 128 nt entries
        // each), fix-up counters (one per phase-3 launch) and tile list
        s = grow_ints(&p.work->panel, &p.work->panel_ints, 4 * (int64_t)fw::kTile * fw::kTile * p.nt,
                      "operand panels");
        if (s != FW_OK) return s;
        s = grow_ints(&p.work->fix, &p.work->fix_ints, 2 * (int64_t)p.rounds + (int64_t)p.nt * p.nt, "fix-up list");
        if (s != FW_OK) return s;
    }
    hipError_t e = timed(tm, 0, p.stream, [&] { return fw::launch_init(p); });
    if (e == hipSuccess && direct) e = fw::launch_fix_reset(p);
    if (e != hipSuccess) return hip_fail(e, "init launch");
    if (persistent) {
        e = timed(tm, 4, p.stream, [&] { return fw::launch_persistent(p); });
        if (e != hipSuccess) return hip_fail(e, "persistent launch");
        return FW_OK;
    }
    // Lookahead (block 128, three rounds or more): phase 3 of round K runs
    // the next band's tiles first; round K+1's phases 1 and 2, which touch
    // only those tiles and the band-K tiles that only they read, then run on
    // an auxiliary stream while the rest of round K's phase 3 runs.  The
    // caller's stream waits for them before round K+1's phase 3, so the solve
    // stays ordered on it (and a captured graph joins both streams).
    const bool ahead = p.bs == fw::kTile && p.rounds >= 3;
    // The direct-copy phase 3 of an int32 solve with successors leaves
    // successor tags (the improving vertex); one pass after the last round
    // turns them into successors (timed with phase 3, whose bookkeeping it
    // completes).
    const bool tags = direct && packed;
    if (!ahead) {
        for (int K = 0; K < p.rounds; ++K) {
            e = timed(tm, 1, p.stream, [&] { return fw::launch_phase1(p, K); });
            if (e != hipSuccess) return hip_fail(e, "phase 1 launch");
            if (p.rounds == 1) break;
            e = timed(tm, 2, p.stream, [&] { return fw::launch_phase2(p, K); });
            if (e != hipSuccess) return hip_fail(e, "phase 2 launch");
            e = timed(tm, 3, p.stream, [&] { return fw::launch_phase3(p, K); });
            if (e != hipSuccess) return hip_fail(e, "phase 3 launch");
        }
    } else {
        s = get_aux(p.work);
        if (s != FW_OK) return s;
        fw::Plan q = p;
        q.stream = p.work->aux;
        e = timed(tm, 1, p.stream, [&] { return fw::launch_phase1(p, 0); });
        if (e == hipSuccess) e = timed(tm, 2, p.stream, [&] { return fw::launch_phase2(p, 0); });
        if (e != hipSuccess) return hip_fail(e, "phase 1/2 launch");
        for (int K = 0; K < p.rounds; ++K) {
            if (K + 1 == p.rounds) {
                e = timed(tm, 3, p.stream, [&] { return fw::launch_phase3(p, K, 0); });
                if (e != hipSuccess) return hip_fail(e, "phase 3 launch");
                break;
            }
            e = timed(tm, 3, p.stream, [&] { return fw::launch_phase3(p, K, 1); });
            if (e == hipSuccess) e = hipEventRecord(p.work->ev_a, p.stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(q.stream, p.work->ev_a, 0);
            if (e == hipSuccess) e = timed(tm, 1, q.stream, [&] { return fw::launch_phase1(q, K + 1); });
            if (e == hipSuccess) e = timed(tm, 2, q.stream, [&] { return fw::launch_phase2(q, K + 1); });
            if (e == hipSuccess) e = hipEventRecord(p.work->ev_b, q.stream);
            if (e == hipSuccess) e = timed(tm, 3, p.stream, [&] { return fw::launch_phase3(p, K, 2); });
            if (e == hipSuccess) e = hipStreamWaitEvent(p.stream, p.work->ev_b, 0);
            if (e != hipSuccess) return hip_fail(e, "lookahead round");
        }
    }
    if (tags && p.rounds > 1) {
        e = timed(tm, 3, p.stream, [&] { return fw::launch_resolve(p); });
        if (e != hipSuccess) return hip_fail(e, "successor resolution launch");
    }
    return FW_OK;
}

// Wall-clock ticks of a dependency wait's bound (20 s; 0 for the test flag).
fw_status wait_bound(bool test_timeout, uint64_t *ticks) {
    hipError_t e;
    int dev = 0, khz = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return hip_fail(e, "wall clock rate");
    if (khz <= 0) khz = 100000;
    *ticks = test_timeout ? 0 : (uint64_t)khz * 1000ull * 20ull;
    return FW_OK;
}

// Automatic team limit: the tuned table when it has an entry for this
// (dtype, successors, largest tile count), else (measured on MI355X) one
// workgroup per graph up to two tiles per side, and 2 nt workgroups above:
// a round's critical path (phase 1, a band tile, a remaining tile) leaves
// larger teams waiting while other graphs could run.
int auto_team(fw::DType dt, bool next, int n_max) {
    const int nt = (n_max + fw::kTile - 1) / fw::kTile;
    const int tuned = tuned_team(dt, next, nt);
    if (tuned > 0) return tuned;
    return nt <= 2 ? 1 : 2 * nt;
}

// ---- allocation-free batched solve (fw_solve_batched_static): the
// scratch is a file-scope device array, one copy per device, whose address
// is resolved once per device (fw_init or the first call) and kept.  The
// first kStaticErrInts ints hold the error word (padded to 256 bytes); the
// batch layout follows.  Host code passes the resolved address, never the
// array's name (a host-side stand-in, not a device address).
constexpr int64_t kStaticScratchInts = int64_t(1) << 20;   // 4 MiB per device
constexpr int64_t kStaticErrInts = 64;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) int scratch[kStaticScratchInts];
std::mutex g_scratch_mu;
int *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (resolved on first use).
fw_status static_scratch(int **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FW_ERR_UNSUPPORTED, "device %d (at most %d devices)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int *p = nullptr;
        e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(FW_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FW_OK;
}

// Device error word of the allocation-free entry point on the current
// device, or nullptr if that device's scratch was never resolved.
int *static_err_word() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// Batched solve.  static_ws: scratch and error word come from the static
// device array (nothing is allocated); otherwise from the per-device
// workspace, grown on demand.
fw_status solve_batched(fw::DType dt, void *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                        int32_t batch, int32_t n_max, const fw_options *opt, void *stream, bool static_ws = false) {
    g_err[0] = 0;
    if (batch < 0) return fail(FW_ERR_INVALID_ARG, "batch = %d is negative", batch);
    if (batch == 0) return FW_OK;
    if (!dist || !d_offset || !d_n) return fail(FW_ERR_INVALID_ARG, "dist, d_offset and d_n must not be NULL");
    if (n_max < 1 || n_max > 65536)
        return fail(FW_ERR_INVALID_ARG, "n_max = %d (allowed: 1 .. 65536)", n_max);
    if (batch > 65535) return fail(FW_ERR_UNSUPPORTED, "batch = %d (at most 65535 graphs per call)", batch);
    fw_options o = {0, FW_SCHED_AUTO, 0, 0, 0};
    if (opt) {
        if (opt->flags & ~(FW_FLAG_EAGER_ARGMIN | FW_FLAG_TEST_TIMEOUT))
            return fail(FW_ERR_INVALID_ARG, "flags = %d", opt->flags);
        if (opt->block != 0 && opt->block != fw::kTile)
            return fail(FW_ERR_UNSUPPORTED, "batched solves run block size %d only", fw::kTile);
        if (opt->team < 0) return fail(FW_ERR_INVALID_ARG, "team = %d is negative", opt->team);
        o = *opt;
    }
    const int team = o.team ? o.team : auto_team(dt, next != nullptr, n_max);
    const int64_t need = fw::batched_workspace_ints(batch, n_max, team);
    int *sc = nullptr, *err = nullptr;
    fw_status s;
    if (static_ws) {
        if (need > kStaticScratchInts - kStaticErrInts)
            return fail(FW_ERR_UNSUPPORTED,
                        "batch = %d, n_max = %d, team = %d needs %lld scratch ints; the allocation-free entry "
                        "point has %lld (use fw_solve_batched_*, or a smaller batch or team)",
                        batch, n_max, team, (long long)need, (long long)(kStaticScratchInts - kStaticErrInts));
        if ((s = static_scratch(&sc)) != FW_OK) return s;
        err = sc;
        sc += kStaticErrInts;
    } else {
        fw::DeviceWork *work = nullptr;
        if ((s = get_work(&work)) != FW_OK) return s;
        if ((s = grow_ints(&work->batch, &work->batch_ints, need, "batch workspace")) != FW_OK) return s;
        sc = work->batch;
        err = work->err;
    }
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
    b.team_cap = team;
    s = wait_bound((o.flags & FW_FLAG_TEST_TIMEOUT) != 0, &b.timeout_ticks);
    if (s != FW_OK) return s;
    b.scratch = sc;
    b.err = err;
    b.stream = (hipStream_t)stream;
    hipError_t e = fw::launch_batched(b);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return FW_OK;
}

// ---- autotuners: time the candidates on the caller's own input (restored
// from a scratch copy before every run) and record the fastest.
struct TuneCtx {
    hipStream_t st;
    void *backup = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    ~TuneCtx() {
        if (backup) (void)hipFree(backup);
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

fw_status device_error() {
    fw::DeviceWork *w = nullptr;
    fw_status s = get_work(&w);
    if (s != FW_OK) return s;
    int code = 0;
    hipError_t e = hipMemcpy(&code, w->err, sizeof code, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(error word)");
    if (code) {
        (void)hipMemset(w->err, 0, sizeof code);
        return fail(code == 2 ? FW_ERR_TIMEOUT : code == 1 ? FW_ERR_NEGATIVE : FW_ERR_INVALID_ARG,
                    "device error %d while tuning", code);
    }
    return FW_OK;
}

// Runs `run` reps times after one warm-up, each after restoring `bytes` of
// dist from the backup; returns the mean time of the run itself.
template <typename F>
fw_status time_runs(TuneCtx &c, void *dist, size_t bytes, int reps, F run, double *ms) {
    hipError_t e;
    double tot = 0;
    for (int r = -1; r < reps; ++r) {
        if ((e = hipMemcpyAsync(dist, c.backup, bytes, hipMemcpyDeviceToDevice, c.st)) != hipSuccess)
            return hip_fail(e, "restore input");
        if ((e = hipEventRecord(c.a, c.st)) != hipSuccess) return hip_fail(e, "event");
        fw_status s = run();
        if (s != FW_OK) return s;
        if ((e = hipEventRecord(c.b, c.st)) != hipSuccess) return hip_fail(e, "event");
        if ((e = hipEventSynchronize(c.b)) != hipSuccess) return hip_fail(e, "event sync");
        float t = 0;
        if ((e = hipEventElapsedTime(&t, c.a, c.b)) != hipSuccess) return hip_fail(e, "event time");
        if (r >= 0) tot += t;
    }
    fw_status s = device_error();
    if (s != FW_OK) return s;
    *ms = tot / reps;
    return FW_OK;
}

fw_status tune_begin(TuneCtx &c, void *dist, size_t bytes, void *stream) {
    c.st = (hipStream_t)stream;
    hipError_t e = hipMalloc(&c.backup, bytes ? bytes : 1);
    if (e != hipSuccess) return hip_fail(e, "tuning backup");
    if ((e = hipEventCreate(&c.a)) != hipSuccess || (e = hipEventCreate(&c.b)) != hipSuccess)
        return hip_fail(e, "tuning events");
    if ((e = hipMemcpyAsync(c.backup, dist, bytes, hipMemcpyDeviceToDevice, c.st)) != hipSuccess)
        return hip_fail(e, "tuning backup copy");
    return FW_OK;
}

fw_status tune_end(TuneCtx &c, void *dist, size_t bytes) {
    hipError_t e = hipMemcpyAsync(dist, c.backup, bytes, hipMemcpyDeviceToDevice, c.st);
    if (e == hipSuccess) e = hipStreamSynchronize(c.st);
    if (e != hipSuccess) return hip_fail(e, "restore input");
    return FW_OK;
}

fw_status tune_batched(fw::DType dt, void *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                       int32_t batch, int32_t n_max, int64_t elems, int32_t reps, int32_t *best_team,
                       double *best_ms, void *stream) {
    g_err[0] = 0;
    if (batch < 0) return fail(FW_ERR_INVALID_ARG, "batch = %d is negative", batch);
    if (batch == 0) return FW_OK;
    if (!dist || !d_offset || !d_n) return fail(FW_ERR_INVALID_ARG, "dist, d_offset and d_n must not be NULL");
    if (n_max < 1 || n_max > 65536) return fail(FW_ERR_INVALID_ARG, "n_max = %d (allowed: 1 .. 65536)", n_max);
    if (elems < 0 || reps < 1) return fail(FW_ERR_INVALID_ARG, "elems = %lld, reps = %d", (long long)elems, reps);
    const size_t bytes = (size_t)elems * fw::dtype_bytes(dt);
    TuneCtx c;
    fw_status s = tune_begin(c, dist, bytes, stream);
    if (s != FW_OK) return s;
    // candidates: 1 (a workgroup per graph), then powers of two up to every
    // tile of the largest graph's round
    const int nt = (n_max + fw::kTile - 1) / fw::kTile;
    const int most = nt * nt;
    std::vector<int> cands;
    for (int v = 1; v < most; v *= 2) cands.push_back(v);
    cands.push_back(most);
    int best = 1;
    double best_t = 1e30;
    for (int cand : cands) {
        fw_options o = {0, FW_SCHED_AUTO, 0, 0, cand};
        double t = 0;
        s = time_runs(c, dist, bytes, reps,
                      [&] { return solve_batched(dt, dist, next, d_offset, d_n, batch, n_max, &o, stream); }, &t);
        if (s != FW_OK) return s;
        if (t < best_t) {
            best_t = t;
            best = cand;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[tune_key(dt, next != nullptr, nt)] = best;
    }
    if ((s = tune_end(c, dist, bytes)) != FW_OK) return s;
    if (best_team) *best_team = best;
    if (best_ms) *best_ms = best_t;
    return FW_OK;
}

fw_status tune_solve(fw::DType dt, void *dist, int32_t *next, int64_t n, int64_t ld, int32_t reps,
                     int32_t *best_block, int32_t *best_schedule, double *best_ms, void *stream) {
    g_err[0] = 0;
    fw_status s = check_args(dist, n, ld, nullptr, fw::dtype_bytes(dt));
    if (s != FW_OK) return s;
    if (reps < 1) return fail(FW_ERR_INVALID_ARG, "reps = %d", reps);
    if (n == 0) return FW_OK;
    const size_t bytes = (size_t)((n - 1) * ld + n) * fw::dtype_bytes(dt);
    TuneCtx c;
    if ((s = tune_begin(c, dist, bytes, stream)) != FW_OK) return s;
    const int cands[][2] = {{32, FW_SCHED_THREE_LAUNCH}, {64, FW_SCHED_THREE_LAUNCH},
                            {128, FW_SCHED_THREE_LAUNCH}, {128, FW_SCHED_PERSISTENT}};
    int bb = 128, bsch = FW_SCHED_THREE_LAUNCH;
    double best_t = 1e30;
    for (auto &cd : cands) {
        if (cd[1] == FW_SCHED_PERSISTENT && n <= fw::kTile) continue;
        fw_options o = {cd[0], cd[1], 0, 0, 0};
        double t = 0;
        s = time_runs(c, dist, bytes, reps, [&] { return solve(dt, dist, next, n, ld, &o, stream); }, &t);
        if (s != FW_OK) return s;
        if (t < best_t) {
            best_t = t;
            bb = cd[0];
            bsch = cd[1];
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned_solve[solve_key(dt, next != nullptr, n)] = (bb << 8) | bsch;
    }
    if ((s = tune_end(c, dist, bytes)) != FW_OK) return s;
    if (best_block) *best_block = bb;
    if (best_schedule) *best_schedule = bsch;
    if (best_ms) *best_ms = best_t;
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

fw_status fw_tune_batched_i32(int32_t *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                              int32_t batch, int32_t n_max, int64_t elems, int32_t reps, int32_t *best_team,
                              double *best_ms, void *stream) {
    return tune_batched(fw::DType::I32, dist, next, d_offset, d_n, batch, n_max, elems, reps, best_team, best_ms,
                        stream);
}

fw_status fw_tune_batched_f32(float *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                              int32_t batch, int32_t n_max, int64_t elems, int32_t reps, int32_t *best_team,
                              double *best_ms, void *stream) {
    return tune_batched(fw::DType::F32, dist, next, d_offset, d_n, batch, n_max, elems, reps, best_team, best_ms,
                        stream);
}

fw_status fw_tune_batched_f64(double *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                              int32_t batch, int32_t n_max, int64_t elems, int32_t reps, int32_t *best_team,
                              double *best_ms, void *stream) {
    return tune_batched(fw::DType::F64, dist, next, d_offset, d_n, batch, n_max, elems, reps, best_team, best_ms,
                        stream);
}

fw_status fw_tune_solve_f64(double *dist, int32_t *next, int64_t n, int64_t ld, int32_t reps, int32_t *best_block,
                            int32_t *best_schedule, double *best_ms, void *stream) {
    return tune_solve(fw::DType::F64, dist, next, n, ld, reps, best_block, best_schedule, best_ms, stream);
}

fw_status fw_tune_solve_i32(int32_t *dist, int32_t *next, int64_t n, int64_t ld, int32_t reps, int32_t *best_block,
                            int32_t *best_schedule, double *best_ms, void *stream) {
    return tune_solve(fw::DType::I32, dist, next, n, ld, reps, best_block, best_schedule, best_ms, stream);
}

fw_status fw_tune_solve_f32(float *dist, int32_t *next, int64_t n, int64_t ld, int32_t reps, int32_t *best_block,
                            int32_t *best_schedule, double *best_ms, void *stream) {
    return tune_solve(fw::DType::F32, dist, next, n, ld, reps, best_block, best_schedule, best_ms, stream);
}

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

fw_status fw_solve_batched_f64(double *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                               int32_t batch, int32_t n_max, const fw_options *opt, void *stream) {
    return solve_batched(fw::DType::F64, dist, next, d_offset, d_n, batch, n_max, opt, stream);
}

fw_status fw_solve_f64(double *dist, int32_t *next, int64_t n, int64_t ld, void *stream) {
    return solve(fw::DType::F64, dist, next, n, ld, nullptr, stream);
}

fw_status fw_solve_ex_f64(double *dist, int32_t *next, int64_t n, int64_t ld, const fw_options *opt, void *stream) {
    return solve(fw::DType::F64, dist, next, n, ld, opt, stream);
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

fw_status fw_init(int device) {
    g_err[0] = 0;
    int cur = 0, count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(FW_ERR_INVALID_ARG, "device = %d (%d devices)", device, count);
    if ((e = hipGetDevice(&cur)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    fw::DeviceWork *w = nullptr;
    int *sc = nullptr;
    fw_status s = get_work(&w);
    if (s == FW_OK) s = get_aux(w);
    if (s == FW_OK) s = static_scratch(&sc);
    if (s == FW_OK && (e = hipDeviceSynchronize()) != hipSuccess) s = hip_fail(e, "hipDeviceSynchronize");
    if ((e = hipSetDevice(cur)) != hipSuccess && s == FW_OK) s = hip_fail(e, "hipSetDevice");
    return s;
}

fw_status fw_solve_batched_static(int32_t dtype, void *dist, int32_t *next, const int64_t *d_offset,
                                  const int32_t *d_n, int32_t batch, int32_t n_max, const fw_options *opt,
                                  void *stream) {
    g_err[0] = 0;
    fw::DType dt;
    switch (dtype) {
    case FW_DTYPE_I32: dt = fw::DType::I32; break;
    case FW_DTYPE_F32: dt = fw::DType::F32; break;
    case FW_DTYPE_F64: dt = fw::DType::F64; break;
    default: return fail(FW_ERR_INVALID_ARG, "dtype = %d", dtype);
    }
    return solve_batched(dt, dist, next, d_offset, d_n, batch, n_max, opt, stream, true);
}

fw_status fw_check(void *stream) {
    g_err[0] = 0;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    fw::DeviceWork *w = nullptr;
    fw_status s = get_work(&w);
    if (s != FW_OK) return s;
    int code = 0;
    int *werr = w->err;
    e = hipMemcpy(&code, werr, sizeof code, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(error word)");
    if (code == 0) {
        // the allocation-free entry point's error word, if that path ran here
        if (int *se = static_err_word()) {
            werr = se;
            e = hipMemcpy(&code, werr, sizeof code, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy(error word)");
        }
    }
    if (code == 0) return FW_OK;
    e = hipMemset(werr, 0, sizeof code);
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
