/*
 * fw.h -- C ABI of the MI355X (gfx950) blocked Floyd-Warshall solver.
 *
 * The operation is all-pairs shortest paths by blocked Floyd-Warshall
 * (Calderon, Rucci, Chichizola, "Enhanced OpenMP Algorithm to Compute
 * All-Pairs Shortest Path on x86 Architectures", Section 2.3): the input is a
 * dense n x n matrix whose entry (i, j) is the weight of edge i -> j, or
 * "infinite" for no edge; the output replaces it, in place, by the length of
 * a shortest path from i to j, and a second matrix records the paths.
 * Section 5 (conclusions and future work) lists a reusable library for
 * third-party C/C++ programs; this header is that library's interface.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All matrix pointers are DEVICE pointers owned by the caller; they must
 *    stay valid until the work enqueued on `stream` has finished.  `stream`
 *    is a hipStream_t passed as void* (NULL = the default stream).  Work is
 *    enqueued asynchronously; a return of FW_OK means "enqueued".
 *  - Row-major storage with leading dimension `ld` (elements, ld >= n); the
 *    distance and next-hop matrices share `ld`.
 *  - int32 weights: an entry >= FW_INF_I32 (2^30) means "no edge" and is
 *    rewritten to FW_INF_I32.  Finite shortest-path lengths must stay below
 *    2^30.  float32 / float64 weights: +INFINITY means "no edge".  Weights
 *    must be >= 0 (no NaN); the diagonal is forced to 0 (self-loops are
 *    ignored).  The float64 entry points (_f64) compute every sum in double
 *    precision (the paper measures float and double, Section 4).
 *  - next (may be NULL: distances only) receives the successor matrix:
 *    next[i][j] is the vertex after i on the chosen shortest path from i to
 *    j, next[i][i] = i, next[i][j] = -1 when j is unreachable.  (The paper's
 *    path matrix P stores the last intermediate vertex instead; a successor
 *    matrix walks a path in order.)  Where several shortest paths tie, any
 *    valid successor matrix may be returned; for a given input, block size
 *    and data type every schedule returns the same bits.  Every successor
 *    walk reaches its destination when the graph has no cycle of zero total
 *    weight; with zero-weight cycles the distances stay exact, but a walk may
 *    circle inside such a cycle (the blocked rounds relax against bands that
 *    already hold the whole round's intermediate vertices, so a path through
 *    a zero-weight cycle can tie with its shortcut).
 *  - Argument errors are detected on the host and returned before anything
 *    is enqueued; the text is then available from fw_last_error().  Errors
 *    found by the device (validate mode, dependency-wait timeout) are
 *    reported by fw_check().  After an error the output contents are
 *    unspecified.
 *  - n == 0 is a valid no-op.  Thread safety: calls from several host threads
 *    are allowed; calls that overlap on the same device share one small
 *    per-device workspace (error word, schedule counters), so concurrent
 *    solves on different streams of one device must be serialised by the
 *    caller.
 *  - Library-owned device memory is allocated on first use.  fw_init(device)
 *    does that set-up ahead of time (error word, the lookahead's stream and
 *    events, the allocation-free entry point's scratch address), so that a
 *    later call can be captured in a hipGraph without an uncaptured call
 *    first, as far as its own buffers are already large enough.
 */
#ifndef FWGPU_FW_H
#define FWGPU_FW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fw_status {
    FW_OK = 0,
    FW_ERR_INVALID_ARG = -1,   /* bad pointer, size, ld or option           */
    FW_ERR_UNSUPPORTED = -2,   /* valid request this build cannot run       */
    FW_ERR_HIP = -3,           /* a HIP runtime call failed (see last error) */
    FW_ERR_NEGATIVE = -4,      /* validate mode: negative or NaN weight      */
    FW_ERR_TIMEOUT = -5        /* persistent schedule: a wait hit its bound  */
} fw_status;

#define FW_INF_I32 1073741824   /* 2^30: int32 "no edge" and unreachable */

/* Element types, for the entry point that takes the type as an argument. */
#define FW_DTYPE_I32 0
#define FW_DTYPE_F32 1
#define FW_DTYPE_F64 2

/* Schedules (fw_options.schedule). */
#define FW_SCHED_AUTO 0         /* library's choice: three launches (or the
                                   autotuned choice for this size)           */
#define FW_SCHED_THREE_LAUNCH 1 /* per round: phase 1, phase 2, phase 3; with
                                   block 128 and >= 3 rounds, phase 3 runs the
                                   next band first and the next round's
                                   phases 1-2 run meanwhile on a library-owned
                                   stream joined back with events (the solve
                                   stays ordered on `stream`, and may be
                                   captured in a hipGraph)                   */
#define FW_SCHED_PERSISTENT 2   /* one launch, per-tile dependency flags;
                                   block size 128 only                       */

typedef struct fw_options {
    int32_t block;     /* block size BS (k-depth of one round): 0 = auto, or 32, 64, 128 */
    int32_t schedule;  /* FW_SCHED_*                                      */
    int32_t validate;  /* non-zero: the device checks every weight (>= 0,
                          not NaN) and fw_check() reports FW_ERR_NEGATIVE  */
    int32_t flags;     /* 0, or FW_FLAG_* bits below                       */
    int32_t team;      /* batched solves: most workgroups that share one
                          graph; 0 = automatic, 1 = one workgroup solves a
                          whole graph (ignored by single solves)           */
} fw_options;

/* fw_options.flags: record a pair of HIP events on the solve's stream around
 * every kernel launch and accumulate their durations per phase (read with
 * fw_phase_times).  The events are stream markers; the kernels are unchanged.
 * (Internally, the three-launch schedule of an int32 solve with successors
 * at block 128 first records, for an entry improved in a phase-3 tile, the
 * vertex it improved through, and turns these tags into successors with one
 * pass after the last round; that pass is timed with phase 3.  The tags never
 * reach the caller.) */
#define FW_FLAG_TIME_PHASES 1
/* fw_options.flags: reference variant of the successor bookkeeping that
 * compares and records k at every relaxation (about 2.5x slower).  It selects
 * the same successors as the default, bit for bit; tests use it as a check. */
#define FW_FLAG_EAGER_ARGMIN 2
/* fw_options.flags, tests only: the persistent schedule's dependency waits
 * get a zero time bound, so a solve ends early with FW_ERR_TIMEOUT (reported
 * by fw_check) and unspecified output. */
#define FW_FLAG_TEST_TIMEOUT 4
/* fw_options.flags, measurements: the three-launch schedule's phase 3 runs
 * the general tile -- the one the persistent schedule runs -- instead of the
 * direct-copy tile, so that the two schedules can be compared with the same
 * tile code.  Same results, bit for bit. */
#define FW_FLAG_GENERAL_TILE 8
/* fw_options.flags, tests only: an int32 solve with successors resolves its
 * successor tags (see below) row by row in memory instead of staging each
 * row in LDS -- the path rows longer than 32768 take.  Same results. */
#define FW_FLAG_TEST_RESOLVE_MEMORY 16

/* Solve in place (Section 2.3, blocked form with block size BS).
 *   dist : n x n (storage n x ld) int32 / float32 weights in, distances out.
 *   next : n x n (storage n x ld) int32 successor matrix out, or NULL.
 *   n    : number of vertices, 0 <= n < 2^31 - 1.
 *   ld   : leading dimension of dist and next, in elements, ld >= max(n, 1).
 * The _ex forms take options (NULL = defaults).  Library-owned device memory
 * (per device, allocated on first use, grown on demand, kept until exit):
 * besides the small workspace, an int32 solve with successors in the
 * three-launch schedule keeps 2 x ceil(n/128) band maxima; at block size 128
 * with 16-byte aligned rows, that solve and a 32-bit solve without
 * successors keep the rounds' operand panels, 4 x 128 x 128 ceil(n/128)
 * int32 (64 MiB at n = 32768), and a phase-3 fix-up list of
 * 2 R + ceil(n/128)^2 int32 (R rounds); a call that has to grow them
 * allocates, so capture a solve in a hipGraph after one uncaptured call of the
 * same or larger n. */
fw_status fw_solve_i32(int32_t *dist, int32_t *next, int64_t n, int64_t ld, void *stream);
fw_status fw_solve_f32(float *dist, int32_t *next, int64_t n, int64_t ld, void *stream);
fw_status fw_solve_ex_i32(int32_t *dist, int32_t *next, int64_t n, int64_t ld,
                          const fw_options *opt, void *stream);
fw_status fw_solve_ex_f32(float *dist, int32_t *next, int64_t n, int64_t ld,
                          const fw_options *opt, void *stream);
fw_status fw_solve_f64(double *dist, int32_t *next, int64_t n, int64_t ld, void *stream);
fw_status fw_solve_ex_f64(double *dist, int32_t *next, int64_t n, int64_t ld,
                          const fw_options *opt, void *stream);

/* Batched solve: `batch` independent graphs in one launch (the batched
 * configuration of the measurements; the paper solves one matrix at a time).
 *   dist, next : one arena each; graph g is the n_g x n_g row-major block at
 *                dist + d_offset[g] (and next + d_offset[g]; next may be NULL
 *                for distances only); blocks must not overlap.
 *   d_offset   : DEVICE array of batch int64 element offsets.
 *   d_n        : DEVICE array of batch int32 sizes n_g (0 = empty graph).
 *   n_max      : host bound on every n_g, 1 .. 65536; a graph with n_g < 0 or
 *                n_g > n_max is skipped and fw_check reports
 *                FW_ERR_INVALID_ARG.
 *   opt        : NULL or options (block 0 or 128, validate, team,
 *                FW_FLAG_EAGER_ARGMIN).
 * Graphs are taken largest first.  With team == 1 one workgroup solves each
 * graph; otherwise a graph of nt = ceil(n_g / 128) tiles per side is shared
 * by a team of up to min(nt^2, team) workgroups that run the persistent
 * schedule (per-tile flags, dependency waits bounded as for single solves:
 * FW_ERR_TIMEOUT from fw_check).  team == 0 takes the limit from the tuned
 * table that fw_tune_batched_* filled for this data type, successor choice
 * and nt of n_max, else 1 when nt <= 2 and 2 nt above.
 * Each graph gets the same results as fw_solve_ex_* with block size 128.  The
 * call enqueues at most four kernels and no allocation after the first call
 * with a given (batch, n_max, team) size or smaller, so it can be captured in
 * a hipGraph. */
fw_status fw_solve_batched_i32(int32_t *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                               int32_t batch, int32_t n_max, const fw_options *opt, void *stream);
fw_status fw_solve_batched_f32(float *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                               int32_t batch, int32_t n_max, const fw_options *opt, void *stream);
fw_status fw_solve_batched_f64(double *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                               int32_t batch, int32_t n_max, const fw_options *opt, void *stream);

/* Allocation-free batched solve: fw_solve_batched_* with the library's
 * scratch taken from a fixed-size device array instead of device memory it
 * allocates.  For callers that cannot allocate: code under hipGraph capture
 * (including a first call), tight serving loops, and harnesses that forbid
 * hipMalloc.  It never calls hipMalloc, hipFree or any other allocating
 * routine.
 *   dtype : FW_DTYPE_I32, FW_DTYPE_F32 or FW_DTYPE_F64; dist points to that
 *           element type.
 *   other arguments and results: as fw_solve_batched_*.
 * Limit: the scratch holds 2^20 - 64 int32 (4 MiB per device, kept until the
 * process ends); a batch whose order arrays and team flags need more --
 * n_max + 2 batch + 67 ints for team 1, plus batch x (21 ceil(n_max/128) + 4,
 * rounded up to 16) with teams -- returns FW_ERR_UNSUPPORTED with the sizes
 * in fw_last_error() and enqueues nothing.  Its device error word is part of
 * that array and is reported (and cleared) by fw_check like the others.
 * Every call on one device uses the same array and leaves its contents
 * behind (each call clears what must start at zero): calls that overlap on
 * one device, on any streams, race and must be serialised by the caller.
 * The array's address is resolved once per device (fw_init, else the first
 * call on that device). */
fw_status fw_solve_batched_static(int32_t dtype, void *dist, int32_t *next, const int64_t *d_offset,
                                  const int32_t *d_n, int32_t batch, int32_t n_max, const fw_options *opt,
                                  void *stream);

/* Set-up of the library on `device` ahead of the first solve: the per-device
 * workspace (error word), the three-launch lookahead's stream and events, and
 * the allocation-free entry point's scratch address.  Restores the caller's
 * current device; synchronises `device`.  Optional: every entry point does
 * the part it needs on first use.  Errors: FW_ERR_INVALID_ARG for a device
 * index outside [0, device count), FW_ERR_HIP. */
fw_status fw_init(int device);

/* Autotuners.  Each times its candidate configurations on the caller's own
 * input -- dist is copied to a scratch buffer first and restored before every
 * run and on return, so dist still holds its input afterwards (next holds the
 * last run's output) -- and records the fastest in a per-process table that
 * the automatic choices (block 0 with FW_SCHED_AUTO; team 0) consult for the
 * same data type, successor choice and size.  Each call synchronises
 * `stream`, allocates and frees a scratch copy of dist, and takes about
 * (candidates x (reps + 1)) solves.  Not for use under hipGraph capture.
 *
 * fw_tune_solve_*: candidates block 32, 64, 128 with three launches per
 * round, and the persistent schedule; the table key is (dtype, next != NULL,
 * n).  Arguments as fw_solve_ex_*; reps >= 1 timed runs per candidate;
 * outputs (host, may be NULL): the winning block, schedule and its mean
 * milliseconds. */
fw_status fw_tune_solve_i32(int32_t *dist, int32_t *next, int64_t n, int64_t ld, int32_t reps, int32_t *best_block,
                            int32_t *best_schedule, double *best_ms, void *stream);
fw_status fw_tune_solve_f32(float *dist, int32_t *next, int64_t n, int64_t ld, int32_t reps, int32_t *best_block,
                            int32_t *best_schedule, double *best_ms, void *stream);
fw_status fw_tune_solve_f64(double *dist, int32_t *next, int64_t n, int64_t ld, int32_t reps, int32_t *best_block,
                            int32_t *best_schedule, double *best_ms, void *stream);

/* fw_tune_batched_*: candidates team = 1, 2, 4, ... up to nt^2 (nt = tiles
 * per side of an n_max graph); the table key is (dtype, next != NULL, nt).
 * Arguments as fw_solve_batched_*, plus elems = number of elements of the
 * dist arena to restore (covering every graph) and reps as above; outputs:
 * the winning team limit and its mean milliseconds. */
fw_status fw_tune_batched_i32(int32_t *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                              int32_t batch, int32_t n_max, int64_t elems, int32_t reps, int32_t *best_team,
                              double *best_ms, void *stream);
fw_status fw_tune_batched_f32(float *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                              int32_t batch, int32_t n_max, int64_t elems, int32_t reps, int32_t *best_team,
                              double *best_ms, void *stream);
fw_status fw_tune_batched_f64(double *dist, int32_t *next, const int64_t *d_offset, const int32_t *d_n,
                              int32_t batch, int32_t n_max, int64_t elems, int32_t reps, int32_t *best_team,
                              double *best_ms, void *stream);

/* Gradient of the distances with respect to the edge weights, float32.
 *
 * After a solve with a successor matrix, every distance D[i][j] (i != j,
 * reachable) is the sum of the weights along the selected path
 * i -> next[i][j] -> next[next[i][j]][j] -> ... -> j.  Given the upstream
 * gradient grad_dist = dL/dD of a loss L, this writes
 *     grad_w[u][v] = sum of grad_dist[i][j] over the pairs (i, j), i != j,
 *                    whose selected path uses the edge (u, v),
 * which is dL/dW wherever the shortest paths are unique (elsewhere it is the
 * gradient along the selected paths).  Diagonal entries, unreachable pairs
 * and edges on no selected path get 0.  The weights themselves are not
 * needed: the successor matrix carries the paths.
 *
 *  grad_dist : device, n x n at stride ld, read only
 *  next      : device, n x n at stride ld, the successor matrix of the solve
 *              (read only); an entry outside [0, n) counts as "no path" and
 *              a successor cycle contributes nothing beyond it
 *  grad_w    : device, n x n at stride ld, overwritten; must not overlap
 *              grad_dist or next
 * Entries are summed with float atomics, so the last bits can differ from
 * run to run.  For n > 4096 the library keeps a scratch buffer of about
 * 16 MiB per 1024 vertices (allocated on first use, kept until exit).
 * Errors: FW_ERR_INVALID_ARG for n < 0, ld < n or NULL pointers. */
fw_status fw_backward_f32(const float *grad_dist, const int32_t *next, float *grad_w, int64_t n, int64_t ld,
                          void *stream);

/* The same for a batch packed as for fw_solve_batched_*: graph g is the
 * d_n[g] x d_n[g] row-major block at element d_offset[g] of grad_dist, next
 * and grad_w.  d_offset / d_n are device arrays; n_max (host) bounds every
 * d_n[g] and must be at most 4096 (FW_ERR_UNSUPPORTED otherwise); batch at
 * most 65535.  A graph with d_n[g] outside [0, n_max] is skipped and
 * reported by fw_check as FW_ERR_INVALID_ARG.  Enqueues a fixed sequence of
 * kernels (no allocation), so it can be captured in a hipGraph. */
fw_status fw_backward_batched_f32(const float *grad_dist, const int32_t *next, float *grad_w,
                                  const int64_t *d_offset, const int32_t *d_n, int32_t batch, int32_t n_max,
                                  void *stream);

/* Waits for `stream`, then returns (and clears) the first error the device
 * recorded for the current device since the last fw_check: FW_ERR_NEGATIVE,
 * FW_ERR_TIMEOUT, or FW_OK. */
fw_status fw_check(void *stream);

/* Kernel time accumulated by solves run with FW_FLAG_TIME_PHASES since the
 * previous call, per kind of launch: index 0 input normalisation, 1 phase 1,
 * 2 phase 2, 3 phase 3 (with its fix-up launches and the successor
 * resolution pass), 4 persistent (whole solve).  Waits for the recorded
 * events, writes total milliseconds to ms[0..4] and launch counts to
 * launches[0..4] (host pointers, either may be NULL), then resets. */
fw_status fw_phase_times(double *ms, int64_t *launches);

/* Static description of a status code. */
const char *fw_status_string(int status);

/* Detail text of the last error returned on the calling host thread. */
const char *fw_last_error(void);

/* ABI version: (major << 16) | minor. */
int32_t fw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FWGPU_FW_H */
