"""Benchmark: blocked Floyd-Warshall APSP on one MI355X.

Default workload: one directed graph, n = 32768, edge probability 0.8, int32
weights uniform on [1, 10000], "no edge" = 2^30, distances + successor
matrix (the headline configuration).  One step = restore the input into the
working matrix (device-to-device copy) + one full solve (input
normalisation and every round's three phases).  The metric is n^3
relaxations per second (one relaxation = one (k, i, j) triple of the
Floyd-Warshall loop; the paper's GFLOPS = 2 n^3 / t counts two operations per
relaxation).

Prints one JSON line.  Besides the driver's fields it carries
  roofline     : the phase-3 (min-plus) kernel, timed live with HIP events on
                 the solver's stream, against the MI355X VALU lane-op peak
                 (two operations per relaxation);
  cpu_baseline : the CPU oracle (plain triple loop) timed on this host on a
                 bounded sample of the same recipe, on every core and on one;
  dist_only    : the same graph solved for distances only;
  plain_512    : n = 512, edge prob 0.5, int32 U[1,1000] (launch-bound:
                 eager and captured steps);
  dense_8192   : n = 8192 complete graph, float32 U[0,1), block size and
                 schedule autotuned first;
  batched      : 4096 graphs, n ~ U{16..256}, edge prob 0.3, float32
                 U[0.1,10): one captured HIP graph (input restore + batched
                 solve) per step, beside the same graphs solved one call each
                 (the calls captured in one HIP graph; the Python loop too);
  fwdbwd       : 64 complete graphs, n ~ U{64..1024}, float32 U[0.5,1.5),
                 N(0,1) upstream: autotuned batched forward, batched gradient
                 pass, beside per-graph forward solves.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X VALU lane-op peak: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz for 32-bit
# operations (the rate behind the published 157.3 TFLOP/s FP32 vector figure,
# one FMA = one lane-op = two flops); 64-bit operations at half that (78.6
# TFLOP/s FP64 vector).
VALU_PEAK_LANE_OPS = {"i32": 256 * 4 * 32 * 2.4e9, "f32": 256 * 4 * 32 * 2.4e9, "f64": 256 * 4 * 16 * 2.4e9}
# algorithmic operations per relaxation: one add and one minimum (the paper's
# two operations per inner iteration); the successor choice rides in the
# packed keys (int32) or in the chunk-end search and adds none per relaxation
OPS_PER_RELAX = {"i32": 2.0, "f32": 2.0, "f64": 2.0}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("fw_kernels.hip", "fw_internal.h"):
        with open(os.path.join(ROOT, "paper_2403_18619_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload_key: str):
    """HBM traffic of the phase-3 kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "phase3_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get(workload_key)
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def phase3_relaxations(n: int, bs: int) -> int:
    """Relaxations done by all phase-3 launches of one solve: round K updates
    the (n - bk)^2 entries outside its band with bk k's each."""
    tot = 0
    for K in range((n + bs - 1) // bs):
        bk = min(bs, n - K * bs)
        tot += (n - bk) * (n - bk) * bk
    return tot


def cpu_baseline(args):
    """The oracle as it is (plain triple loop, OpenMP over i within each k)
    on this host: every core on a full n = cpu_n solve of the same recipe,
    and one thread on a smaller one (n = cpu_n1)."""
    import oracle
    import synth

    def recipe(m):
        if args.dtype == "i32":
            return synth.graph_i32(m, args.seed, args.p, int(args.lo), int(args.hi)), oracle.fw_i32
        if args.dtype == "f32":
            return synth.graph_f32(m, args.seed, args.p, args.lo, args.hi), oracle.fw_f32
        return synth.graph_f32(m, args.seed, args.p, args.lo, args.hi).astype("float64"), oracle.fw_f64

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    out = {}
    for key, m, th in (("all", args.cpu_n, threads), ("one", args.cpu_n1, 1)):
        W, fn = recipe(m)
        log(f"cpu baseline: oracle on n={m}, {th} thread(s)")
        t0 = time.perf_counter()
        fn(W, next_hop=not args.no_next, nthreads=th)
        out[key] = (m, th, time.perf_counter() - t0)
    m, th, dt = out["all"]
    m1, _, dt1 = out["one"]
    what = "dist+next" if not args.no_next else "dist"
    return {"value": m ** 3 / dt, "unit": "relaxations/s", "cores": th, "kind": "oracle",
            "sample": (f"plain triple-loop oracle, one full solve of the same recipe at n={m} "
                       f"(seed {args.seed}), {what}, {dt:.2f} s on {th} threads; rate scales as n^3 work"),
            "seconds": dt,
            "one_thread": {"value": m1 ** 3 / dt1, "unit": "relaxations/s", "cores": 1,
                           "sample": f"the same oracle, one full solve at n={m1}, {what}, {dt1:.2f} s",
                           "seconds": dt1}}


def _pack(sizes, gen):
    import numpy as np
    offs = np.concatenate([[0], np.cumsum([int(n) * int(n) for n in sizes])[:-1]]).astype(np.int64)
    arena = np.concatenate([gen(int(n), g).reshape(-1) for g, n in enumerate(sizes)])
    return offs, arena


def _time_graph(torch, graph, stream, reps):
    """Mean ms of `reps` replays of a captured HIP graph (events on `stream`)."""
    graph.replay()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        graph.replay()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def _per_graph_loop(torch, fw, Ws, next_hop=True, reps=2):
    """Plain per-graph method: one restore + fw_solve call per graph.
    Returns (ms of the host loop from Python -- which includes the Python and
    ctypes cost of every call --, ms of one replay of the same calls captured
    in a HIP graph -- the kernels alone, launched one graph at a time)."""
    Ds = [torch.empty_like(w) for w in Ws]
    Ns = [torch.empty(w.shape, dtype=torch.int32, device=w.device) for w in Ws] if next_hop else [None] * len(Ws)
    for d, w, nx in zip(Ds, Ws, Ns):                   # warm-up: every size's workspace exists
        d.copy_(w)
        fw.solve_(d, nx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d, w, nx in zip(Ds, Ws, Ns):
        d.copy_(w)
        fw.solve_(d, nx)
    torch.cuda.synchronize()
    fw.check()
    loop_ms = (time.perf_counter() - t0) * 1e3
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for d, w, nx in zip(Ds, Ws, Ns):
            d.copy_(w)
            fw.solve_(d, nx)
    graph_ms = _time_graph(torch, g, torch.cuda.current_stream(), reps)
    fw.check()
    del g
    return loop_ms, graph_ms


def _time_call(torch, fn, reps, pre=None):
    """Mean ms of `reps` eager calls of `fn`, each bracketed by its own HIP
    events on the current stream (the stream the library launches on);
    `pre` (untimed) runs before each call, e.g. to restore the input so that
    every timed solve starts from the same weights."""
    st = torch.cuda.current_stream()
    if pre is not None:
        pre()
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        if pre is not None:
            pre()
        a.record(st)
        fn()
        b.record(st)
    ev[-1][1].synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / reps


def _valu_roofline(relax, ms, what):
    ops = OPS_PER_RELAX["f32"]
    achieved = ops * relax / (ms / 1e3)
    peak = VALU_PEAK_LANE_OPS["f32"]
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "Top/s",
            "frac": achieved / peak, "traffic": None, "kernel": what, "avg_launch_ms": ms,
            "ops_per_relaxation": ops}


def bench_batched(torch, fw, synth, reps):
    import numpy as np
    sizes = [int(x) for x in synth.batch_sizes()]
    offs, arena = _pack(sizes, lambda n, g: synth.batch_graph_f32(n, g))
    relax = float(sum(n ** 3 for n in sizes))
    W0 = torch.from_numpy(arena).cuda()
    D = torch.empty_like(W0)
    NX = torch.empty(W0.numel(), dtype=torch.int32, device="cuda")
    off = torch.from_numpy(offs).cuda()
    sz = torch.from_numpy(np.asarray(sizes, np.int32)).cuda()
    D.copy_(W0)
    team, tune_ms = fw.tune_batched_(D, NX, off, sz, 256, reps=2)
    D.copy_(W0)
    fw.solve_batched_(D, NX, off, sz, 256)
    torch.cuda.synchronize()
    fw.check()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        D.copy_(W0)
        fw.solve_batched_(D, NX, off, sz, 256)
    ms = _time_graph(torch, g, torch.cuda.current_stream(), reps)
    fw.check()
    del g
    call_ms = _time_call(torch, lambda: fw.solve_batched_(D, NX, off, sz, 256), reps, pre=lambda: D.copy_(W0))
    fw.check()
    log(f"batched: {ms:.3f} ms per captured step, {call_ms:.3f} ms per solve call (team {team})")
    Ws = [torch.from_numpy(synth.batch_graph_f32(n, i)).cuda() for i, n in enumerate(sizes)]
    loop_ms, loop_graph_ms = _per_graph_loop(torch, fw, Ws)
    log(f"batched: per-graph loop {loop_ms:.1f} ms from Python, {loop_graph_ms:.1f} ms as a captured graph")
    return {"workload": "4096 directed graphs, n ~ U{16..256}, edge prob 0.3, float32 U[0.1,10), dist + next",
            "graphs": len(sizes), "relaxations": relax, "ms_per_step": ms, "value": relax / (ms / 1e3),
            "unit": "relaxations/s", "team": team, "step": "one HIP graph replay: input restore + fw_solve_batched",
            "roofline": _valu_roofline(relax, call_ms, "fw_solve_batched (order, normalise, solve kernels)"),
            "per_graph_ms": loop_graph_ms, "per_graph_value": relax / (loop_graph_ms / 1e3),
            "per_graph_step": "4096 x (restore + fw_solve_ex) captured in one HIP graph, one stream",
            "per_graph_python_loop_ms": loop_ms,
            "per_graph_python_loop_note": "the same 4096 calls issued from Python: adds the Python and ctypes "
                                          "cost of each call",
            "speedup_vs_per_graph": loop_graph_ms / ms}


def bench_fwdbwd(torch, fw, synth, reps):
    import numpy as np
    sizes = [int(x) for x in synth.fwdbwd_sizes()]
    n_max = max(sizes)
    offs, arena = _pack(sizes, lambda n, g: synth.fwdbwd_graph_f32(n, g))
    _, ups = _pack(sizes, lambda n, g: synth.fwdbwd_upstream(n, g))
    relax = float(sum(n ** 3 for n in sizes))
    W0 = torch.from_numpy(arena).cuda()
    G = torch.from_numpy(ups).cuda()
    D = torch.empty_like(W0)
    NX = torch.empty(W0.numel(), dtype=torch.int32, device="cuda")
    dW = torch.empty_like(W0)
    off = torch.from_numpy(offs).cuda()
    sz = torch.from_numpy(np.asarray(sizes, np.int32)).cuda()
    D.copy_(W0)
    team, _ = fw.tune_batched_(D, NX, off, sz, n_max, reps=2)
    D.copy_(W0)
    fw.solve_batched_(D, NX, off, sz, n_max)
    fw.backward_batched_(G, NX, dW, off, sz, n_max)
    torch.cuda.synchronize()
    fw.check()
    gf = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gf):
        D.copy_(W0)
        fw.solve_batched_(D, NX, off, sz, n_max)
    gb = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gb):
        fw.backward_batched_(G, NX, dW, off, sz, n_max)
    st = torch.cuda.current_stream()
    fwd_ms = _time_graph(torch, gf, st, reps)
    bwd_ms = _time_graph(torch, gb, st, reps)
    fw.check()
    del gf, gb
    fcall_ms = _time_call(torch, lambda: fw.solve_batched_(D, NX, off, sz, n_max), reps, pre=lambda: D.copy_(W0))
    bcall_ms = _time_call(torch, lambda: fw.backward_batched_(G, NX, dW, off, sz, n_max), reps)
    fw.check()
    log(f"fwdbwd: forward {fwd_ms:.3f} ms (team {team}), backward {bwd_ms:.3f} ms")
    Ws = [torch.from_numpy(synth.fwdbwd_graph_f32(n, i)).cuda() for i, n in enumerate(sizes)]
    loop_ms, loop_graph_ms = _per_graph_loop(torch, fw, Ws)
    elems = float(sum(n * n for n in sizes))
    # gradient pass: algorithmic bytes = read the upstream gradient and the
    # successor matrix, write the weight gradient (12 B per entry); the
    # two-pass kernels also write and read back one float per entry (24 B)
    bwd_alg = 12.0 * elems
    return {"workload": "64 complete directed graphs, n ~ U{64..1024}, float32 U[0.5,1.5), upstream N(0,1)",
            "graphs": len(sizes), "relaxations": relax, "team": team,
            "forward_ms": fwd_ms, "backward_ms": bwd_ms, "total_ms": fwd_ms + bwd_ms,
            "forward_value": relax / (fwd_ms / 1e3), "unit": "relaxations/s",
            "fwdbwd_value": relax / ((fwd_ms + bwd_ms) / 1e3),
            "forward_roofline": _valu_roofline(relax, fcall_ms, "fw_solve_batched (team schedule)"),
            "backward_roofline": {"bound": "hbm", "achieved": bwd_alg / (bcall_ms / 1e3) / 1e9, "peak": 8000.0,
                                  "unit": "GB/s", "frac": bwd_alg / (bcall_ms / 1e3) / 8e12, "traffic": None,
                                  "kernel": "fw_backward_batched_f32 (two passes)", "avg_launch_ms": bcall_ms,
                                  "bytes_per_entry": 12, "implementation_bytes_per_entry": 24},
            "per_graph_forward_ms": loop_graph_ms, "per_graph_forward_value": relax / (loop_graph_ms / 1e3),
            "per_graph_step": "64 x (restore + fw_solve_ex) captured in one HIP graph",
            "per_graph_python_loop_ms": loop_ms,
            "speedup_forward_vs_per_graph": loop_graph_ms / fwd_ms}


def profile_extras(torch, fw, synth):
    """The batched (4096 graphs) and forward+backward (64 graphs) workloads
    as plain calls on the current stream, one each after a warm-up call,
    with the library's automatic team choice: a short, capture-free command
    for counter profiles of their kernels."""
    import numpy as np
    for name, sizes, gen, ups in (
            ("batched", [int(x) for x in synth.batch_sizes()], lambda n, g: synth.batch_graph_f32(n, g), None),
            ("fwdbwd", [int(x) for x in synth.fwdbwd_sizes()], lambda n, g: synth.fwdbwd_graph_f32(n, g),
             lambda n, g: synth.fwdbwd_upstream(n, g))):
        n_max = max(sizes)
        offs, arena = _pack(sizes, gen)
        W0 = torch.from_numpy(arena).cuda()
        D = torch.empty_like(W0)
        NX = torch.empty(W0.numel(), dtype=torch.int32, device="cuda")
        off = torch.from_numpy(offs).cuda()
        sz = torch.from_numpy(np.asarray(sizes, np.int32)).cuda()
        for _ in range(2):
            D.copy_(W0)
            fw.solve_batched_(D, NX, off, sz, n_max)
        if ups is not None:
            G = torch.from_numpy(_pack(sizes, ups)[1]).cuda()
            dW = torch.empty_like(W0)
            for _ in range(2):
                fw.backward_batched_(G, NX, dW, off, sz, n_max)
        torch.cuda.synchronize()
        fw.check()
        log(f"profile extras: {name} done")


PHASE_NOTE = ("per kind of launch, the summed durations of its launches (HIP events on the solve's streams); "
              "the next round's phases 1-2 run on a second stream beside phase 3, so the kinds overlap "
              "and their sum exceeds ms_per_step")


def auto_block(n: int, dtype: str = "i32") -> int:
    """The library's automatic block size for a single solve without a tuned
    entry."""
    if n <= 32:
        return 32
    return 64 if n <= (3072 if dtype == "f64" else 4096) else 128


def measure_single(torch, fw, Wd, nx, dtype, steps, warmup, block=0, schedule=0, eff_block=None,
                   traffic_key=None, flags=0):
    """Warm up, then time `steps` solves of Wd (distances, and successors
    when nx is given), each after restoring the input: ms per step, the
    roofline of the dominant kernel (phase 3, or the persistent kernel) and
    the summed kernel time per kind of launch."""
    n = Wd.shape[0]
    bs = eff_block or block or auto_block(n, dtype)
    stream = torch.cuda.current_stream()
    D = torch.empty_like(Wd)

    def step(timing):
        D.copy_(Wd)
        fw.solve_(D, nx, block=block, schedule=schedule, flags=flags | timing, stream=stream)

    log(f"n={n}: warmup x{warmup} ({'dist + next' if nx is not None else 'dist only'})")
    for _ in range(warmup):
        step(0)
    torch.cuda.synchronize()
    fw.check()
    fw.phase_times()
    log(f"n={n}: timing x{steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(fw.FLAG_TIME_PHASES)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fw.check()
    ph = fw.phase_times()
    ms = (t1 - t0) * 1e3 / steps
    log(f"n={n}: {ms:.2f} ms/step, {n ** 3 / (ms / 1e3):.4g} relaxations/s")
    kind = "persistent" if ph["persistent"][1] else "phase3"
    k_ms, k_launches = ph[kind]
    roofline = None
    if k_launches:
        relax_per_solve = phase3_relaxations(n, bs) if kind == "phase3" else n ** 3
        relax_per_launch = relax_per_solve / (k_launches / steps)
        avg_s = k_ms / k_launches / 1e3
        ops = OPS_PER_RELAX[dtype]
        achieved = ops * relax_per_launch / avg_s
        peak = VALU_PEAK_LANE_OPS[dtype]
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                    "unit": "Top/s", "frac": achieved / peak,
                    "traffic": load_traffic(traffic_key) if traffic_key else None,
                    "kernel": kind, "avg_launch_ms": avg_s * 1e3, "launches_per_step": k_launches / steps,
                    "ops_per_relaxation": ops}
    phase_ms = {k: (v[0] / steps) for k, v in ph.items() if v[1]}
    del D
    return ms, roofline, phase_ms


def bench_plain_512(torch, fw, synth, steps):
    """cfg1: one directed graph n = 512, edge prob 0.5, int32 U[1,1000],
    distances + successors.  Launch-bound: timed as eager calls and as
    one captured HIP graph (input restore + solve) per step."""
    n = 512
    Wd = torch.from_numpy(synth.plain_512()).cuda()
    NX = torch.empty((n, n), dtype=torch.int32, device="cuda")
    ms, roof, phase = measure_single(torch, fw, Wd, NX, "i32", steps, 10)
    D = torch.empty_like(Wd)
    g = torch.cuda.CUDAGraph()
    D.copy_(Wd)
    fw.solve_(D, NX)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        D.copy_(Wd)
        fw.solve_(D, NX)
    gms = _time_graph(torch, g, torch.cuda.current_stream(), steps)
    fw.check()
    del g
    log(f"plain n=512: {ms:.3f} ms per eager step, {gms:.3f} ms per captured step")
    return {"workload": "plain FW, one directed graph n=512, edge prob 0.5, int32 U[1,1000], INF 2^30, "
                        "dist + next (seed 1)",
            "n": n, "block": auto_block(n), "schedule": "auto (three launches)", "steps": steps,
            "ms_per_step": ms, "value": n ** 3 / (ms / 1e3), "unit": "relaxations/s",
            "captured_ms_per_step": gms, "captured_value": n ** 3 / (gms / 1e3),
            "roofline": roof, "phase_kernel_ms_per_step": phase}


def bench_dense_8192(torch, fw, synth, steps):
    """cfg2: one complete directed graph n = 8192, float32 U[0,1), distances
    + successors, block size and schedule autotuned on this input first."""
    n = 8192
    Wd = torch.from_numpy(synth.dense_f32(n)).cuda()
    NX = torch.empty((n, n), dtype=torch.int32, device="cuda")
    block, sched, tune_ms = fw.tune_solve_(Wd, NX, reps=2)
    log(f"dense n=8192: tuned block {block}, schedule {sched} ({tune_ms:.1f} ms)")
    ms, roof, phase = measure_single(torch, fw, Wd, NX, "f32", steps, 2, eff_block=block,
                                     traffic_key=f"f32_n{n}_bs{block}_next")
    return {"workload": "blocked FW, one complete directed graph n=8192, float32 U[0,1), dist + next (seed 2), "
                        "block size and schedule autotuned",
            "n": n, "block": block, "schedule": {1: "three-launch", 2: "persistent"}.get(sched, str(sched)),
            "steps": steps, "ms_per_step": ms, "value": n ** 3 / (ms / 1e3), "unit": "relaxations/s",
            "roofline": roof, "phase_kernel_ms_per_step": phase}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--dtype", choices=["i32", "f32", "f64"], default="i32")
    ap.add_argument("--p", type=float, default=0.8)
    ap.add_argument("--lo", type=float, default=1)
    ap.add_argument("--hi", type=float, default=10000)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--no-next", action="store_true")
    ap.add_argument("--general-tile", action="store_true",
                    help="three-launch phase 3 on the general tile (the persistent schedule's tile)")
    ap.add_argument("--cpu-n", type=int, default=8192)
    ap.add_argument("--cpu-n1", type=int, default=2048, help="size of the one-thread oracle run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the distances-only, n=512, n=8192, batched and forward+backward lines")
    ap.add_argument("--extra-reps", type=int, default=5)
    ap.add_argument("--profile-extras", action="store_true",
                    help="for counter profiles: only the batched and forward+backward solves, as plain calls "
                         "(no autotuning, no HIP graphs, no per-graph loops), then exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "row-strip design is described but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2403_18619_amd as fw

    if args.profile_extras:
        profile_extras(torch, fw, synth)
        return

    n = args.n
    log(f"generating n={n} {args.dtype} graph (p={args.p}, U[{args.lo},{args.hi}], seed {args.seed})")
    if args.dtype == "i32":
        W = synth.graph_i32(n, args.seed, args.p, int(args.lo), int(args.hi))
    elif args.dtype == "f32":
        W = synth.graph_f32(n, args.seed, args.p, args.lo, args.hi)
    else:
        W = synth.graph_f32(n, args.seed, args.p, args.lo, args.hi).astype(np.float64)
    dev = torch.device("cuda:0")
    Wd = torch.from_numpy(W).to(dev)
    del W
    NX = None if args.no_next else torch.empty((n, n), dtype=torch.int32, device=dev)
    bs = args.block or auto_block(n, args.dtype)

    def key(nx):
        return f"{args.dtype}_n{n}_bs{bs}_{'next' if nx is not None else 'dist'}"

    gflag = fw.FLAG_GENERAL_TILE if args.general_tile else 0
    ms_per_step, roofline, phase_ms = measure_single(torch, fw, Wd, NX, args.dtype, args.steps, args.warmup,
                                                     args.block, args.schedule, traffic_key=key(NX), flags=gflag)
    value = n ** 3 / (ms_per_step / 1e3)

    # the same graph for distances only, reported beside the primary result
    dist_only = None
    if NX is not None and not args.no_extras:
        d_ms, d_roof, d_phase = measure_single(torch, fw, Wd, None, args.dtype, args.steps, 1, args.block,
                                               args.schedule, traffic_key=key(None), flags=gflag)
        dist_only = {"workload": "the same graph, distances only (next = NULL)", "steps": args.steps,
                     "ms_per_step": d_ms, "value": n ** 3 / (d_ms / 1e3), "unit": "relaxations/s",
                     "roofline": d_roof, "phase_kernel_ms_per_step": d_phase}

    has_next = NX is not None
    del NX, Wd
    torch.cuda.empty_cache()
    batched = fwdbwd = plain = dense = None
    if not args.no_extras:
        plain = bench_plain_512(torch, fw, synth, 200)
        dense = bench_dense_8192(torch, fw, synth, 10)
        torch.cuda.empty_cache()
        batched = bench_batched(torch, fw, synth, args.extra_reps)
        fwdbwd = bench_fwdbwd(torch, fw, synth, args.extra_reps)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args)

    wl = (f"blocked FW, one directed graph n={n}, edge prob {args.p}, "
          f"{ {'i32': 'int32', 'f32': 'float32', 'f64': 'float64'}[args.dtype]} weights U[{args.lo:g},{args.hi:g}]"
          f"{', INF 2^30' if args.dtype == 'i32' else ''}, "
          f"{'dist + int32 next-hop' if has_next else 'dist only'}")
    out = {
        "metric": "n^3 relaxations/s, blocked FW n=32768; batched + fwd/bwd vs plain, 1 GPU",
        "value": value, "unit": "relaxations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"i32": "int32", "f32": "f32", "f64": "f64"}[args.dtype],
        "data": "synthetic (seeded counter-based generator)",
        "config": {"workload": wl, "n": n, "block": bs,
                   "schedule": {0: "auto", 1: "three-launch", 2: "persistent"}[args.schedule],
                   "general_tile": bool(args.general_tile), "next_hop": has_next, "seed": args.seed},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phase_kernel_ms_per_step": phase_ms,
        "phase_kernel_ms_note": PHASE_NOTE,
        "dist_only": dist_only,
        "plain_512": plain,
        "dense_8192": dense,
        "batched": batched,
        "fwdbwd": fwdbwd,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
