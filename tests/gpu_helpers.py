"""Shared helpers of the GPU parity tests: run the HIP solver through the C ABI
on seeded inputs and compare with the oracle."""
from __future__ import annotations

import functools
import sys

import numpy as np

import oracle
import synth

INF = 1 << 30


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_solve(W, next_hop=True, block=0, schedule=0, ld=None, stream=None, flags=0):
    """Copy W to the GPU (optionally into an n x ld buffer), solve, copy back."""
    import torch
    import paper_2403_18619_amd as fw
    n = W.shape[0]
    dt = {np.dtype(np.int32): torch.int32, np.dtype(np.float32): torch.float32,
          np.dtype(np.float64): torch.float64}[W.dtype]
    ld = n if ld is None else ld
    D = torch.empty((n, max(ld, 1)), dtype=dt, device="cuda")[:, :n]
    D.copy_(torch.from_numpy(np.ascontiguousarray(W)))
    NX = torch.empty((n, max(ld, 1)), dtype=torch.int32, device="cuda")[:, :n] if next_hop else None
    fw.solve_(D, NX, block=block, schedule=schedule, stream=stream, flags=flags)
    fw.check(stream)
    torch.cuda.synchronize()
    return D.cpu().numpy(), (NX.cpu().numpy() if next_hop else None)


@functools.lru_cache(maxsize=64)
def oracle_i32(n, seed, p, lo, hi):
    W = synth.graph_i32(n, seed, p, lo, hi)
    D, NX = oracle.fw_i32(W)
    return W, D, NX


@functools.lru_cache(maxsize=64)
def oracle_f32(n, seed, p, a, b):
    W = synth.graph_f32(n, seed, p, a, b)
    D, NX = oracle.fw_f64(W)
    return W, D, NX


def assert_close_f32(Dg, D64, rtol=1e-5):
    """float32 distances vs the float64 oracle: same reachability, relative 1e-5."""
    inf_g = np.isinf(Dg)
    inf_o = np.isinf(D64)
    assert (inf_g == inf_o).all(), f"reachability differs at {np.argwhere(inf_g != inf_o)[:5]}"
    fin = ~inf_o
    err = np.abs(Dg[fin].astype(np.float64) - D64[fin])
    tol = rtol * np.abs(D64[fin])
    bad = err > tol
    assert not bad.any(), (f"{bad.sum()} entries beyond rtol {rtol}; worst rel "
                           f"{(err / np.maximum(np.abs(D64[fin]), 1e-300)).max():.3g}")


def assert_walks(W, D, NX, rows=None, rtol=1e-5):
    bad, first = oracle.validate_walk(W, D, NX, rows=rows, rtol=rtol)
    assert bad == 0, f"{bad} bad successor walks; first (i, j, reason) = {first}"


def assert_next_unique_or_tied(W, D64, NXo, NXg, rtol=1e-5):
    """Successors must equal the oracle's except where the GPU's choice h is
    itself a shortest path within rtol (a near-tie in float32)."""
    diff = np.argwhere(NXg != NXo)
    Wd = W.astype(np.float64)
    for i, j in diff:
        h = NXg[i, j]
        assert h >= 0 and i != j, (i, j, h)
        alt = Wd[i, h] + D64[h, j]
        assert abs(alt - D64[i, j]) <= rtol * abs(D64[i, j]), (i, j, h, alt, D64[i, j])
    return len(diff)


def pool_size():
    """Worker threads for host-side checks: the machine's CPU share (16 per GPU)
    or fewer where the machine has fewer cores."""
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_many(graphs, fn=None):
    """Float64 oracle distances of many small graphs, one OpenMP thread per
    graph and a pool of host threads over the graphs (the C calls release
    the GIL).  Returns the list of distance matrices."""
    from concurrent.futures import ThreadPoolExecutor
    fn = fn or (lambda W: oracle.fw_f64(W, next_hop=False, nthreads=1)[0])
    with ThreadPoolExecutor(pool_size()) as ex:
        return list(ex.map(fn, graphs))
