"""Seeded synthetic graphs for the shortest-path solver, its tests and bench.

This module only draws inputs; it holds none of the shortest-path
arithmetic and is shared by the oracle-side tests and the GPU side alike.
The C source (``synth.c``) documents the counter-based draw.  Workload
recipes below mirror the configurations the solver is measured on.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libfwsynth.so")
_SRC = os.path.join(_HERE, "synth.c")

INF_I32 = 1 << 30   # "no edge" sentinel used for int32 inputs


def build() -> str:
    """Compile libfwsynth.so (host C, OpenMP)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i64, u64, dbl, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int32
        vp = ctypes.c_void_p
        lib.synth_draw.argtypes = [u64, u64, u64, u64]
        lib.synth_draw.restype = u64
        lib.synth_graph_i32.argtypes = [vp, i64, i64, u64, u64, dbl, i32, i32, i32]
        lib.synth_graph_f32.argtypes = [vp, i64, i64, u64, u64, dbl, dbl, dbl]
        lib.synth_uniform_int.argtypes = [vp, i64, u64, u64, i64, i64]
        lib.synth_normal_f32.argtypes = [vp, i64, i64, i64, u64, u64]
        for f in (lib.synth_graph_i32, lib.synth_graph_f32, lib.synth_uniform_int,
                  lib.synth_normal_f32):
            f.restype = None
        _lib = lib
    return _lib


def draw(seed: int, g: int, i: int, j: int) -> int:
    return int(_load().synth_draw(seed, g, i, j))


def graph_i32(n: int, seed: int, p: float, lo: int, hi: int, g: int = 0,
              absent: int = INF_I32, ld: int | None = None) -> np.ndarray:
    """n x n int32 weights (n x ld storage); diagonal 0, absent edges = ``absent``."""
    ld = n if ld is None else ld
    out = np.zeros((n, ld), dtype=np.int32)
    if n:
        _load().synth_graph_i32(out.ctypes.data, n, ld, seed, g, p, lo, hi, absent)
    return out


def graph_f32(n: int, seed: int, p: float, a: float, b: float, g: int = 0,
              ld: int | None = None) -> np.ndarray:
    """n x n float32 weights uniform on [a, b); absent edges = +inf; diagonal 0."""
    ld = n if ld is None else ld
    out = np.zeros((n, ld), dtype=np.float32)
    if n:
        _load().synth_graph_f32(out.ctypes.data, n, ld, seed, g, p, a, b)
    return out


def uniform_int(count: int, seed: int, lo: int, hi: int, g: int = 0) -> np.ndarray:
    out = np.zeros(count, dtype=np.int64)
    if count:
        _load().synth_uniform_int(out.ctypes.data, count, seed, g, lo, hi)
    return out


def normal_f32(rows: int, cols: int, seed: int, g: int = 0) -> np.ndarray:
    out = np.zeros((rows, cols), dtype=np.float32)
    if rows and cols:
        _load().synth_normal_f32(out.ctypes.data, rows, cols, cols, seed, g)
    return out


# ---------------------------------------------------------------------------
# Workload recipes (seed c for workload c).  Sizes and value distributions
# follow the measured configurations; the paper's own inputs are synthetic
# dense matrices with a share of absent entries.

def plain_512(seed: int = 1) -> np.ndarray:
    """n=512 directed graph, edge prob 0.5, int32 weights U[1,1000], INF 2^30."""
    return graph_i32(512, seed, 0.5, 1, 1000)


def dense_f32(n: int = 8192, seed: int = 2) -> np.ndarray:
    """Complete directed graph, float32 weights U[0,1)."""
    return graph_f32(n, seed, 1.0, 0.0, 1.0)


def sparse80_i32(n: int = 32768, seed: int = 3) -> np.ndarray:
    """Directed graph with edge prob 0.8, int32 weights U[1,10000], INF 2^30."""
    return graph_i32(n, seed, 0.8, 1, 10000)


def batch_sizes(count: int = 4096, seed: int = 4, lo: int = 16, hi: int = 256) -> np.ndarray:
    return uniform_int(count, seed, lo, hi, g=0xB47C)


def batch_graph_f32(n: int, index: int, seed: int = 4) -> np.ndarray:
    """Graph ``index`` of the batched workload: edge prob 0.3, f32 U[0.1, 10)."""
    return graph_f32(n, seed, 0.3, 0.1, 10.0, g=index + 1)


def fwdbwd_sizes(count: int = 64, seed: int = 5) -> np.ndarray:
    return uniform_int(count, seed, 64, 1024, g=0xB47C)


def fwdbwd_graph_f32(n: int, index: int, seed: int = 5) -> np.ndarray:
    """Complete graph, f32 U[0.5, 1.5): shortest paths are unique almost surely."""
    return graph_f32(n, seed, 1.0, 0.5, 1.5, g=index + 1)


def fwdbwd_upstream(n: int, index: int, seed: int = 5) -> np.ndarray:
    """Upstream gradient dL/dD ~ N(0,1), float32."""
    return normal_f32(n, n, seed, g=0x10000 + index)
