"""CPU oracle for all-pairs shortest paths -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It shares no code with the GPU library
(``paper_2403_18619_amd``) and neither imports the other.

``fw_oracle.c`` is the plain Floyd-Warshall triple loop (Section 2.3, Fig. 1
of the paper), with a strict comparison and a successor ("next hop") matrix;
``validate.c`` checks any distance / next-hop pair by walking paths;
``grad.c`` is the plain definition of the shortest-path gradient (every
selected path walked, its upstream value added to each edge on it).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, "fw_oracle.c"), os.path.join(_HERE, "validate.c"), os.path.join(_HERE, "grad.c")]

INF_I32 = 1 << 30


def build(extra_flags=()) -> str:
    """Compile liboracle.so: plain C, no intrinsics, IEEE arithmetic."""
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-std=c11", *extra_flags, *_SRCS, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


def load_library(path: str = _SO):
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    for name in ("oracle_fw_i32", "oracle_fw_f64", "oracle_fw_f32"):
        f = getattr(lib, name)
        f.argtypes = [vp, i64, i64, vp, vp, i64, i32]
        f.restype = i32
    lib.oracle_sssp_i32.argtypes = [vp, i64, i64, vp, i64, vp, i32]
    lib.oracle_sssp_i32.restype = None
    lib.oracle_sssp_f64.argtypes = [vp, i64, i64, vp, i64, vp, i32]
    lib.oracle_sssp_f64.restype = None
    lib.validate_walk_i32.argtypes = [vp, i64, vp, vp, i64, i64, vp, i64, vp]
    lib.validate_walk_i32.restype = i64
    lib.validate_walk_f32.argtypes = [vp, i64, vp, vp, i64, i64, vp, i64, dbl, vp]
    lib.validate_walk_f32.restype = i64
    lib.validate_walk_f64.argtypes = [vp, i64, vp, vp, i64, i64, vp, i64, dbl, vp]
    lib.validate_walk_f64.restype = i64
    lib.oracle_grad_f64.argtypes = [vp, i64, vp, i64, i64, vp, i64]
    lib.oracle_grad_f64.restype = i64
    return lib


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = load_library()
    return _lib


def _square(W, dtype):
    W = np.ascontiguousarray(W, dtype=dtype)
    assert W.ndim == 2 and W.shape[0] <= W.shape[1]
    return W


def fw_i32(W, next_hop: bool = True, nthreads: int = 0, lib=None):
    """Plain FW on int32 weights (absent >= 2^30).  Returns (D, NX or None)."""
    lib = lib or _L()
    W = _square(W, np.int32)
    n = W.shape[0]
    D = np.empty((n, n), np.int32)
    NX = np.empty((n, n), np.int32) if next_hop else None
    rc = lib.oracle_fw_i32(W.ctypes.data, n, W.shape[1], D.ctypes.data,
                           NX.ctypes.data if next_hop else None, n, nthreads)
    if rc != 0:
        raise ValueError("negative weight")
    return D, NX


def fw_f64(W, next_hop: bool = True, nthreads: int = 0, lib=None):
    """Plain FW with float64 sums (float32 weights convert exactly)."""
    lib = lib or _L()
    W = _square(W, np.float64)
    n = W.shape[0]
    D = np.empty((n, n), np.float64)
    NX = np.empty((n, n), np.int32) if next_hop else None
    rc = lib.oracle_fw_f64(W.ctypes.data, n, W.shape[1], D.ctypes.data,
                           NX.ctypes.data if next_hop else None, n, nthreads)
    if rc != 0:
        raise ValueError("negative or NaN weight")
    return D, NX


def fw_f32(W, next_hop: bool = True, nthreads: int = 0, lib=None):
    """Plain FW with every sum rounded to float32."""
    lib = lib or _L()
    W = _square(W, np.float32)
    n = W.shape[0]
    D = np.empty((n, n), np.float32)
    NX = np.empty((n, n), np.int32) if next_hop else None
    rc = lib.oracle_fw_f32(W.ctypes.data, n, W.shape[1], D.ctypes.data,
                           NX.ctypes.data if next_hop else None, n, nthreads)
    if rc != 0:
        raise ValueError("negative or NaN weight")
    return D, NX


def sssp_i32(W, sources, nthreads: int = 0):
    """Rows ``sources`` of the distance matrix by Dijkstra (int32 weights)."""
    W = _square(W, np.int32)
    n = W.shape[0]
    src = np.ascontiguousarray(sources, dtype=np.int64)
    out = np.empty((len(src), n), np.int32)
    _L().oracle_sssp_i32(W.ctypes.data, n, W.shape[1], src.ctypes.data, len(src),
                         out.ctypes.data, nthreads)
    return out


def sssp_f64(W, sources, nthreads: int = 0):
    """Rows ``sources`` by Dijkstra on float32 weights, float64 sums."""
    W = _square(W, np.float32)
    n = W.shape[0]
    src = np.ascontiguousarray(sources, dtype=np.int64)
    out = np.empty((len(src), n), np.float64)
    _L().oracle_sssp_f64(W.ctypes.data, n, W.shape[1], src.ctypes.data, len(src),
                         out.ctypes.data, nthreads)
    return out


def validate_walk(W, D, NX, rows=None, rtol: float = 1e-5, lib=None):
    """Walk-check rows of (D, NX) against W.  Returns (n_bad, (i, j, reason))."""
    lib = lib or _L()
    n = D.shape[0]
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, np.int64)
    first = np.zeros(3, np.int64)
    NX = np.ascontiguousarray(NX, np.int32)
    if np.issubdtype(D.dtype, np.integer):
        W = np.ascontiguousarray(W, np.int32)
        D = np.ascontiguousarray(D, np.int32)
        bad = lib.validate_walk_i32(W.ctypes.data, W.shape[1], D.ctypes.data, NX.ctypes.data,
                                     D.shape[1], n, rows.ctypes.data, len(rows), first.ctypes.data)
    elif D.dtype == np.float64:
        W = np.ascontiguousarray(W, np.float64)
        D = np.ascontiguousarray(D, np.float64)
        bad = lib.validate_walk_f64(W.ctypes.data, W.shape[1], D.ctypes.data, NX.ctypes.data,
                                     D.shape[1], n, rows.ctypes.data, len(rows), rtol,
                                     first.ctypes.data)
    else:
        W = np.ascontiguousarray(W, np.float32)
        D = np.ascontiguousarray(D, np.float32)
        bad = lib.validate_walk_f32(W.ctypes.data, W.shape[1], D.ctypes.data, NX.ctypes.data,
                                     D.shape[1], n, rows.ctypes.data, len(rows), rtol,
                                     first.ctypes.data)
    return int(bad), tuple(int(x) for x in first)


def triangle_violations(D, ks=None):
    """Count (i, j, k) with D[i][j] > D[i][k] + D[k][j] over the given k's."""
    n = D.shape[0]
    ks = range(n) if ks is None else ks
    Dw = D.astype(np.float64) if D.dtype.kind == "f" else D.astype(np.int64)
    bad = 0
    for k in ks:
        bad += int(np.count_nonzero(Dw > Dw[:, k:k + 1] + Dw[k:k + 1, :]))
    return bad


def grad_ref(G, NX, lib=None):
    """dL/dW for L = sum(G * D): every pair (i, j), i != j, with a path adds
    G[i][j] to each edge of the path that the successor matrix NX selects.
    Float64 result; raises if a walk is broken."""
    lib = lib or _L()
    G = np.ascontiguousarray(G, np.float32)
    NX = np.ascontiguousarray(NX, np.int32)
    n = NX.shape[0]
    out = np.empty((n, n), np.float64)
    bad = lib.oracle_grad_f64(G.ctypes.data, G.shape[1], NX.ctypes.data, NX.shape[1], n,
                              out.ctypes.data, n)
    if bad:
        raise ValueError(f"{bad} successor walks are broken")
    return out


def grad_abs_ref(G, NX, lib=None):
    """The same sums over |G|: the scale of each gradient entry's rounding."""
    return grad_ref(np.abs(np.asarray(G, np.float32)), NX, lib=lib)
