"""ctypes binding of libfwgpu.so: argument marshalling only.

Every step of a solve runs in the library's HIP kernels; torch provides the
device memory and the stream.  There is no fallback: if the library is not
built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
import re

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfwgpu.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "fw.h")

FW_OK = 0
FW_ERR_INVALID_ARG = -1
FW_ERR_UNSUPPORTED = -2
FW_ERR_HIP = -3
FW_ERR_NEGATIVE = -4
FW_ERR_TIMEOUT = -5
FW_INF_I32 = 1 << 30

SCHED_AUTO, SCHED_THREE_LAUNCH, SCHED_PERSISTENT = 0, 1, 2
DTYPE_I32, DTYPE_F32, DTYPE_F64 = 0, 1, 2
FLAG_TIME_PHASES = 1
FLAG_EAGER_ARGMIN = 2
FLAG_TEST_TIMEOUT = 4
FLAG_GENERAL_TILE = 8
FLAG_TEST_RESOLVE_MEMORY = 16
PHASE_KINDS = ("init", "phase1", "phase2", "phase3", "persistent")


class fw_options(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("flags", ctypes.c_int32), ("team", ctypes.c_int32)]


class FwError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{status_string(status)} ({detail})" if detail else status_string(status))
        self.status = status


def _load():
    # torch ships its own HIP runtime (same soname as the system one); loading
    # it first makes the library bind to it, so the process has one runtime.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python paper_2403_18619_amd/build.py` "
                          "(hipcc, gfx950); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    opt_p = ctypes.POINTER(fw_options)
    for name in ("fw_solve_i32", "fw_solve_f32", "fw_solve_f64"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, i64, i64, vp]
        f.restype = i32
    for name in ("fw_solve_ex_i32", "fw_solve_ex_f32", "fw_solve_ex_f64"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, i64, i64, opt_p, vp]
        f.restype = i32
    for name in ("fw_solve_batched_i32", "fw_solve_batched_f32", "fw_solve_batched_f64"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp, vp, i32, i32, opt_p, vp]
        f.restype = i32
    lib.fw_solve_batched_static.argtypes = [i32, vp, vp, vp, vp, i32, i32, opt_p, vp]
    lib.fw_solve_batched_static.restype = i32
    lib.fw_init.argtypes = [ctypes.c_int]
    lib.fw_init.restype = i32
    lib.fw_backward_f32.argtypes = [vp, vp, vp, i64, i64, vp]
    lib.fw_backward_f32.restype = i32
    lib.fw_backward_batched_f32.argtypes = [vp, vp, vp, vp, vp, i32, i32, vp]
    lib.fw_backward_batched_f32.restype = i32
    for name in ("fw_tune_batched_i32", "fw_tune_batched_f32", "fw_tune_batched_f64"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp, vp, i32, i32, i64, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), vp]
        f.restype = i32
    for name in ("fw_tune_solve_i32", "fw_tune_solve_f32", "fw_tune_solve_f64"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, i64, i64, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                      ctypes.POINTER(ctypes.c_double), vp]
        f.restype = i32
    lib.fw_check.argtypes = [vp]
    lib.fw_check.restype = i32
    lib.fw_status_string.argtypes = [ctypes.c_int]
    lib.fw_status_string.restype = ctypes.c_char_p
    lib.fw_last_error.argtypes = []
    lib.fw_last_error.restype = ctypes.c_char_p
    lib.fw_phase_times.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.fw_phase_times.restype = i32
    lib.fw_version.argtypes = []
    lib.fw_version.restype = i32
    return lib


lib = _load()


def status_string(status: int) -> str:
    return lib.fw_status_string(status).decode()


def last_error() -> str:
    return lib.fw_last_error().decode()


def _raise_if(status: int):
    if status != FW_OK:
        raise FwError(status, last_error())


def header_symbols(path: str = HEADER):
    """Names of every function the C header declares."""
    text = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(fw_\w+)\s*\(", text, re.M)))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_matrix(t, name):
    import torch
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (cuda/hip) tensor")
    if t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError(f"{name} must be a square matrix, got shape {tuple(t.shape)}")
    n = t.shape[0]
    if n and (t.stride(1) != 1 or t.stride(0) < n):
        raise ValueError(f"{name} must be row-major with unit column stride and row stride >= n")
    return n, (t.stride(0) if n else 1)


def solve_(dist, next=None, *, block: int = 0, schedule: int = 0, validate: bool = False,
           stream=None, flags: int = 0):
    """In-place solve of ``dist`` (n x n view of an n x ld row-major matrix).

    ``next``: None (distances only) or an int32 tensor with the same shape and
    strides as ``dist``; receives the successor matrix."""
    import torch
    n, ld = _check_matrix(dist, "dist")
    fn = {torch.int32: lib.fw_solve_ex_i32, torch.float32: lib.fw_solve_ex_f32,
          torch.float64: lib.fw_solve_ex_f64}.get(dist.dtype)
    if fn is None:
        raise ValueError(f"dist dtype {dist.dtype} is not supported (int32, float32 or float64)")
    nptr = None
    if next is not None:
        if next.dtype != torch.int32 or next.shape != dist.shape or (n and next.stride() != dist.stride()):
            raise ValueError("next must be int32 with the same shape and strides as dist")
        if next.device != dist.device:
            raise ValueError("next must be on the same device as dist")
        nptr = next.data_ptr()
    opt = fw_options(block, schedule, 1 if validate else 0, flags, 0)
    with torch.cuda.device(dist.device):
        st = fn(dist.data_ptr(), nptr, n, ld, ctypes.byref(opt), _stream_handle(stream))
    _raise_if(st)
    return dist, next


def solve(W, next_hop: bool = True, *, block: int = 0, schedule: int = 0,
          validate: bool = False, stream=None, flags: int = 0):
    """Out-of-place solve: returns (D, NX) (NX is None when next_hop is False).

    W: square int32 or float32 device tensor of edge weights (int32: >= 2^30
    = no edge; float32: +inf = no edge)."""
    import torch
    n, ld = _check_matrix(W, "W")
    D = torch.empty((n, ld), dtype=W.dtype, device=W.device)[:, :n]
    D.copy_(W)
    NX = torch.empty((n, ld), dtype=torch.int32, device=W.device)[:, :n] if next_hop else None
    solve_(D, NX, block=block, schedule=schedule, validate=validate, stream=stream, flags=flags)
    return D, NX


def init(device: int = 0):
    """Set up the library on a device ahead of the first solve (fw_init)."""
    _raise_if(lib.fw_init(int(device)))


def solve_batched_(dist, next, offsets, sizes, n_max: int, *, validate: bool = False,
                   stream=None, flags: int = 0, team: int = 0, static: bool = False):
    """In-place batched solve.  dist / next: 1-D device arenas (int32 or
    float32 / int32); graph g is the sizes[g] x sizes[g] row-major block at
    element offsets[g].  offsets (int64) and sizes (int32) are device tensors.
    static=True calls the allocation-free entry point
    (fw_solve_batched_static) instead of fw_solve_batched_*."""
    import torch
    for t, name in ((dist, "dist"), (offsets, "offsets"), (sizes, "sizes")):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
    if offsets.dtype != torch.int64 or sizes.dtype != torch.int32:
        raise ValueError("offsets must be int64 and sizes int32")
    if offsets.numel() != sizes.numel():
        raise ValueError("offsets and sizes must have one entry per graph")
    fn = {torch.int32: lib.fw_solve_batched_i32, torch.float32: lib.fw_solve_batched_f32,
          torch.float64: lib.fw_solve_batched_f64}.get(dist.dtype)
    if fn is None:
        raise ValueError(f"dist dtype {dist.dtype} is not supported")
    if next is not None and (next.dtype != torch.int32 or next.numel() < dist.numel()):
        raise ValueError("next must be an int32 arena at least as large as dist")
    opt = fw_options(0, 0, 1 if validate else 0, flags, team)
    args = (dist.data_ptr(), None if next is None else next.data_ptr(), offsets.data_ptr(),
            sizes.data_ptr(), sizes.numel(), int(n_max), ctypes.byref(opt), _stream_handle(stream))
    with torch.cuda.device(dist.device):
        if static:
            dt = {torch.int32: DTYPE_I32, torch.float32: DTYPE_F32, torch.float64: DTYPE_F64}[dist.dtype]
            st = lib.fw_solve_batched_static(dt, *args)
        else:
            st = fn(*args)
    _raise_if(st)
    return dist, next


def backward_(grad_dist, next, grad_w, *, stream=None):
    """grad_w <- gradient of the distances with respect to the edge weights
    along the paths of the successor matrix ``next`` (fw_backward_f32).  All
    three are n x n device tensors with the same strides; grad_w is
    overwritten."""
    import torch
    n, ld = _check_matrix(grad_dist, "grad_dist")
    if grad_dist.dtype != torch.float32 or grad_w.dtype != torch.float32:
        raise ValueError("grad_dist and grad_w must be float32")
    if next.dtype != torch.int32:
        raise ValueError("next must be int32")
    for t, name in ((next, "next"), (grad_w, "grad_w")):
        if t.shape != grad_dist.shape or (n and t.stride() != grad_dist.stride()) or t.device != grad_dist.device:
            raise ValueError(f"{name} must have the shape, strides and device of grad_dist")
    with torch.cuda.device(grad_dist.device):
        st = lib.fw_backward_f32(grad_dist.data_ptr(), next.data_ptr(), grad_w.data_ptr(), n, ld,
                                 _stream_handle(stream))
    _raise_if(st)
    return grad_w


def backward_batched_(grad_dist, next, grad_w, offsets, sizes, n_max: int, *, stream=None):
    """Batched fw_backward: 1-D float32 / int32 / float32 arenas packed as for
    solve_batched_ (graph g: sizes[g] x sizes[g] at element offsets[g])."""
    import torch
    for t, name in ((grad_dist, "grad_dist"), (next, "next"), (grad_w, "grad_w"), (offsets, "offsets"),
                    (sizes, "sizes")):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
    if grad_dist.dtype != torch.float32 or grad_w.dtype != torch.float32 or next.dtype != torch.int32:
        raise ValueError("grad_dist / grad_w must be float32 and next int32")
    if offsets.dtype != torch.int64 or sizes.dtype != torch.int32 or offsets.numel() != sizes.numel():
        raise ValueError("offsets (int64) and sizes (int32) must have one entry per graph")
    if next.numel() < grad_dist.numel() or grad_w.numel() < grad_dist.numel():
        raise ValueError("next and grad_w must be at least as large as grad_dist")
    with torch.cuda.device(grad_dist.device):
        st = lib.fw_backward_batched_f32(grad_dist.data_ptr(), next.data_ptr(), grad_w.data_ptr(),
                                         offsets.data_ptr(), sizes.data_ptr(), sizes.numel(), int(n_max),
                                         _stream_handle(stream))
    _raise_if(st)
    return grad_w


def tune_solve_(dist, next=None, *, reps: int = 2, stream=None):
    """Autotune the block size and schedule of single solves of this size on
    this input (fw_tune_solve_*).  dist keeps its input contents.  Returns
    (block, schedule, mean_ms); later solves with block=0 and the automatic
    schedule use the winner."""
    import torch
    n, ld = _check_matrix(dist, "dist")
    fn = {torch.int32: lib.fw_tune_solve_i32, torch.float32: lib.fw_tune_solve_f32,
          torch.float64: lib.fw_tune_solve_f64}.get(dist.dtype)
    if fn is None:
        raise ValueError(f"dist dtype {dist.dtype} is not supported")
    if next is not None and (next.dtype != torch.int32 or next.shape != dist.shape or
                             (n and next.stride() != dist.stride())):
        raise ValueError("next must be int32 with the same shape and strides as dist")
    bb, bs, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0)
    with torch.cuda.device(dist.device):
        st = fn(dist.data_ptr(), None if next is None else next.data_ptr(), n, ld, reps, ctypes.byref(bb),
                ctypes.byref(bs), ctypes.byref(ms), _stream_handle(stream))
    _raise_if(st)
    return bb.value, bs.value, ms.value


def tune_batched_(dist, next, offsets, sizes, n_max: int, *, reps: int = 2, stream=None):
    """Autotune the team limit of batched solves of this batch
    (fw_tune_batched_*).  dist keeps its input contents.  Returns (team,
    mean_ms); later batched solves with team=0 use the winner."""
    import torch
    fn = {torch.int32: lib.fw_tune_batched_i32, torch.float32: lib.fw_tune_batched_f32,
          torch.float64: lib.fw_tune_batched_f64}.get(dist.dtype)
    if fn is None:
        raise ValueError(f"dist dtype {dist.dtype} is not supported")
    for t, name in ((dist, "dist"), (offsets, "offsets"), (sizes, "sizes")):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
    if offsets.dtype != torch.int64 or sizes.dtype != torch.int32 or offsets.numel() != sizes.numel():
        raise ValueError("offsets (int64) and sizes (int32) must have one entry per graph")
    if next is not None and (next.dtype != torch.int32 or next.numel() < dist.numel()):
        raise ValueError("next must be an int32 arena at least as large as dist")
    team, ms = ctypes.c_int32(0), ctypes.c_double(0)
    with torch.cuda.device(dist.device):
        st = fn(dist.data_ptr(), None if next is None else next.data_ptr(), offsets.data_ptr(), sizes.data_ptr(),
                sizes.numel(), int(n_max), dist.numel(), reps, ctypes.byref(team), ctypes.byref(ms),
                _stream_handle(stream))
    _raise_if(st)
    return team.value, ms.value


def check(stream=None):
    """Wait for the stream and raise the first device-side error, if any."""
    _raise_if(lib.fw_check(_stream_handle(stream)))


def phase_times():
    """{kind: (total_ms, launches)} accumulated by solves run with
    flags=FLAG_TIME_PHASES since the previous call (waits for them)."""
    ms = (ctypes.c_double * 5)()
    cnt = (ctypes.c_int64 * 5)()
    _raise_if(lib.fw_phase_times(ms, cnt))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(PHASE_KINDS)}


def version() -> int:
    return int(lib.fw_version())
