"""Blocked Floyd-Warshall all-pairs shortest paths for AMD MI355X (gfx950).

The solver is a C-ABI library (``include/fw.h``, ``libfwgpu.so``) of
hand-written HIP kernels; this package is its thin Python binding.
"""
from ._binding import (FW_ERR_HIP, FW_ERR_INVALID_ARG, FW_ERR_NEGATIVE, FW_ERR_TIMEOUT,
                       FW_ERR_UNSUPPORTED, FLAG_EAGER_ARGMIN, FLAG_GENERAL_TILE, FLAG_TEST_RESOLVE_MEMORY, FLAG_TEST_TIMEOUT, FLAG_TIME_PHASES, FW_INF_I32, FW_OK, LIB_PATH, PHASE_KINDS, SCHED_AUTO,
                       SCHED_PERSISTENT, SCHED_THREE_LAUNCH, DTYPE_F32, DTYPE_F64, DTYPE_I32, FwError, backward_, backward_batched_, check, tune_batched_, tune_solve_,
                       header_symbols,
                       init, last_error, lib, phase_times, solve, solve_, solve_batched_, status_string, version)

from .autograd import FloydWarshall, shortest_paths

__all__ = ["init", "solve", "solve_", "solve_batched_", "DTYPE_I32", "DTYPE_F32", "DTYPE_F64", "backward_", "backward_batched_", "tune_solve_", "tune_batched_",
           "FloydWarshall",
           "shortest_paths", "check", "phase_times", "FLAG_TIME_PHASES", "FLAG_EAGER_ARGMIN", "FLAG_GENERAL_TILE", "FLAG_TEST_RESOLVE_MEMORY", "FLAG_TEST_TIMEOUT", "PHASE_KINDS", "FwError", "lib", "version", "status_string",
           "last_error", "header_symbols", "LIB_PATH", "FW_INF_I32", "SCHED_AUTO",
           "SCHED_THREE_LAUNCH", "SCHED_PERSISTENT", "FW_OK", "FW_ERR_INVALID_ARG",
           "FW_ERR_UNSUPPORTED", "FW_ERR_HIP", "FW_ERR_NEGATIVE", "FW_ERR_TIMEOUT"]
