"""Shortest-path distances as a differentiable torch operation.

Forward: one solve (fw_solve_ex_f32) of the weight matrix, keeping the
successor matrix.  Backward: fw_backward_f32, which routes every upstream
gradient entry dL/dD[i][j] onto the edges of the selected path from i to j.
Both run in the library's HIP kernels.
"""
from __future__ import annotations

import torch

from ._binding import backward_, solve_


class FloydWarshall(torch.autograd.Function):
    """W (n x n float32, device; +inf = no edge) -> (D, NX).  D is
    differentiable with respect to W; NX (int32 successors) is not."""

    @staticmethod
    def forward(ctx, W, block: int = 0, schedule: int = 0):
        if W.dtype != torch.float32:
            raise ValueError("FloydWarshall needs float32 weights")
        D = W.detach().contiguous().clone()
        NX = torch.empty(D.shape, dtype=torch.int32, device=D.device)
        solve_(D, NX, block=block, schedule=schedule)
        ctx.save_for_backward(NX)
        ctx.mark_non_differentiable(NX)
        return D, NX

    @staticmethod
    def backward(ctx, grad_d, grad_nx):
        (NX,) = ctx.saved_tensors
        if grad_d is None:
            return None, None, None
        G = grad_d.contiguous()
        dW = torch.empty_like(G)
        backward_(G, NX, dW)
        return dW, None, None


def shortest_paths(W, block: int = 0, schedule: int = 0):
    """(D, NX) = FloydWarshall.apply(W, block, schedule)."""
    return FloydWarshall.apply(W, block, schedule)
