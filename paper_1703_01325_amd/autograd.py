"""Differentiable block-sparse solve x = A^{-1} b for PyTorch.

Forward runs the preconditioned Krylov solve on the GPU.  Backward solves
the adjoint system A^T lambda = dL/dx with the transposed sweeps of the same
preconditioner (M^{-T} = L^{-T} D^{-T} U'^{-T}) and the A^T SpMV, then
returns dL/db = lambda and dL/dA = -lambda x^T restricted to A's stored
blocks (one b x b block per stored block, column-major like Ax).  The
preconditioner is a fixed operator of the solve: it is not differentiated.
"""
from __future__ import annotations

import torch

from .api import BlockILU


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Ax, b, M, method, rtol, maxit, restart):
        x, st, info = M.solve(Ax, b, method=method, rtol=rtol, maxit=maxit, restart=restart)
        if st != 0:
            raise RuntimeError(f"forward solve did not converge: status {st}, {info}")
        ctx.M = M
        ctx.opts = (method, rtol, maxit, restart)
        ctx.save_for_backward(Ax, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        Ax, x = ctx.saved_tensors
        M = ctx.M
        method, rtol, maxit, restart = ctx.opts
        lam, st, info = M.solve(Ax, gx.contiguous(), method=method, rtol=rtol, maxit=maxit, restart=restart,
                                transpose=True)
        if st != 0:
            raise RuntimeError(f"adjoint solve did not converge: status {st}, {info}")
        dA = M.grad_A(lam, x) if ctx.needs_input_grad[0] else None
        db = lam if ctx.needs_input_grad[1] else None
        return dA, db, None, None, None, None, None


def solve(Ax: torch.Tensor, b: torch.Tensor, M: BlockILU, method: str = "bicgstab", rtol: float = 1e-13,
          maxit: int = 5000, restart: int = 30) -> torch.Tensor:
    """x = A^{-1} b, differentiable in Ax and b.  M must have been built with
    transpose=True and factored from the same Ax."""
    if not M.transpose:
        raise ValueError("the preconditioner must be analysed with transpose=True for the adjoint")
    return _Solve.apply(Ax, b, M, method, rtol, maxit, restart)
