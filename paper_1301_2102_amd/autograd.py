"""Differentiable solve: X = A^{-1} B as a torch.autograd.Function.

Not part of the paper.  The forward pass is the block MINRES solve of
Algorithm 7.1 (``bmr_solve``); the backward pass is the adjoint method:

    Lam = A^{-1} dL/dX        (a second block MINRES solve: A is symmetric,
                               so the adjoint system has the same operator)
    dL/dB   = Lam
    dL/dval = -(Lam_i . X_j + Lam_j . X_i) / 2 for the stored entry (i, j)
              (``bmr_pattern_grad``: the gradient restricted to A's pattern,
              symmetrised)

Both solves and the pattern gradient run in the library's HIP kernels; the
map from user parameters to the matrix values (for instance
val = L.val + scatter(theta - sigma) on the diagonal) is ordinary torch code
and differentiates through torch.
"""
from __future__ import annotations

import torch

from . import CONVERGED, BmrError, DeviceCsr, pattern_grad, solve


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, val, B, A: DeviceCsr, opts: dict):
        Av = DeviceCsr(A.n, A.row_ptr, A.col_idx, val.detach().contiguous())
        X, info = solve(Av, B.detach().contiguous(), **opts)
        if info.status != CONVERGED:
            raise BmrError(info.status, "differentiable solve (forward)")
        ctx.A = Av
        ctx.opts = opts
        ctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(ctx, G):
        (X,) = ctx.saved_tensors
        Lam, info = solve(ctx.A, G.contiguous(), **ctx.opts)
        if info.status != CONVERGED:
            raise BmrError(info.status, "differentiable solve (adjoint)")
        dval = pattern_grad(ctx.A, Lam, X) if ctx.needs_input_grad[0] else None
        dB = Lam if ctx.needs_input_grad[1] else None
        return dval, dB, None, None


def solve_diff(A: DeviceCsr, B: torch.Tensor, val: torch.Tensor = None, tol: float = 1e-10,
               max_iter: int = 1_000_000, **kw) -> torch.Tensor:
    """X = A(val)^{-1} B, differentiable with respect to ``val`` (the stored
    values of A, default A.val) and ``B``.  A must stay symmetric: build
    ``val`` from a symmetric parametrisation.  Forward and adjoint solves use
    ``tol`` and ``max_iter`` (and any other ``bmr.solve`` keyword); a solve that
    does not converge raises BmrError.
    """
    val = A.val if val is None else val
    if val.dtype != torch.float64 or val.numel() != A.nnz:
        raise ValueError("val must be a float64 tensor with one value per stored entry of A")
    opts = dict(tol=tol, max_iter=max_iter, **kw)
    return _Solve.apply(val, B, A, opts)
