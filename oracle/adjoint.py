"""Gradients of a loss of the block MINRES solution, by the adjoint method, in
binary64.

TEST INFRASTRUCTURE (see ``oracle/__init__.py``): only tests, the smoke check
and the benchmark's CPU-baseline leg may use this module.

Not part of the paper: the differentiable solve is an extension built on the
solver of Algorithm 7.1.  What is computed is the textbook derivative of a
linear solve, written out.  For X = A^{-1} B with A symmetric and a scalar
loss L(X) with G = dL/dX:

    dX = A^{-1} (dB - dA X)
    dL = <G, dX> = <Lam, dB> - <Lam X^T, dA>,   Lam = A^{-T} G = A^{-1} G,

so the adjoint system has the same operator and is solved by the same block
MINRES.  Then

    dL/dB = Lam,
    dL/dA restricted to A's pattern and symmetrised (the gradient with respect
        to symmetric perturbations supported on the pattern):
        g_e = -(Lam_i . X_j + Lam_j . X_i) / 2 for the stored entry e = (i, j),
    and for A(theta, sigma) = L + diag(theta) - sigma I:
        dL/dtheta_i = -Lam_i . X_i,   dL/dsigma = sum_i Lam_i . X_i,

where Lam_i . X_j is the dot product of row i of Lam with row j of X.

Pin: central finite differences of dense direct solves (numpy.linalg.solve)
on small systems, in ``tests/test_oracle_adjoint.py``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .block_minres import CONVERGED, solve


def pattern_grad(indptr, indices, Lam, X):
    """g_e = -(Lam_i . X_j + Lam_j . X_i) / 2 for every stored entry e = (i, j)."""
    rows = np.repeat(np.arange(len(indptr) - 1), np.diff(indptr))
    cols = np.asarray(indices)
    return -0.5 * (np.einsum("ec,ec->e", Lam[rows], X[cols]) + np.einsum("ec,ec->e", Lam[cols], X[rows]))


@dataclass
class Grad:
    X: np.ndarray        # forward solution
    Lam: np.ndarray      # adjoint solution A^{-1} G
    dB: np.ndarray       # dL/dB
    dA: np.ndarray       # dL/dA on the pattern (one value per stored entry), symmetrised
    dtheta: np.ndarray   # dL/dtheta for A = L + diag(theta) - sigma I
    dsigma: float        # dL/dsigma


def loss_grad(A, B, G, tol: float = 1e-12, max_iter: int = 100000, indptr=None, indices=None) -> Grad:
    """Forward solve A X = B and adjoint solve A Lam = G with the oracle's
    block MINRES, then the gradients above.  A: scipy CSR (symmetric)."""
    rx = solve(A, B, tol=tol, max_iter=max_iter)
    rl = solve(A, G, tol=tol, max_iter=max_iter)
    if rx.status != CONVERGED or rl.status != CONVERGED:
        raise RuntimeError(f"oracle solves did not converge: {rx.status}, {rl.status}")
    X, Lam = rx.X, rl.X
    indptr = A.indptr if indptr is None else indptr
    indices = A.indices if indices is None else indices
    dA = pattern_grad(indptr, indices, Lam, X)
    xl = np.einsum("ic,ic->i", Lam, X)
    return Grad(X, Lam, Lam.copy(), dA, -xl, float(xl.sum()))
