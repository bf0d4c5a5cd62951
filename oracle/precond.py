"""Preconditioned band-Lanczos block MINRES: incomplete Cholesky IC(0) and
split preconditioning, in binary64.

TEST INFRASTRUCTURE (see ``oracle/__init__.py``): only tests, the smoke check
and the benchmark's CPU-baseline leg may use this module.

The paper's experiments precondition with the incomplete Cholesky factor of
the (negated) Laplacian part of the matrix (Section 8, ``ichol``), but do not
say how the preconditioner enters Algorithm 7.1.  Readings taken here:

  P1  IC(0): C is lower triangular with the sparsity pattern of the lower
      triangle of M (diagonal included) and (C C^T)_{ij} = M_{ij} for every
      (i, j) in that pattern; equivalently, Cholesky's row recurrence with
      every entry outside the pattern dropped:
          C_{ij} = (M_{ij} - sum_{k<j} C_{ik} C_{jk}) / C_{jj}   (j < i, (i,j) in pattern)
          C_{ii} = sqrt(M_{ii} - sum_{k<i} C_{ik}^2)
      For a matrix whose Cholesky factor has no fill (tridiagonal, for one)
      this is the Cholesky factor itself.  A non-positive pivot stops the
      factorisation (IC(0) does not exist for every SPD matrix).
  P2  Split preconditioning with the symmetric positive definite
      M = C C^T: block MINRES (the oracle of ``block_minres``, unchanged) runs
      on the symmetric operator C^{-1} A C^{-T} with right-hand sides
      C^{-1} B, and X = C^{-T} X-hat.  Column i of X_j then minimises
      ||C^{-1}(b_i - A x)|| = ||b_i - A x||_{M^{-1}} over the preconditioned
      block Krylov space, which is what preconditioned MINRES minimises
      (for p = 1: the iterates of MINRES with the preconditioner M^{-1}).
  P3  The stopping test and the residual history are those of the
      preconditioned system: rho_j^{(i)} / ||C^{-1} b_i||.

The triangular solves use a library routine (``spsolve_triangular``).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import LinearOperator, spsolve_triangular

from .block_minres import solve as _bminres


class Ic0Breakdown(ArithmeticError):
    """A pivot of the incomplete factorisation was not positive."""


def ichol0(M) -> sp.csr_matrix:
    """IC(0) factor C (lower triangular CSR, pattern of tril(M)) of a
    symmetric matrix M with a positive incomplete factorisation (P1).

    Row by row: every entry of row i needs the finished rows j < i of its
    pattern and the entries of row i to its left, so rows are taken in order
    and each row's entries from left to right."""
    M = sp.csr_matrix(M)
    M.sort_indices()
    n = M.shape[0]
    rows = []       # rows[i] = (cols ascending, values) of C, diagonal last
    for i in range(n):
        lo, hi = M.indptr[i], M.indptr[i + 1]
        cols = M.indices[lo:hi]
        vals = M.data[lo:hi]
        keep = cols <= i
        cols, vals = cols[keep], vals[keep]
        if len(cols) == 0 or cols[-1] != i:
            raise Ic0Breakdown(f"row {i} has no diagonal entry")
        ci = {}     # computed entries of row i: column -> value
        for c, mij in zip(cols[:-1], vals[:-1]):
            j = int(c)
            jcols, jvals = rows[j]
            s = mij
            for k, cjk in zip(jcols[:-1], jvals[:-1]):   # k < j
                cik = ci.get(int(k))
                if cik is not None:
                    s -= cik * cjk
            ci[j] = s / jvals[-1]
        d = vals[-1] - sum(v * v for v in ci.values())
        if not d > 0.0:
            raise Ic0Breakdown(f"pivot {d} at row {i}")
        rc = np.array(sorted(ci) + [i], dtype=np.int64)
        rv = np.array([ci[k] for k in sorted(ci)] + [np.sqrt(d)])
        rows.append((rc, rv))
    indptr = np.zeros(n + 1, dtype=np.int64)
    for i, (rc, _) in enumerate(rows):
        indptr[i + 1] = indptr[i] + len(rc)
    indices = np.concatenate([r[0] for r in rows])
    data = np.concatenate([r[1] for r in rows])
    return sp.csr_matrix((data, indices, indptr), shape=(n, n))


def apply_cinv(C, X):
    """C^{-1} X (forward substitution, column by column)."""
    X = np.asarray(X, dtype=np.float64)
    return spsolve_triangular(C, X, lower=True)


def apply_cinvt(C, X):
    """C^{-T} X (backward substitution, column by column)."""
    X = np.asarray(X, dtype=np.float64)
    return spsolve_triangular(sp.csr_matrix(C.T), X, lower=False)


def preconditioned_operator(A, C) -> LinearOperator:
    """The symmetric operator C^{-1} A C^{-T} (P2)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]

    def mm(V):
        V = np.asarray(V, dtype=np.float64)
        if V.ndim == 1:
            V = V[:, None]
        return apply_cinv(C, A @ apply_cinvt(C, V))

    return LinearOperator((n, n), matvec=lambda v: mm(v)[:, 0], matmat=mm, dtype=np.float64)


def solve(A, M, B, tol: float = 1e-8, max_iter: int = 1000, gamma: float = 1e-10, n_bench: int = 2,
          seed: int = 0, record: bool = False, C=None):
    """Block MINRES for A X = B preconditioned by IC(0) of M (P1-P3).

    Returns the oracle's Result for the preconditioned system with ``X``
    replaced by C^{-T} X-hat (the solution of A X = B); ``hist`` and the
    stopping test refer to the preconditioned residual (P3).  ``C`` may be
    given to skip the factorisation."""
    if C is None:
        C = ichol0(M)
    Bh = apply_cinv(C, B)
    if Bh.ndim == 1:
        Bh = Bh[:, None]
    r = _bminres(preconditioned_operator(A, C), Bh, tol=tol, max_iter=max_iter, gamma=gamma, n_bench=n_bench,
                 seed=seed, record=record)
    Xh = r.X
    r.X = apply_cinvt(C, Xh).reshape(Xh.shape)
    r.Xhat = Xh
    r.C = C
    return r
