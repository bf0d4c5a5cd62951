"""Pins of the preconditioned oracle (IC(0) and split preconditioning)
against what the mathematics fixes, independently of the oracle itself:

  * IC(0) of a matrix whose Cholesky factor has no fill (tridiagonal) is the
    Cholesky factor (LAPACK, dense);
  * IC(0) of 2-D/3-D Laplacians and of a random diagonally dominant matrix
    has the defining property (C C^T)_{ij} = M_{ij} on the lower pattern of
    M, with C lower triangular on exactly that pattern and a positive
    diagonal (while C C^T differs from M off the pattern: fill was dropped);
  * the preconditioned solve converges to the dense direct solution;
  * at p = 1 its iterates are those of scipy's preconditioned MINRES with the
    preconditioner (C C^T)^{-1}: the same preconditioned residual norms
    ||C^{-1}(b - A x_k)|| iteration by iteration;
  * with M = I it is the unpreconditioned solve;
  * the residual history is the explicit preconditioned residual.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import oracle
import oracle.precond as pc
from workloads import laplacian, random_symmetric, rhs_normal


def _tridiag(n, seed):
    rng = np.random.default_rng(seed)
    off = -rng.uniform(0.2, 1.0, n - 1)
    diag = np.abs(np.concatenate([[0.0], off])) + np.abs(np.concatenate([off, [0.0]])) + rng.uniform(0.1, 1.0, n)
    return sp.diags([off, diag, off], [-1, 0, 1], format="csr")


@pytest.mark.parametrize("seed", [0, 1])
def test_ichol0_of_tridiagonal_is_cholesky(seed):
    M = _tridiag(60, seed)
    C = pc.ichol0(M).toarray()
    L = np.linalg.cholesky(M.toarray())
    assert np.allclose(C, L, rtol=0, atol=1e-14 * np.abs(L).max())


def _diag_dominant(n, seed):
    A = random_symmetric(n, draws=3, seed=seed).to_scipy().tolil()
    A.setdiag(0.0)
    A = sp.csr_matrix(A)
    A.data = -np.abs(A.data)
    d = np.asarray(abs(A).sum(axis=1)).ravel() + 0.5
    return sp.csr_matrix(A + sp.diags(d))


@pytest.mark.parametrize("which", ["lap2d", "lap3d", "rand"])
def test_ichol0_defining_property(which):
    if which == "lap2d":
        M = laplacian((12, 13), 0.0).to_scipy()
    elif which == "lap3d":
        M = laplacian((6, 5, 4), 0.0).to_scipy()
    else:
        M = _diag_dominant(300, 4)
    C = pc.ichol0(M)
    lower = sp.tril(M).tocsr()
    lower.sort_indices()
    # exactly the lower pattern of M, positive diagonal
    assert np.array_equal(C.indptr, lower.indptr) and np.array_equal(C.indices, lower.indices)
    assert np.all(C.diagonal() > 0)
    P = (C @ C.T).toarray()
    Md = M.toarray()
    rows, cols = lower.nonzero()
    assert np.allclose(P[rows, cols], Md[rows, cols], rtol=0, atol=1e-13 * np.abs(Md).max())
    # and fill outside the pattern was dropped, so C C^T is not M
    assert np.abs(P - Md).max() > 1e-6


def test_ichol0_breakdown_on_indefinite():
    with pytest.raises(pc.Ic0Breakdown):
        pc.ichol0(laplacian((6, 6), 7.0).to_scipy())


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_preconditioned_converges_to_direct_solution(p):
    A = laplacian((9, 8), 0.7).to_scipy()
    M = laplacian((9, 8), 0.0).to_scipy()
    B = rhs_normal(A.shape[0], p, seed=5)
    r = pc.solve(A, M, B, tol=1e-12, max_iter=2000)
    assert r.status == oracle.CONVERGED
    Xd = np.linalg.solve(A.toarray(), B)
    kappa = np.linalg.cond(A.toarray())
    err = np.linalg.norm(r.X - Xd, axis=0) / np.linalg.norm(Xd, axis=0)
    assert err.max() <= 10 * kappa * 1e-12, (err, kappa)


def test_p1_matches_scipy_preconditioned_minres():
    A = laplacian((16, 16), 0.7).to_scipy()
    M = laplacian((16, 16), 0.0).to_scipy()
    b = rhs_normal(256, 1, seed=2)[:, 0]
    # the preconditioned iteration converges fast and both Lanczos processes
    # lose orthogonality from j ~ 25 on (after that each follows its own
    # rounding); compare the iterations before it
    J = 24
    r = pc.solve(A, M, b[:, None], tol=1e-30, max_iter=J, record=True)
    C = r.C
    Minv = sla.LinearOperator(A.shape, matvec=lambda v: pc.apply_cinvt(C, pc.apply_cinv(C, v)))
    xs = []
    sla.minres(A, b, M=Minv, rtol=1e-30, maxiter=J, callback=lambda x: xs.append(x.copy()))
    assert len(xs) == J
    nb = np.linalg.norm(pc.apply_cinv(C, b))
    for j in range(1, J + 1):
        xo = pc.apply_cinvt(C, r.Xs[j - 1][:, 0])
        ro = np.linalg.norm(pc.apply_cinv(C, b - A @ xo)) / nb
        rs = np.linalg.norm(pc.apply_cinv(C, b - A @ xs[j - 1])) / nb
        assert abs(ro - rs) <= 1e-10 * rs, (j, ro, rs)
        # the recurrence residual is the explicit preconditioned one
        assert abs(r.hist[j - 1, 0] - ro) <= 1e-10 * ro, j
    # and the final iterates agree
    assert np.linalg.norm(r.X[:, 0] - xs[-1]) <= 1e-8 * np.linalg.norm(xs[-1])


def test_identity_preconditioner_is_the_plain_solve():
    A = laplacian((7, 6, 5), 0.3).to_scipy()
    B = rhs_normal(A.shape[0], 3, seed=1)
    I = sp.identity(A.shape[0], format="csr")
    r = pc.solve(A, I, B, tol=1e-10, max_iter=500)
    q = oracle.solve(A, B, tol=1e-10, max_iter=500)
    assert r.iters == q.iters and r.status == q.status
    assert np.allclose(r.X, q.X, rtol=0, atol=1e-14 * np.abs(q.X).max())
    assert np.allclose(r.hist, q.hist, rtol=1e-14, atol=0)


@pytest.mark.parametrize("p", [2, 4])
def test_preconditioned_history_is_explicit_residual(p):
    A = laplacian((10, 9, 8), 0.3).to_scipy()
    M = laplacian((10, 9, 8), 0.0).to_scipy()
    B = rhs_normal(A.shape[0], p, seed=3)
    r = pc.solve(A, M, B, tol=1e-30, max_iter=40, record=True)
    C = r.C
    nb = np.linalg.norm(pc.apply_cinv(C, B), axis=0)
    for j in range(1, 41):
        X = pc.apply_cinvt(C, r.Xs[j - 1])
        ex = np.linalg.norm(pc.apply_cinv(C, B - A @ X), axis=0) / nb
        assert np.allclose(r.hist[j - 1], ex, rtol=1e-9, atol=1e-14), j
    # fewer iterations than the unpreconditioned solve to the same tolerance
    rp = pc.solve(A, M, B, tol=1e-8, max_iter=3000)
    ru = oracle.solve(A, B, tol=1e-8, max_iter=3000)
    assert rp.status == ru.status == oracle.CONVERGED
    assert rp.iters < ru.iters
