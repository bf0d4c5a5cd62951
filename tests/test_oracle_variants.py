"""Pins of the oracle's two variant modes against constructions made here
from their definitions.

Retained candidates (Section 5.1, last paragraph; reading R13 in
``oracle/block_minres.py``):

  * with the default dependence tolerance nothing is retained (an exactly
    dependent candidate leaves only rounding noise) and the solve is the
    discarding one, bit for bit;
  * a near-dependent candidate is retained in place of the basis vector it
    would have been (u_m), and exactly the new basis vectors u_{m+1} ..
    u_{m+2p} are orthogonal to it: the remainder is rebuilt here from B (or
    from A u_j and the recorded basis) and compared with the recorded basis;
  * the retained steps change the iterate (their coefficients are not in
    H-bar), so the mode is not the discarding one when something is kept.

Accumulated rotations (Section 4's remark; reading R14): the same iterates,
residuals and band factor R as the sequential rotations to rounding, with
the same zero pattern (also through an in-iteration replacement), and the
dense direct solution at convergence.
"""
import numpy as np
import pytest

import oracle
from workloads import laplacian, rhs_near_copy, rhs_near_e1_ae1, rhs_normal, rhs_stress, rhs_e1_ae1


def _A():
    return laplacian((10, 11, 12), 0.3).to_scipy()


def near_initial(A):
    return rhs_near_copy(A.shape[0], p=4)


def near_iteration(A):
    return rhs_near_e1_ae1(laplacian((10, 11, 12), 0.3))


@pytest.mark.parametrize("make", ["copy", "e1ae1"])
def test_default_gamma_retains_nothing(make):
    A = _A()
    B = rhs_stress(A.shape[0], 0, p=4, seed=1) if make == "copy" else rhs_e1_ae1(laplacian((10, 11, 12), 0.3))
    a = oracle.solve(A, B, tol=1e-9, max_iter=3000)
    b = oracle.solve(A, B, tol=1e-9, max_iter=3000, retain=True)
    assert len(a.replaced) >= 1 and b.retained == []
    assert a.iters == b.iters and np.array_equal(a.X, b.X) and np.array_equal(a.hist, b.hist)


def test_retained_at_initial_qr_window():
    A = _A()
    B = near_initial(A)
    p = B.shape[1]
    r = oracle.solve(A, B, tol=1e-30, max_iter=4 * p, gamma=1e-3, retain=True, record=True)
    assert r.replaced == [2] and r.retained == [2]
    U = r.U
    # the removed candidate: b_2 after CGS2 against u_1, normalised
    w = B[:, 1].copy()
    for _ in range(2):
        w -= (U[:, 0] @ w) * U[:, 0]
    rh = w / np.linalg.norm(w)
    m = 2
    for i in range(m + 1, m + 2 * p + 1):        # u_{m+1} .. u_{m+2p}: orthogonal
        assert abs(rh @ U[:, i - 1]) <= 1e-12, i
    # the first vector past the window is no longer kept orthogonal to it
    assert abs(rh @ U[:, m + 2 * p]) > 1e-10
    d = oracle.solve(A, B, tol=1e-30, max_iter=4 * p, gamma=1e-3, record=True)
    assert np.linalg.norm(r.X - d.X) > 1e-8 * np.linalg.norm(d.X)


def test_retained_in_iteration_window():
    A = _A()
    B = near_iteration(A)
    p = B.shape[1]
    r = oracle.solve(A, B, tol=1e-30, max_iter=5 * p, gamma=1e-3, retain=True, record=True)
    m = 1 + p                                     # the candidate of iteration 1 would have been u_{1+p}
    assert r.retained == [m] and r.replaced == [m]
    U = r.U
    # the removed candidate: A u_1 orthogonalised against u_1 .. u_p, normalised
    w = A @ U[:, 0]
    for i in range(p):
        w -= (U[:, i] @ w) * U[:, i]
    rh = w / np.linalg.norm(w)
    for i in range(m + 1, m + 2 * p + 1):
        assert abs(rh @ U[:, i - 1]) <= 1e-12, i
    assert abs(rh @ U[:, m + 2 * p]) > 1e-10


# --------------------------------------------------------------------------
# Accumulated rotations (reading R14): the same mathematics, by matrices
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 2, 3, 4, 8])
def test_accumulated_rotations_equal_sequential(p):
    A = _A()
    B = rhs_normal(A.shape[0], p, seed=p)
    a = oracle.solve(A, B, tol=1e-10, max_iter=3000, record=True)
    b = oracle.solve(A, B, tol=1e-10, max_iter=3000, record=True, accumulate=True)
    assert a.status == b.status == oracle.CONVERGED and a.iters == b.iters
    assert np.abs(a.X - b.X).max() <= 1e-12 * np.abs(a.X).max()
    assert np.abs(a.hist - b.hist).max() <= 1e-14
    # the band QR factor itself: same entries (Givens signs), same zero pattern
    assert np.abs(a.R - b.R).max() <= 1e-12 * np.abs(a.R).max()
    assert np.array_equal(a.R == 0.0, b.R == 0.0)


def test_accumulated_rotations_direct_solution_and_dependence():
    A = laplacian((8, 8), 0.7).to_scipy()
    B = rhs_normal(A.shape[0], 3, seed=11)
    r = oracle.solve(A, B, tol=1e-12, max_iter=1000, accumulate=True)
    Xd = np.linalg.solve(A.toarray(), B)
    kappa = np.linalg.cond(A.toarray())
    assert r.status == oracle.CONVERGED
    assert (np.linalg.norm(r.X - Xd, axis=0) / np.linalg.norm(Xd, axis=0)).max() <= 10 * kappa * 1e-12
    # with an in-iteration replacement (the exact zeros of Section 5.1 move through the matrices)
    L = laplacian((10, 11, 12), 0.3)
    B2 = rhs_e1_ae1(L, extra=2)
    a = oracle.solve(L.to_scipy(), B2, tol=1e-10, max_iter=3000)
    b = oracle.solve(L.to_scipy(), B2, tol=1e-10, max_iter=3000, accumulate=True)
    assert a.replaced == b.replaced and a.iters == b.iters
    assert np.abs(a.X - b.X).max() <= 1e-12 * np.abs(a.X).max()
