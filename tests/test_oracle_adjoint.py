"""Pins of the oracle's adjoint gradients: central finite differences of dense
direct solves (numpy.linalg.solve, i.e. LAPACK), on small systems, so that a
dropped factor 1/2, a sign, a transposed product or a wrong row/column pairing
in the pattern gradient fails."""
import numpy as np
import pytest

import oracle
from workloads import laplacian, random_symmetric, theta_problem, diag_positions


def _loss_dense(Ad, B, W):
    return float(np.sum(W * np.linalg.solve(Ad, B)))


def _dense(A):
    return A.to_scipy().toarray()


@pytest.mark.parametrize("p", [1, 3])
def test_theta_sigma_and_B_gradients_match_central_differences(p):
    t = theta_problem((5, 4, 3), sigma=0.3, p=p, seed=4)
    A = t.matrix()
    g = oracle.loss_grad(A.to_scipy(), t.B, t.W, tol=1e-13, max_iter=5000)
    h = 1e-6
    rng = np.random.default_rng(0)
    # theta: along random directions and single coordinates
    for _ in range(3):
        d = rng.standard_normal(A.n)
        fp = _loss_dense(_dense(t.matrix(theta=t.theta + h * d)), t.B, t.W)
        fm = _loss_dense(_dense(t.matrix(theta=t.theta - h * d)), t.B, t.W)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g.dtheta @ d) <= 1e-6 * abs(fd) + 1e-9
    for i in (0, 17, A.n - 1):
        d = np.zeros(A.n)
        d[i] = 1.0
        fd = (_loss_dense(_dense(t.matrix(theta=t.theta + h * d)), t.B, t.W)
              - _loss_dense(_dense(t.matrix(theta=t.theta - h * d)), t.B, t.W)) / (2 * h)
        assert abs(fd - g.dtheta[i]) <= 1e-6 * abs(fd) + 1e-9
    # sigma
    fd = (_loss_dense(_dense(t.matrix(sigma=t.sigma + h)), t.B, t.W)
          - _loss_dense(_dense(t.matrix(sigma=t.sigma - h)), t.B, t.W)) / (2 * h)
    assert abs(fd - g.dsigma) <= 1e-6 * abs(fd) + 1e-9
    # B
    Ad = _dense(A)
    D = rng.standard_normal(t.B.shape)
    fd = (_loss_dense(Ad, t.B + h * D, t.W) - _loss_dense(Ad, t.B - h * D, t.W)) / (2 * h)
    assert abs(fd - np.sum(g.dB * D)) <= 1e-6 * abs(fd) + 1e-9


def test_pattern_gradient_symmetric_perturbation():
    """Along a symmetric perturbation E on the pattern, dL = sum_e g_e E_e."""
    A = random_symmetric(70, draws=4, seed=1)
    rng = np.random.default_rng(2)
    B = rng.standard_normal((A.n, 2))
    W = rng.standard_normal((A.n, 2))
    g = oracle.loss_grad(A.to_scipy(), B, W, tol=1e-13, max_iter=5000)
    # symmetric E: one value per unordered pair, copied to both stored entries
    rows = np.repeat(np.arange(A.n), np.diff(A.indptr))
    cols = A.indices
    key = np.minimum(rows, cols) * A.n + np.maximum(rows, cols)
    vals = {k: v for k, v in zip(np.unique(key), rng.standard_normal(len(np.unique(key))))}
    E = np.array([vals[k] for k in key])
    import scipy.sparse as sp
    Es = sp.csr_matrix((E, cols, A.indptr), shape=(A.n, A.n)).toarray()
    assert np.allclose(Es, Es.T)
    h = 1e-6
    Ad = _dense(A)
    fd = (_loss_dense(Ad + h * Es, B, W) - _loss_dense(Ad - h * Es, B, W)) / (2 * h)
    assert abs(fd - g.dA @ E) <= 1e-6 * abs(fd) + 1e-9
    # diagonal entries of the pattern gradient are the theta gradient
    assert np.allclose(g.dA[diag_positions(A)], g.dtheta)


def test_pattern_grad_small_explicit():
    """Two-by-two pattern, values worked out by hand."""
    indptr = np.array([0, 2, 4])
    indices = np.array([0, 1, 0, 1])
    Lam = np.array([[1.0, 2.0], [3.0, 4.0]])
    X = np.array([[5.0, 6.0], [7.0, 8.0]])
    g = oracle.pattern_grad(indptr, indices, Lam, X)
    # (0,0): -(1*5+2*6); (0,1): -((1*7+2*8) + (3*5+4*6))/2; (1,1): -(3*7+4*8)
    assert np.allclose(g, [-17.0, -31.0, -31.0, -53.0])
