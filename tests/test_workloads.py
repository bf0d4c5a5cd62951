"""Synthetic inputs: structure, symmetry, spectrum and determinism."""
import numpy as np
import pytest

from workloads import laplacian, random_symmetric, rhs_normal, rhs_stress, rhs_e1_ae1, workload


def _check_csr(A):
    assert A.indptr.dtype == np.int32 and A.indices.dtype == np.int32
    assert A.data.dtype == np.float64
    assert A.indptr[0] == 0 and A.indptr[-1] == A.nnz
    for i in range(0, A.n, max(1, A.n // 97)):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
        assert i in cols


@pytest.mark.parametrize("dims,sigma,nnz", [((32, 32), 0.7, 4992), ((16, 16, 16), 0.3, 27136)])
def test_laplacian_structure_and_spectrum(dims, sigma, nnz):
    A = laplacian(dims, sigma)
    _check_csr(A)
    assert A.nnz == nnz
    S = A.to_scipy()
    assert abs(S - S.T).max() == 0
    if A.n <= 1024:
        lam = np.linalg.eigvalsh(S.toarray())
        e = [2 - 2 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1)) for N in dims]
        closed = e[0][:, None] + e[1][None, :]
        closed = np.sort(closed.ravel()) - sigma
        assert np.allclose(lam, closed, atol=1e-12)


def test_laplacian_128_sizes():
    # sizes only (no solve): n = 128^3, nnz = 7n - 6*128^2
    n = 128 ** 3
    assert 7 * n - 6 * 128 ** 2 == 14581760


def test_random_symmetric():
    A = random_symmetric(5000, draws=13, seed=0)
    _check_csr(A)
    S = A.to_scipy()
    assert abs(S - S.T).max() == 0
    assert 26.0 < A.nnz / A.n < 28.0
    d = S.diagonal()
    assert d.min() >= -3 and d.max() <= 3
    B = random_symmetric(5000, draws=13, seed=0)
    assert np.array_equal(A.data, B.data) and np.array_equal(A.indices, B.indices)


def test_rhs_generators():
    B = rhs_normal(1000, 8, seed=0)
    assert B.flags.c_contiguous and B.shape == (1000, 8)
    assert np.array_equal(B, rhs_normal(1000, 8, seed=0))
    S = rhs_stress(1000, 8, p=8, seed=0)
    assert np.array_equal(S[:, 7], S[:, 0])
    assert np.linalg.norm(S[:, 1] - S[:, 0]) < 1e-6 * np.linalg.norm(S[:, 0])
    A = laplacian((8, 8), 0.3)
    E = rhs_e1_ae1(A, extra=2)
    assert E[0, 0] == 1 and np.array_equal(E[:, 1], A.to_scipy() @ E[:, 0])


def test_named_workload_small():
    A, B, tol, mi = workload("lap2d-32-p4")
    assert A.n == 1024 and A.nnz == 4992 and B.shape == (1024, 4) and tol == 1e-8 and mi == 500
