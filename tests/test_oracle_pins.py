"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each one checks it
against an independent construction (a dense direct solve, the least-squares
definition over a brute-force basis, classical MINRES, the displayed
structure of Section 5.1, the C_{pxp} layout of Section 7, the dependence
demonstration of Section 8, closed-form invariances).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import oracle
from oracle.rng import bench_vector, splitmix64
from workloads import laplacian, random_symmetric, rhs_normal, rhs_e1_ae1, rhs_stress

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _lap(dims, sigma):
    return laplacian(dims, sigma).to_scipy()


# --------------------------------------------------------------------------
# Whole solve: dense direct solve (LAPACK) on tiny systems
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_converges_to_direct_solution(p):
    A = _lap((8, 8), 0.7)
    B = rhs_normal(A.shape[0], p, seed=11)
    r = oracle.solve(A, B, tol=1e-12, max_iter=1000)
    assert r.status == oracle.CONVERGED
    Xd = np.linalg.solve(A.toarray(), B)
    kappa = np.linalg.cond(A.toarray())
    err = np.linalg.norm(r.X - Xd, axis=0) / np.linalg.norm(Xd, axis=0)
    assert err.max() <= 10 * kappa * 1e-12, (err, kappa)
    # the explicit residual satisfies the stopping test (Algorithm 7.1 output)
    res = np.linalg.norm(B - A @ r.X, axis=0) / np.linalg.norm(B, axis=0)
    assert res.max() < 1e-11


# --------------------------------------------------------------------------
# Iterates: the plain least-squares definition over a brute-force basis
# --------------------------------------------------------------------------
def _band_basis_bruteforce(A, B, J):
    """span{u_1..u_{J+p}} built with full re-orthogonalisation (twice against
    every earlier vector) in the band order of eq. (2.4): u_1..u_p from the
    columns of B, then u_{j+p} from A u_j."""
    A = np.asarray(A.toarray() if sp.issparse(A) else A)
    n, p = B.shape
    U = []
    for v in list(B.T) + [None] * J:
        if v is None:
            v = A @ U[len(U) - p]
        w = v.copy()
        for _ in range(2):
            for q in U:
                w -= (q @ w) * q
        U.append(w / np.linalg.norm(w))
    return np.column_stack(U)


@pytest.mark.parametrize("p,seed", [(1, 3), (2, 4), (3, 5)])
def test_iterates_match_least_squares_definition(p, seed):
    A = random_symmetric(80, draws=4, seed=seed).to_scipy()
    B = rhs_normal(80, p, seed=seed)
    J = 24
    r = oracle.solve(A, B, tol=1e-30, max_iter=J, record=True)
    assert r.iters == J
    U = _band_basis_bruteforce(A, B, J)
    Ad = A.toarray()
    for j in range(1, J + 1):
        Uj = U[:, :j]
        AU = Ad @ Uj
        for i in range(p):
            y = np.linalg.lstsq(AU, B[:, i], rcond=None)[0]
            x = Uj @ y
            xo = r.Xs[j - 1][:, i]
            assert np.linalg.norm(xo - x) <= 1e-8 * max(np.linalg.norm(x), 1e-300), (j, i)
            rho = np.linalg.norm(B[:, i] - Ad @ x) / np.linalg.norm(B[:, i])
            assert abs(r.hist[j - 1, i] - rho) <= 1e-9 * max(rho, 1e-6), (j, i)


def test_block_krylov_at_multiples_of_p():
    """At j = kp the band space is the k-th block Krylov space (eq. (2.5)):
    span{B, AB, ..., A^{k-1}B}, so X_{kp} is the block-GMRES iterate."""
    A = _lap((6, 6), 0.5)
    Ad = A.toarray()
    p = 3
    B = rhs_normal(36, p, seed=7)
    for k in (1, 2, 3):
        r = oracle.solve(A, B, tol=1e-30, max_iter=k * p)
        K = np.column_stack([np.linalg.matrix_power(Ad, e) @ B for e in range(k)])
        Q, _ = np.linalg.qr(K)
        for i in range(p):
            y = np.linalg.lstsq(Ad @ Q, B[:, i], rcond=None)[0]
            assert np.allclose(r.X[:, i], Q @ y, rtol=0, atol=1e-9 * np.linalg.norm(Q @ y))


# --------------------------------------------------------------------------
# p = 1 reduces to MINRES (Paige-Saunders)
# --------------------------------------------------------------------------
def _minres_by_definition(A, b, J):
    """MINRES iterates by their definition: symmetric Lanczos on b, then
    x_k = V_k argmin ||beta e_1 - T-bar_k y|| for every k <= J."""
    n = b.size
    V = np.zeros((n, J + 1))
    T = np.zeros((J + 1, J))
    beta = np.linalg.norm(b)
    V[:, 0] = b / beta
    xs = []
    for k in range(J):
        w = A @ V[:, k]
        if k:
            w -= T[k - 1, k] * V[:, k - 1]
        T[k, k] = V[:, k] @ w
        w -= T[k, k] * V[:, k]
        T[k + 1, k] = np.linalg.norm(w)
        if k + 1 < J:
            T[k, k + 1] = T[k + 1, k]
        V[:, k + 1] = w / T[k + 1, k]
        e1 = np.zeros(k + 2)
        e1[0] = beta
        y = np.linalg.lstsq(T[:k + 2, :k + 1], e1, rcond=None)[0]
        xs.append(V[:, :k + 1] @ y)
    return xs


def test_p1_matches_textbook_and_scipy_minres():
    A = _lap((16, 16), 0.7)
    b = rhs_normal(256, 1, seed=2)[:, 0]
    J = 60
    r = oracle.solve(A, b[:, None], tol=1e-30, max_iter=J, record=True)
    xs_def = _minres_by_definition(A, b, J)
    xs_sp = []
    sla.minres(A, b, rtol=1e-30, maxiter=J, callback=lambda x: xs_sp.append(x.copy()))
    nb = np.linalg.norm(b)
    for j in range(1, J + 1):
        ro = np.linalg.norm(b - A @ r.Xs[j - 1][:, 0]) / nb
        rd = np.linalg.norm(b - A @ xs_def[j - 1]) / nb
        rs = np.linalg.norm(b - A @ xs_sp[j - 1]) / nb
        assert abs(ro - rd) <= 1e-10 * rd, j
        assert abs(ro - rs) <= 1e-10 * rs, j
        # the recurrence residual is the explicit one (eq. (3.5))
        assert abs(r.hist[j - 1, 0] - ro) <= 1e-10 * ro, j


# --------------------------------------------------------------------------
# Basis: band Arnoldi relation, symmetry and bandwidth, orthogonality
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 2, 4])
def test_band_arnoldi_relation(p):
    A = _lap((10, 10), 0.7)
    B = rhs_normal(100, p, seed=21)
    J = 40
    r = oracle.solve(A, B, tol=1e-30, max_iter=J, record=True)
    U, H = r.U, r.H
    assert U.shape == (100, J + p) and H.shape == (J + p, J)
    nA = np.linalg.norm(A.toarray(), 2)
    # A U_j = U_{j+p} H-bar_j (eq. (2.2))
    assert np.linalg.norm(A @ U[:, :J] - U @ H) <= 1e-13 * nA * np.sqrt(J)
    # H_j = U_j^T A U_j is symmetric (eq. (2.3)) with bandwidth p
    Hj = H[:J, :J]
    assert np.array_equal(Hj, Hj.T)
    i, k = np.nonzero(H)
    assert np.all(np.abs(i - k) <= p)
    # the lowest p x p block C_j is upper triangular (Section 2)
    C = H[J:, J - p:]
    assert np.all(np.tril(C, -1) == 0)
    # local orthogonality over the 2p window; global while j is small
    G = U.T @ U
    for a in range(J + p):
        for b in range(max(0, a - 2 * p), a + 1):
            assert abs(G[a, b] - (a == b)) <= 1e-12
    assert np.abs(G[:16, :16] - np.eye(16)).max() <= 1e-12
    assert np.abs(G[:30, :30] - np.eye(30)).max() <= 1e-9


# --------------------------------------------------------------------------
# Residual recurrence
# --------------------------------------------------------------------------
def test_residual_recurrence_and_monotonicity():
    A = _lap((12, 12), 0.6)
    p = 3
    B = rhs_normal(144, p, seed=5)
    r = oracle.solve(A, B, tol=1e-30, max_iter=120, record=True)
    h = r.hist
    # nested spaces give nonincreasing minimal residuals (eq. (2.4))
    assert np.all(np.diff(h, axis=0) <= 1e-14)
    # recurrence residual equals the explicit one (eq. (3.5))
    for j in range(1, 121):
        ex = np.linalg.norm(B - A @ r.Xs[j - 1], axis=0) / r.beta
        mask = ex >= 1e-9
        assert np.all(np.abs(h[j - 1][mask] - ex[mask]) <= 1e-10), j


def test_at_least_as_good_as_single_rhs_minres():
    """Column i of the block iterate is no worse than J_i(j) steps of MINRES on
    b_i alone (Section 6).  The count of vectors of K(A, b_i) among u_1..u_j
    is J_i(j) = floor((j - i)/p) + 1; the paper's J is one higher (its
    subspace index counts the p starting vectors twice)."""
    A = _lap((12, 12), 0.6)
    p = 3
    B = rhs_normal(144, p, seed=9)
    J = 60
    r = oracle.solve(A, B, tol=1e-30, max_iter=J)
    for i in range(1, p + 1):
        b = B[:, i - 1]
        xs = _minres_by_definition(A, b, J)
        for j in range(1, J + 1):
            Ji = (j - i) // p + 1
            if Ji < 1:
                continue
            rm = np.linalg.norm(b - A @ xs[Ji - 1]) / np.linalg.norm(b)
            assert r.hist[j - 1, i - 1] <= rm * (1 + 1e-8), (i, j)


# --------------------------------------------------------------------------
# Invariances that follow from the subspace definition
# --------------------------------------------------------------------------
def test_block_and_scaling_invariance():
    A = _lap((7, 7), 0.4)
    p = 3
    B = rhs_normal(49, p, seed=31)
    k = 4
    X = oracle.solve(A, B, tol=1e-30, max_iter=k * p).X
    G = np.array([[2.0, -1.0, 0.5], [0.3, 1.5, -0.7], [-0.2, 0.4, 1.1]])
    XG = oracle.solve(A, B @ G, tol=1e-30, max_iter=k * p).X
    assert np.allclose(XG, X @ G, atol=1e-10 * np.abs(X).max())
    Pm = np.eye(p)[:, [2, 0, 1]]
    XP = oracle.solve(A, B @ Pm, tol=1e-30, max_iter=k * p).X
    assert np.allclose(XP, X @ Pm, atol=1e-10 * np.abs(X).max())
    j = 11  # any j, not only multiples of p
    Xj = oracle.solve(A, B, tol=1e-30, max_iter=j).X
    assert np.allclose(oracle.solve(A, 3.0 * B, tol=1e-30, max_iter=j).X, 3.0 * Xj,
                       atol=1e-12 * np.abs(Xj).max())
    assert np.allclose(oracle.solve(4.0 * A, B, tol=1e-30, max_iter=j).X, Xj / 4.0,
                       atol=1e-12 * np.abs(Xj).max())
    # the dependence test is relative to ||A u_j||, so a tiny scale of A
    # neither triggers replacements nor changes the iterate beyond 1/alpha
    rs = oracle.solve(1e-12 * A, B, tol=1e-30, max_iter=j)
    assert rs.replaced == []
    assert np.allclose(rs.X * 1e-12, Xj, atol=1e-12 * np.abs(Xj).max())


# --------------------------------------------------------------------------
# Dependence: Section 5.1 worked example, Section 8 demonstration, copies
# --------------------------------------------------------------------------
def _read_pattern(path):
    mats = {}
    cur = None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] in ("H", "R"):
            cur = tok[0]
            mats[cur] = []
            continue
        mats[cur].append(tok)
    return {k: np.array(v) for k, v in mats.items()}


def _grade3_rhs(n=40, seed=0):
    """A symmetric A and B = [b1, b2] with b1 inside a 3-dimensional invariant
    subspace: K(A, b1) has grade 3, so with p = 2 the candidate A u_5 (u_5 is
    the A^2 b1 direction) is dependent at band iteration j = 5."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(-2.0, 5.0, n)
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    b1 = Q[:, [3, 17, 30]] @ np.array([1.0, -0.7, 0.4])
    b2 = rng.standard_normal(n)
    return A, np.column_stack([b1, b2])


def test_replacement_structure_matches_section_5_1():
    A, B = _grade3_rhs()
    r = oracle.solve(A, B, tol=1e-30, max_iter=10, record=True)
    assert r.replaced == [7]  # u_7 replaced, i.e. h_{7,5} := 0 at j = 5
    pat = _read_pattern(os.path.join(GOLD, "replacement_structure_p2.txt"))
    H, R = r.H, r.R
    assert H.shape == pat["H"].shape and R.shape == pat["R"].shape
    for M, P in ((H, pat["H"]), (R, pat["R"])):
        assert np.all(M[P == "."] == 0.0)
        assert np.all(M[P == "0"] == 0.0)  # exact zeros, also in floating point
        assert np.all(np.abs(M[P == "x"]) > 1e-12)


def test_c_queue_antidiagonal_section_7():
    A = _lap((6, 6), 0.5)
    p = 5
    B = rhs_normal(36, p, seed=3)
    r = oracle.solve(A, B, tol=1e-30, max_iter=7, record=True)
    H = r.H
    C = np.zeros((p, p))
    for line in open(os.path.join(GOLD, "cqueue_p5_j7.txt")):
        if line.startswith("#") or not line.strip():
            continue
        rr, cc, row, col = map(int, line.split())
        C[rr - 1, cc - 1] = H[row - 1, col - 1]
    # C holds the subdiagonal entries of the p latest columns (2..6) ...
    for c in range(p):
        col = 2 + c
        assert np.array_equal(C[:, c], H[col:col + p, col - 1])
    # ... and its antidiagonal is the superdiagonal part of column 7
    anti = np.array([C[p - 1 - c, c] for c in range(p)])
    assert np.array_equal(anti, H[1:6, 6])
    assert np.all(anti != 0)


def test_dependence_demonstration_e1_ae1():
    """B = [e_1, A e_1] (Section 8, Fig. 3): the first candidate is dependent,
    column 2 converges at once with x_2 = e_1, column 1 continues."""
    Acsr = laplacian((10, 10), 0.7)
    A = Acsr.to_scipy()
    B = rhs_e1_ae1(Acsr)
    r = oracle.solve(A, B, tol=1e-10, max_iter=400, record=True)
    assert r.replaced[0] == 3  # u_{1+p} with p = 2
    assert r.H[2, 0] == 0.0
    assert np.all(r.hist[:, 1] <= 1e-14)
    e1 = np.zeros(100)
    e1[0] = 1.0
    assert np.linalg.norm(r.Xs[0][:, 1] - e1) <= 1e-14
    assert np.linalg.norm(r.X[:, 1] - e1) <= 1e-13
    assert r.status == oracle.CONVERGED
    Xd = np.linalg.solve(A.toarray(), B)
    assert np.linalg.norm(r.X[:, 0] - Xd[:, 0]) <= 1e-6 * np.linalg.norm(Xd[:, 0])


def test_exact_zeros_after_in_iteration_replacement():
    """After a replacement at iteration j: h_{j+p,j} = h_{j,j+p} = 0,
    r_{j-p,j+p} = 0 and r_{j,j+2p} = 0 (Section 5.1), here with p = 2, j = 5."""
    A, B = _grade3_rhs(seed=4)
    r = oracle.solve(A, B, tol=1e-30, max_iter=12, record=True)
    j, p = 5, 2
    assert r.H[j + p - 1, j - 1] == 0.0 and r.H[j - 1, j + p - 1] == 0.0
    assert r.R[j - p - 1, j + p - 1] == 0.0 and r.R[j - 1, j + 2 * p - 1] == 0.0


def test_copy_column_replaced_at_initial_qr():
    A = _lap((6, 6, 6), 0.3)
    B = rhs_stress(216, k=0, p=4, seed=1)
    r = oracle.solve(A, B, tol=1e-10, max_iter=2000)
    assert r.replaced[0] == 4 and r.S[3, 3] == 0.0
    assert r.status == oracle.CONVERGED
    assert np.linalg.norm(r.X[:, 3] - r.X[:, 0]) <= 1e-10 * np.linalg.norm(r.X[:, 0])


def test_zero_column_and_bench_exhaustion():
    A = random_symmetric(60, draws=4, seed=1).to_scipy()
    B = rhs_normal(60, 3, seed=2)
    B[:, 1] = 0.0
    r = oracle.solve(A, B, tol=1e-10, max_iter=500)
    # a zero column is dependent at the initial QR (S(2,2) = 0), keeps x = 0
    # and does not hold up the stopping test
    assert r.replaced == [2] and r.S[1, 1] == 0.0
    assert r.status == oracle.CONVERGED and np.all(r.X[:, 1] == 0.0)
    assert np.all(r.hist[:, 1] == 0.0)
    A = _lap((5, 5), 0.3)
    # a duplicate column with an empty bench stops at the initial QR
    B2 = rhs_stress(25, k=0, p=3, seed=2)
    r2 = oracle.solve(A, B2, tol=1e-10, max_iter=200, n_bench=0)
    assert r2.status == oracle.BENCH_EXHAUSTED and r2.iters == 0


def test_bench_vectors_stay_orthogonal_to_basis():
    """Section 5.1: a substitute must be orthogonal to every Lanczos vector so
    far; with B = [e_1, A e_1] the substitute at j = 1 joins a basis whose
    first vectors it must be orthogonal to."""
    A = _lap((8, 8), 0.5)
    Acsr = laplacian((8, 8), 0.5)
    B = rhs_e1_ae1(Acsr)
    r = oracle.solve(A, B, tol=1e-30, max_iter=6, record=True)
    U = r.U
    assert np.abs(U.T @ U - np.eye(U.shape[1])).max() <= 1e-12


# --------------------------------------------------------------------------
# Substitute generator: SplitMix64 known answers
# --------------------------------------------------------------------------
def test_splitmix64_known_answers():
    for line in open(os.path.join(GOLD, "splitmix64_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        seed, c, out = (int(t) for t in line.split())
        assert int(splitmix64(seed, np.array([c]))[0]) == out


def test_bench_vector_mapping():
    n = 1000
    v = bench_vector(n, 1, 7)
    bits = splitmix64(7, np.arange(n, 2 * n)) >> np.uint64(11)
    assert np.array_equal(v, bits.astype(np.float64) / 2.0 ** 52 - 1.0)
    assert v.min() >= -1.0 and v.max() < 1.0
    assert abs(v.mean()) < 0.1
