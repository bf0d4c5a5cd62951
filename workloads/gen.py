"""Seeded synthetic inputs: sparse symmetric indefinite matrices and blocks of
right-hand sides, with the shapes and structure of the workloads the solver is
measured on.

Everything is deterministic: matrices depend only on their parameters and
right-hand sides on an explicit ``seed`` fed to ``numpy.random.default_rng``
(PCG64).  The paper's own experiments used Matlab's mt19937ar with seed 0 on a
preconditioned 2-D model problem (Section 8); those streams cannot be
reproduced here, so these generators stand in for them.

No solver arithmetic lives here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Csr:
    """Compressed sparse row matrix, int32 indices, float64 values.

    Column indices are sorted within each row and unique; the matrix is
    structurally and numerically symmetric for every generator below.
    """

    n: int
    indptr: np.ndarray   # (n+1,) int32
    indices: np.ndarray  # (nnz,) int32
    data: np.ndarray     # (nnz,) float64

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))

    def column(self, j: int) -> np.ndarray:
        """Dense column j (equal to row j by symmetry)."""
        out = np.zeros(self.n)
        lo, hi = self.indptr[j], self.indptr[j + 1]
        out[self.indices[lo:hi]] = self.data[lo:hi]
        return out


def laplacian(dims, sigma: float) -> Csr:
    """Dirichlet finite-difference Laplacian on a regular grid, shifted.

    ``dims`` is (nx, ny) for the 5-point or (nx, ny, nz) for the 7-point
    stencil.  Lexicographic ordering with x fastest; diagonal 2d - sigma,
    off-diagonals -1, no wrap-around.  Eigenvalues are
    sum_d (2 - 2 cos(k_d pi / (N_d + 1))) - sigma, so sigma > 0 below the
    largest-but-one level makes the matrix indefinite.
    """
    dims = tuple(int(d) for d in dims)
    if len(dims) not in (2, 3):
        raise ValueError("dims must have 2 or 3 entries")
    if len(dims) == 2:
        dims = dims + (1,)
        ndim = 2
    else:
        ndim = 3
    nx, ny, nz = dims
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    # neighbours in increasing column order: z-1, y-1, x-1, self, x+1, y+1, z+1
    offs = [-nx * ny, -nx, -1, 0, 1, nx, nx * ny]
    valid = [z > 0, y > 0, x > 0, np.ones(n, bool), x < nx - 1, y < ny - 1, z < nz - 1]
    vals = [-1.0, -1.0, -1.0, 2.0 * ndim - sigma, -1.0, -1.0, -1.0]
    if ndim == 2:
        offs, valid, vals = offs[1:6], valid[1:6], vals[1:6]
    cols = np.stack([idx + o for o in offs], axis=1)
    mask = np.stack(valid, axis=1)
    data = np.broadcast_to(np.array(vals), cols.shape)
    counts = mask.sum(axis=1)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return Csr(n, indptr.astype(np.int32), cols[mask].astype(np.int32),
               np.ascontiguousarray(data[mask], dtype=np.float64))


def random_symmetric(n: int, draws: int = 13, seed: int = 0, diag_range: float = 3.0) -> Csr:
    """Random sparse symmetric indefinite matrix.

    For each row, ``draws`` column indices are drawn uniformly from
    [0, n) without the row itself; the pattern is symmetrised and duplicates
    merged, giving about 2*draws+1 entries per row.  One N(0,1)/sqrt(2*draws+1)
    value is drawn per unordered off-diagonal pair; the diagonal is
    U[-diag_range, diag_range].
    """
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), draws)
    cols = rng.integers(0, n - 1, size=rows.size, dtype=np.int64)
    cols += cols >= rows  # skip the diagonal
    lo = np.minimum(rows, cols)
    hi = np.maximum(rows, cols)
    key = np.unique(lo * n + hi)
    lo, hi = key // n, key % n
    off = rng.standard_normal(key.size) / np.sqrt(2 * draws + 1)
    diag = rng.uniform(-diag_range, diag_range, size=n)
    r = np.concatenate([lo, hi, np.arange(n)])
    c = np.concatenate([hi, lo, np.arange(n)])
    v = np.concatenate([off, off, diag])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=indptr[1:])
    return Csr(n, indptr.astype(np.int32), c.astype(np.int32), v.astype(np.float64))


def permuted(A: Csr, perm: np.ndarray) -> Csr:
    """P A P^T for the row order ``perm`` (row i of the result is row perm[i]
    of A), columns sorted: the same operator with the unknowns renumbered."""
    import scipy.sparse as sp
    n = A.n
    P = sp.csr_matrix((np.ones(n), (np.arange(n), np.asarray(perm))), shape=(n, n))
    B = (P @ A.to_scipy() @ P.T).tocsr()
    B.sort_indices()
    return Csr(n, B.indptr.astype(np.int32), B.indices.astype(np.int32), B.data.astype(np.float64))


def redblack_order(dims) -> np.ndarray:
    """Red-black (two-colour) ordering of a regular grid in lexicographic
    x-fastest numbering: every point with an even coordinate sum first, in
    lexicographic order, then the others.  Stencil neighbours have opposite
    colours, so the lower triangle of the reordered Laplacian couples only
    black rows to red ones."""
    dims = tuple(int(d) for d in dims)
    idx = np.indices(dims[::-1]).reshape(len(dims), -1)  # (z, y, x) or (y, x), lexicographic
    parity = idx.sum(axis=0) % 2
    lex = np.arange(int(np.prod(dims)))
    return np.concatenate([lex[parity == 0], lex[parity == 1]])


def rhs_normal(n: int, p: int, seed: int = 0) -> np.ndarray:
    """(n, p) block of independent N(0,1) columns, C-contiguous (row-interleaved)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((p, n)).T)


def rhs_stress(n: int, k: int, p: int = 8, seed: int = 0) -> np.ndarray:
    """Nearly dependent right-hand sides: columns 1..p-1 are b0 + 10^-k r_j with
    b0, r_j ~ N(0,1); the last column is an exact copy of the first."""
    rng = np.random.default_rng(seed)
    b0 = rng.standard_normal(n)
    r = rng.standard_normal((p - 1, n))
    cols = [b0 + 10.0 ** (-k) * r[j] for j in range(p - 1)]
    cols.append(cols[0].copy())
    return np.ascontiguousarray(np.stack(cols, axis=1))


def rhs_e1_ae1(A: Csr, extra: int = 0, seed: int = 0) -> np.ndarray:
    """B = [e_1, A e_1, N(0,1) ...]: the second column is the image of the
    first, so the first band iteration produces a dependent vector (the
    paper's dependence demonstration, Section 8, Fig. 3)."""
    n = A.n
    e1 = np.zeros(n)
    e1[0] = 1.0
    cols = [e1, A.column(0)]
    if extra:
        rng = np.random.default_rng(seed)
        cols += list(rng.standard_normal((extra, n)))
    return np.ascontiguousarray(np.stack(cols, axis=1))


def rhs_near_copy(n: int, p: int = 4, delta: float = 1e-5, seed: int = 3, pert_seed: int = 5) -> np.ndarray:
    """N(0,1) columns with column 2 replaced by column 1 + delta * N(0,1): a
    candidate that is dependent at the initial QR for a dependence tolerance
    above about delta, with a remainder well above rounding."""
    B = rhs_normal(n, p, seed=seed)
    B[:, 1] = B[:, 0] + delta * np.random.default_rng(pert_seed).standard_normal(n)
    return B


def rhs_near_e1_ae1(A: Csr, delta: float = 1e-5, extra: int = 1, seed: int = 5) -> np.ndarray:
    """[e_1, A e_1 + delta ||A e_1|| g / sqrt(n), N(0,1) ...] with g ~ N(0,1):
    the candidate of the first band iteration lies within about delta of the
    basis (near dependence inside the iteration)."""
    n = A.n
    e1 = np.zeros(n)
    e1[0] = 1.0
    Ae1 = A.column(0)
    g = np.random.default_rng(seed).standard_normal(n)
    cols = [e1, Ae1 + delta * np.linalg.norm(Ae1) * g / np.sqrt(n)]
    if extra:
        cols += [rhs_normal(n, 1, seed=9 + q)[:, 0] for q in range(extra)]
    return np.ascontiguousarray(np.stack(cols, axis=1))


def diag_positions(A: Csr) -> np.ndarray:
    """Index into A.data of the diagonal entry of every row (each row must
    store its diagonal)."""
    rows = np.repeat(np.arange(A.n), np.diff(A.indptr))
    pos = np.nonzero(A.indices == rows)[0]
    if pos.size != A.n:
        raise ValueError("every row must store its diagonal")
    return pos


def with_diagonal_shift(A: Csr, d) -> Csr:
    """A + diag(d) on A's pattern (d a scalar or an n-vector)."""
    data = A.data.copy()
    data[diag_positions(A)] += np.broadcast_to(np.asarray(d, dtype=np.float64), (A.n,))
    return Csr(A.n, A.indptr, A.indices, data)


@dataclass(frozen=True)
class ThetaProblem:
    """Parametrised system A(theta, sigma) X = B with loss sum(W * X):
    A(theta, sigma) = L + diag(theta) - sigma I for the unshifted grid
    Laplacian L."""

    L: Csr
    theta: np.ndarray
    sigma: float
    B: np.ndarray
    W: np.ndarray

    def matrix(self, theta=None, sigma=None) -> Csr:
        theta = self.theta if theta is None else theta
        sigma = self.sigma if sigma is None else sigma
        return with_diagonal_shift(self.L, np.asarray(theta) - sigma)


def theta_problem(dims=(96, 96, 96), sigma: float = 0.3, p: int = 8, seed: int = 0,
                  theta_range: float = 0.1) -> ThetaProblem:
    """Differentiable-solve workload: theta ~ U(-theta_range, theta_range),
    B and the loss weights W ~ N(0, 1), n x p."""
    L = laplacian(dims, 0.0)
    rng = np.random.default_rng(seed)
    theta = rng.uniform(-theta_range, theta_range, L.n)
    B = np.ascontiguousarray(rng.standard_normal((p, L.n)).T)
    W = np.ascontiguousarray(rng.standard_normal((p, L.n)).T)
    return ThetaProblem(L, theta, float(sigma), B, W)


# Named workloads: the matrices and right-hand sides the tests and the
# benchmark run.  ``tol``/``max_iter`` are the solve parameters.
WORKLOADS = {
    # 2-D 5-point Laplacian on 32x32, shift -0.7: n=1024, p=4
    "lap2d-32-p4": dict(matrix=("laplacian", (32, 32), 0.7), rhs=("normal", 4), tol=1e-8, max_iter=500),
    # 3-D 7-point Laplacian on 128^3, shift -0.3: n=2,097,152, p=8
    "lap3d-128-p8": dict(matrix=("laplacian", (128, 128, 128), 0.3), rhs=("normal", 8), tol=1e-8, max_iter=400000),
    "lap3d-128-p1": dict(matrix=("laplacian", (128, 128, 128), 0.3), rhs=("normal", 1), tol=1e-8, max_iter=400000),
    "lap3d-128-p16": dict(matrix=("laplacian", (128, 128, 128), 0.3), rhs=("normal", 16), tol=1e-8, max_iter=400000),
    # 3-D Laplacian on 64^3 with nearly dependent columns and an exact copy
    "stress-64-k0": dict(matrix=("laplacian", (64, 64, 64), 0.3), rhs=("stress", 0), tol=1e-8, max_iter=40000),
    "stress-64-k4": dict(matrix=("laplacian", (64, 64, 64), 0.3), rhs=("stress", 4), tol=1e-8, max_iter=40000),
    "stress-64-k8": dict(matrix=("laplacian", (64, 64, 64), 0.3), rhs=("stress", 8), tol=1e-8, max_iter=40000),
    "stress-64-e3": dict(matrix=("laplacian", (64, 64, 64), 0.3), rhs=("e1ae1", 6), tol=1e-8, max_iter=40000),
    # random sparse symmetric indefinite, n = 2^20, ~27 nnz/row, p=16
    "rand-1m-p16": dict(matrix=("random", 1 << 20, 13), rhs=("normal", 16), tol=1e-10, max_iter=40000),
}


def workload(name: str, seed: int = 0):
    """Return (A, B, tol, max_iter) for a named workload."""
    w = WORKLOADS[name]
    kind = w["matrix"][0]
    if kind == "laplacian":
        A = laplacian(w["matrix"][1], w["matrix"][2])
    elif kind == "random":
        A = random_symmetric(w["matrix"][1], w["matrix"][2], seed=seed)
    else:
        raise ValueError(kind)
    rk = w["rhs"]
    if rk[0] == "normal":
        B = rhs_normal(A.n, rk[1], seed=seed)
    elif rk[0] == "stress":
        B = rhs_stress(A.n, rk[1], seed=seed)
    elif rk[0] == "e1ae1":
        B = rhs_e1_ae1(A, extra=rk[1], seed=seed)
    else:
        raise ValueError(rk[0])
    return A, B, w["tol"], w["max_iter"]
