"""GPU tests of the mixed-precision solver: an FP32 block MINRES inner solve
(block operator, Gram products, update pass and n-length data in binary32)
inside binary64 iterative refinement on the explicit residual.

The refinement loop is not in the paper, so there is no oracle trajectory to
follow step by step.  What pins the results:
  * the FP32 block operator against the FP64 product of the same (rounded)
    operands, within the binary32 accumulation bound (m + 1) u |A||V|,
    u = 2^-24, m = entries per row;
  * every converged solve: the explicit residual max_i ||b_i - A x_i|| / ||b_i||,
    recomputed on the CPU in FP64, is below tol; the error against the dense
    direct solve obeys ||x_i - x_i*|| <= ||r_i|| / sigma_min(A) (exact for
    symmetric A), and the error against the FP64 oracle's solution is
    printed and bounded the same way;
  * a single cycle cut after j band iterations is the FP32 run of the same
    method as the oracle's first j iterations: agreement to FP32 level.
"""
import numpy as np
import pytest

import oracle
from workloads import laplacian, random_symmetric, rhs_normal, rhs_stress, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1301_2102_amd as bmr  # noqa: E402

DEV = "cuda:0"
U32 = 2.0 ** -24


def _dev(B, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(B)).to(DEV).to(dtype)


def _colrel(D, Y):
    return np.linalg.norm(D, axis=0) / np.maximum(np.linalg.norm(Y, axis=0), 1e-300)


def _sigma_min(A):
    return np.abs(np.linalg.eigvalsh(A.to_scipy().toarray())).min()


# ---------------------------------------------------------------------------
# FP32 block operator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 2, 3, 8, 13, 16])
@pytest.mark.parametrize("kind", ["lap", "rand"])
def test_spmm_f32_within_binary32_bound(p, kind):
    A = laplacian((17, 19, 23), 0.3) if kind == "lap" else random_symmetric(5003, draws=13, seed=2)
    V = np.random.default_rng(p).standard_normal((A.n, p)).astype(np.float32)
    a32 = A.data.astype(np.float32)
    Ad = bmr.to_device(A, DEV)
    W = bmr.spmm_f32(Ad, torch.from_numpy(a32).to(DEV), _dev(V, torch.float32)).cpu().numpy().astype(np.float64)
    S = A.to_scipy().copy()
    S.data = a32.astype(np.float64)   # the same rounded operands, product in FP64
    ref = S @ V.astype(np.float64)
    m = int(np.diff(A.indptr).max())
    bound = (m + 1) * U32 * (abs(S) @ abs(V.astype(np.float64)))
    assert np.all(np.abs(W - ref) <= bound)


# ---------------------------------------------------------------------------
# converged solves
# ---------------------------------------------------------------------------
def _mixed(A, B, tol, max_iter=200000, **kw):
    Ad = bmr.to_device(A, DEV)
    X, info = bmr.solve(Ad, _dev(B), tol=tol, max_iter=max_iter, precision="mixed", hist_cap=64, **kw)
    return X.cpu().numpy(), info


def _check_converged(A, B, X, info, tol):
    S = A.to_scipy()
    beta = np.linalg.norm(B, axis=0)
    r = np.linalg.norm(B - S @ X, axis=0) / beta
    assert info.status == bmr.CONVERGED, info.status_name
    assert r.max() < tol, r
    # The library's FP64 residual (another summation order) agrees with the
    # CPU's.  Row i of B - A X carries at most (m + 1) u (|A||X| + |B|)_i of
    # rounding on either side (m entries per row), so the two norms differ
    # by at most twice that bound's norm; near convergence this cancellation
    # term dominates the residual's own size.
    m = int(np.diff(A.indptr).max())
    cancel = np.linalg.norm(abs(S) @ abs(X) + abs(B), axis=0)
    bound = 2 * (m + 1) * 2.0**-53 * cancel / beta + 1e-12 * r
    assert np.all(np.abs(info.res_true - r) <= bound), (info.res_true, r, bound)
    return r


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 16])
def test_mixed_lap3d_12_converges_and_error_bounds(p):
    A = laplacian((12, 12, 12), 0.3)
    B = rhs_normal(A.n, p, seed=p)
    tol = 1e-10
    X, info = _mixed(A, B, tol)
    r = _check_converged(A, B, X, info, tol)
    smin = _sigma_min(A)
    beta = np.linalg.norm(B, axis=0)
    Xd = np.linalg.solve(A.to_scipy().toarray(), B)
    err_direct = np.linalg.norm(X - Xd, axis=0)
    assert np.all(err_direct <= 1.01 * r * beta / smin + 1e-13 * np.linalg.norm(Xd, axis=0))
    ro = oracle.solve(A.to_scipy(), B, tol=1e-12, max_iter=20000)
    assert ro.status == oracle.CONVERGED
    err_orc = _colrel(X - ro.X, ro.X)
    print(f"p={p}: cycles={info.n_refine} j={info.band_iters} explicit={r.max():.2e} "
          f"err vs FP64 oracle={err_orc.max():.2e} vs direct={_colrel(X - Xd, Xd).max():.2e}")
    assert np.all(np.linalg.norm(X - ro.X, axis=0) <= 1.01 * (r + 1e-12) * beta / smin * 2)


@pytest.mark.parametrize("p", [1, 4, 16])
def test_mixed_random_indefinite_converges(p):
    A = random_symmetric(2000, draws=13, seed=3)
    B = rhs_normal(A.n, p, seed=10 + p)
    X, info = _mixed(A, B, 1e-10)
    r = _check_converged(A, B, X, info, 1e-10)
    Xd = np.linalg.solve(A.to_scipy().toarray(), B)
    beta = np.linalg.norm(B, axis=0)
    assert np.all(np.linalg.norm(X - Xd, axis=0) <= 1.01 * r * beta / _sigma_min(A) + 1e-12)


def test_mixed_cycle_history():
    """tol far below inner_tol forces several cycles; each recorded cycle
    halves the worst explicit residual at least (else STAGNATED)."""
    A = laplacian((12, 12, 12), 0.3)
    B = rhs_normal(A.n, 4, seed=7)
    X, info = _mixed(A, B, 1e-12, inner_tol=1e-3)
    _check_converged(A, B, X, info, 1e-12)
    h = info.hist
    assert info.n_refine >= 3 and h.shape == (info.n_refine, 4)
    worst = h.max(axis=1)
    assert np.all(worst[1:] <= 0.5 * worst[:-1])
    assert np.allclose(h[-1], info.res_true)


def test_mixed_single_cycle_prefix_matches_oracle():
    """One refinement cycle cut after 40 band iterations is the FP32 run of the
    oracle's first 40 iterations (X_0 = 0, R = B)."""
    A = laplacian((16, 16, 16), 0.3)
    B = rhs_normal(A.n, 4, seed=3)
    j = 40
    X, info = _mixed(A, B, 1e-10, max_iter=j, max_refine=1)
    assert info.n_refine == 1 and info.band_iters == j
    ro = oracle.solve(A.to_scipy(), B, tol=1e-10, max_iter=j)
    err = _colrel(X - ro.X, ro.X).max()
    print(f"FP32 prefix of {j} iterations: max column error vs oracle {err:.2e}")
    assert err < 1e-4


def test_mixed_copy_column_stress():
    """Exact copy column (the deflation stress right-hand side): the inner
    solves take the dependent column from the bench and the refinement still
    converges; the two solution columns agree within the residual bound."""
    A = laplacian((12, 12, 12), 0.3)
    B = rhs_stress(A.n, 0, p=8, seed=0)
    tol = 1e-10
    X, info = _mixed(A, B, tol)
    r = _check_converged(A, B, X, info, tol)
    assert info.n_replaced >= 1
    beta = np.linalg.norm(B, axis=0)
    d = np.linalg.norm(X[:, 7] - X[:, 0])
    assert d <= 1.01 * (r[0] + r[7]) * beta[0] / _sigma_min(A)


def test_mixed_bitwise_reproducible():
    A = laplacian((14, 13, 12), 0.3)
    B = rhs_normal(A.n, 8, seed=1)
    X1, i1 = _mixed(A, B, 1e-10)
    X2, i2 = _mixed(A, B, 1e-10)
    assert np.array_equal(X1, X2) and i1.band_iters == i2.band_iters


def test_mixed_nonfinite_rejected():
    A = laplacian((8, 8, 8), 0.3)
    B = rhs_normal(A.n, 2, seed=0)
    B[5, 1] = np.nan
    with pytest.raises(bmr.BmrError) as e:
        _mixed(A, B, 1e-8)
    assert e.value.status == bmr.NONFINITE


# ---------------------------------------------------------------------------
# full size
# ---------------------------------------------------------------------------
def test_full_size_lap3d_128_p8_mixed():
    """128^3 Laplacian, p = 8, to 1e-8 on the explicit FP64 residual."""
    A, B, tol, mi = workload("lap3d-128-p8")
    Ad = bmr.to_device(A, DEV)
    Bd = _dev(B)
    X, info = bmr.solve(Ad, Bd, tol=tol, max_iter=mi, precision="mixed")
    assert info.status == bmr.CONVERGED, info.status_name
    norms = bmr.residual(Ad, Bd, X)
    rel = norms / np.linalg.norm(B, axis=0)
    assert rel.max() < tol and np.allclose(rel, info.res_true, rtol=1e-6)
    # sampled rows of the residual, recomputed on the CPU
    S = A.to_scipy()
    rows = np.random.default_rng(0).choice(A.n, 4096, replace=False)
    Xh = X.cpu().numpy()
    Rg = bmr.residual(Ad, Bd, X, want_R=True)[1].cpu().numpy()
    assert np.allclose(Rg[rows], B[rows] - S[rows] @ Xh, rtol=0, atol=1e-12 * np.abs(B).max())
    print(f"128^3 p=8 mixed: {info.n_refine} cycles, {info.band_iters} band iterations, "
          f"{info.time_ms/1e3:.2f} s, explicit {rel.max():.2e}")
