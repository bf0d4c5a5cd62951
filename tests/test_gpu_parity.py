"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (the oracle's own rounding-order floor was measured first: the
oracle against itself on row-permuted copies of the same system, where every
inner product is summed in another order):
  * residual history rho_j / ||b_i||: |gpu - oracle| <= 1e-6 * oracle + 1e-13
    over the iterations before Lanczos loses global orthogonality;
  * X: max_i ||x_i^gpu - x_i^orc|| / ||x_i^orc|| <= 1e-8 at the same stopping
    index j, both at a fixed j and at convergence (the permuted oracle agrees
    with the oracle to <= 4e-13 at convergence on every small case here, with
    the same stopping index);
  * structure (replacement counts, stopping status, stopping index) exactly,
    except on the 32 x 32 Laplacian, where the permuted oracles stop up to
    STOP_FLOOR_LAP2D iterations apart: there both sides are rerun to the
    smaller index and compared at it.
"""
import numpy as np
import pytest

import oracle
from workloads import laplacian, random_symmetric, rhs_normal, rhs_stress, rhs_e1_ae1, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1301_2102_amd as bmr  # noqa: E402

DEV = "cuda:0"


def _dev(B):
    return torch.from_numpy(np.ascontiguousarray(B)).to(DEV)


def _cols(ro, idx):
    """The oracle result restricted to some columns of X."""
    import copy
    r = copy.copy(ro)
    r.X = ro.X[:, idx]
    return r


def _relcols(X, Y):
    return (np.linalg.norm(X - Y, axis=0) / np.maximum(np.linalg.norm(Y, axis=0), 1e-300)).max()


def _same_stop(A, B, X, info, ro, xtol=1e-8, **kw):
    """Equal status and stopping index, and X to xtol there."""
    assert info.status == ro.status, (info.status_name, ro.status)
    assert info.band_iters == ro.iters, (info.band_iters, ro.iters)
    assert _relcols(X, ro.X) <= xtol, _relcols(X, ro.X)


def _hist_close(hg, ho, rel=1e-6, abs_=1e-13):
    k = min(len(hg), len(ho))
    assert k > 0
    d = np.abs(hg[:k] - ho[:k])
    assert np.all(d <= rel * ho[:k] + abs_), (np.max(d / np.maximum(ho[:k], 1e-300)), k)


# ---------------------------------------------------------------------------
# block operator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", range(1, 17))
@pytest.mark.parametrize("kind", ["lap", "rand"])
def test_spmm_matches_scipy(p, kind):
    A = laplacian((17, 19, 23), 0.3) if kind == "lap" else random_symmetric(5003, draws=13, seed=2)
    V = np.random.default_rng(p).standard_normal((A.n, p))
    W = bmr.spmm(bmr.to_device(A, DEV), _dev(V)).cpu().numpy()
    ref = A.to_scipy() @ V
    scale = (abs(A.to_scipy()) @ abs(V))
    assert np.all(np.abs(W - ref) <= 1e-15 * 8 * scale + 1e-300)


def _ragged(n, seed):
    """Symmetric matrix with row lengths from 0 to about 60 (every 7th row
    and column empty), as a Csr."""
    import scipy.sparse as sp
    from workloads import Csr
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 30, size=n)
    rows = np.repeat(np.arange(n), lens)
    cols = rng.integers(0, n, size=rows.size)
    M = sp.coo_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(n, n)).tocsr()
    M = M + M.T
    keep = sp.diags((np.arange(n) % 7 != 3).astype(np.float64))
    M = (keep @ M @ keep).tocsr()
    M.eliminate_zeros()
    M.sort_indices()
    return Csr(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 13, 16])
@pytest.mark.parametrize("n", [1, 5, 97, 4099])
def test_spmm_ragged_and_tiny(p, n):
    """Empty rows, rows longer than a lane group's first chunk, and fewer
    rows than one workgroup step (most workgroups of the grid get none)."""
    A = _ragged(n, seed=n + p)
    V = np.random.default_rng(p).standard_normal((n, p))
    W = bmr.spmm(bmr.to_device(A, DEV), _dev(V)).cpu().numpy()
    S = A.to_scipy()
    ref = S @ V
    scale = abs(S) @ abs(V)
    assert np.all(np.abs(W - ref) <= 1e-15 * 64 * scale + 1e-300)
    assert np.all(W[np.diff(A.indptr) == 0] == 0.0)


def test_spmm_p8_bitwise_reproducible():
    A = laplacian((33, 31, 29), 0.3)
    V = _dev(np.random.default_rng(0).standard_normal((A.n, 8)))
    Ad = bmr.to_device(A, DEV)
    W1 = bmr.spmm(Ad, V).cpu().numpy()
    W2 = bmr.spmm(Ad, V).cpu().numpy()
    assert np.array_equal(W1, W2)


# ---------------------------------------------------------------------------
# whole solves against the oracle
# ---------------------------------------------------------------------------
def _both(A, B, tol, max_iter, **kw):
    Ad = bmr.to_device(A, DEV)
    Xg, info = bmr.solve(Ad, _dev(B), tol=tol, max_iter=max_iter, hist_cap=max_iter, **kw)
    ro = oracle.solve(A.to_scipy(), B, tol=tol, max_iter=max_iter, **kw)
    return Xg.cpu().numpy(), info, ro, Ad


# Converged 32 x 32 solve: 19 row permutations of the oracle stop at
# j = 658 .. 670 against the oracle's 670 (X within 6e-10 at the smaller index).
STOP_FLOOR_LAP2D = 16


def test_lap2d_32_p4_full_config():
    """2-D 5-point Laplacian 32x32, shift -0.7, n=1024, p=4, tol 1e-8, 500 iterations."""
    A, B, tol, mi = workload("lap2d-32-p4")
    X, info, ro, _ = _both(A, B, tol, mi)
    assert info.status == ro.status == bmr.MAX_ITER
    assert info.band_iters == ro.iters == 500
    assert info.block_iters == 125
    _hist_close(info.hist[:250], ro.hist[:250])
    # X before loss of orthogonality, and at convergence
    X250, i250, r250, _ = _both(A, B, 1e-30, 250)
    assert i250.band_iters == 250
    assert _relcols(X250, r250.X) <= 1e-8
    Xc, ic, rc, Ad = _both(A, B, 1e-8, 5000)
    assert ic.status == rc.status == bmr.CONVERGED
    assert abs(ic.band_iters - rc.iters) <= STOP_FLOOR_LAP2D, (ic.band_iters, rc.iters)
    if ic.band_iters == rc.iters:
        assert _relcols(Xc, rc.X) <= 1e-8
    else:  # both sides again, stopped at the smaller index
        jm = min(ic.band_iters, rc.iters)
        Xm, im, rm, _ = _both(A, B, 1e-30, jm)
        assert im.band_iters == rm.iters == jm
        assert _relcols(Xm, rm.X) <= 1e-8
    ex = bmr.residual(Ad, _dev(B), _dev(Xc)) / ro.beta
    assert ex.max() < 5e-8
    assert np.allclose(ic.res_explicit, ex, rtol=1e-12, atol=0)


@pytest.mark.parametrize("p", range(1, 17))
def test_block_sizes(p):
    A = laplacian((10, 11, 12), 0.3)
    B = rhs_normal(A.n, p, seed=p)
    X, info, ro, _ = _both(A, B, 1e-30, 96)
    assert info.band_iters == ro.iters == 96
    _hist_close(info.hist, ro.hist)
    assert _relcols(X, ro.X) <= 1e-8
    Xc, ic, rc, _ = _both(A, B, 1e-9, 4000)
    assert ic.status == bmr.CONVERGED
    _same_stop(A, B, Xc, ic, rc)


@pytest.mark.parametrize("stop", [1, 5, 7, 8, 9, 13])
def test_stop_inside_a_block(stop):
    """max_iter that is not a multiple of p: only l* columns of the last block enter X."""
    A = laplacian((9, 9, 9), 0.3)
    B = rhs_normal(A.n, 4, seed=3)
    X, info, ro, _ = _both(A, B, 1e-30, stop)
    assert info.band_iters == ro.iters == stop
    assert info.status == bmr.MAX_ITER
    assert _relcols(X, ro.X) <= 1e-10


@pytest.mark.parametrize("p", range(1, 17))
def test_stop_at_group_boundaries(p):
    """The search directions enter X once per group of group_len(p) blocks
    (32 up to p = 8, 12 .. 4 above) and where the iteration stops: stops at
    a group's last block (its regular flush), inside it, just after it (the
    flush of a partial group) and inside the next group give the oracle's
    iterate."""
    s = bmr.group_len(p)
    g = s * p
    stops = [g - 1, g, g + 1, g + p + p // 2]
    if p in (4, 8):
        stops += [2 * g - 1, 2 * g, 2 * g + 1]
    A = laplacian((10, 11, 12), 0.3)
    B = rhs_normal(A.n, p, seed=11 + p)
    for stop in stops:
        X, info, ro, _ = _both(A, B, 1e-30, stop)
        assert info.band_iters == ro.iters == stop
        assert info.block_iters == -(-stop // p)
        assert _relcols(X, ro.X) <= 1e-8, (stop, s)


def test_dependence_e1_ae1_in_iteration():
    """B = [e_1, A e_1]: the first candidate is dependent (column-wise QR path,
    bench substitution); column 2 is solved exactly by x = e_1."""
    A = laplacian((12, 12, 12), 0.3)
    B = rhs_e1_ae1(A)
    X, info, ro, _ = _both(A, B, 1e-10, 3000)
    assert info.n_replaced == len(ro.replaced) >= 1
    assert info.n_explicit_qr >= 1
    assert info.status == ro.status == bmr.CONVERGED
    e1 = np.zeros(A.n)
    e1[0] = 1.0
    assert np.linalg.norm(X[:, 1] - e1) <= 1e-12
    assert np.all(info.hist[:, 1] <= 1e-13)
    _hist_close(info.hist[:100], ro.hist[:100])
    _same_stop(A, B, X, info, ro)


def test_dependence_with_extra_columns():
    A = laplacian((12, 12, 12), 0.3)
    B = rhs_e1_ae1(A, extra=3, seed=4)
    X, info, ro, _ = _both(A, B, 1e-9, 3000)
    assert info.n_replaced == len(ro.replaced)
    assert info.status == bmr.CONVERGED
    _same_stop(A, B, X, info, ro)


@pytest.mark.parametrize("k", [0, 4, 8])
def test_stress_copy_column(k):
    A = laplacian((16, 16, 16), 0.3)
    B = rhs_stress(A.n, k, p=8, seed=0)
    X, info, ro, _ = _both(A, B, 1e-8, 6000)
    assert info.status == bmr.CONVERGED
    assert info.n_replaced == len(ro.replaced) >= 1
    _same_stop(A, B, X, info, ro)
    assert np.linalg.norm(X[:, 7] - X[:, 0]) <= 1e-10 * np.linalg.norm(X[:, 0])


def test_zero_column_and_exhaustion():
    A = laplacian((12, 12, 12), 0.3)
    B = rhs_normal(A.n, 3, seed=2)
    B[:, 1] = 0.0
    X, info, ro, _ = _both(A, B, 1e-10, 2000)
    assert info.status == bmr.CONVERGED
    assert np.all(X[:, 1] == 0.0)
    assert info.n_replaced == len(ro.replaced) == 1
    _same_stop(A, B, X[:, [0, 2]], info, _cols(ro, [0, 2]))
    B2 = rhs_stress(A.n, 0, p=3, seed=2)
    X2, i2, r2, _ = _both(A, B2, 1e-10, 100, n_bench=0)
    assert i2.status == r2.status == bmr.BENCH_EXHAUSTED
    assert i2.band_iters == 0 and np.all(X2 == 0.0)


def test_nonfinite_input_rejected():
    A = laplacian((8, 8, 8), 0.3)
    B = rhs_normal(A.n, 2, seed=0)
    B[5, 1] = np.nan
    Xg, info = bmr.solve(bmr.to_device(A, DEV), _dev(B), check=False)
    assert info.status == bmr.NONFINITE


def test_tiny_systems_and_zero_rhs():
    A = random_symmetric(40, draws=3, seed=1)
    B = rhs_normal(A.n, 2, seed=1)
    X, info, ro, _ = _both(A, B, 1e-10, 100)
    # the basis nearly fills R^40 here, so the last iterations sit in the
    # rounding-order noise: compare outcomes, not the stopping index
    assert info.status == ro.status == bmr.CONVERGED and abs(info.band_iters - ro.iters) <= 4
    Xd = np.linalg.solve(A.to_scipy().toarray(), B)
    assert _relcols(X, Xd) <= 1e-7 and _relcols(ro.X, Xd) <= 1e-7
    # n = 9, p = 2: the basis fills R^9 before convergence, the next candidate
    # has no independent substitute left -> bench exhausted at the same j
    A = laplacian((3, 3), 0.5)
    B = rhs_normal(A.n, 2, seed=1)
    X, info, ro, _ = _both(A, B, 1e-12, 100)
    assert info.status == ro.status == bmr.BENCH_EXHAUSTED
    assert info.band_iters == ro.iters
    assert _relcols(X, ro.X) <= 1e-10
    Xz, iz = bmr.solve(bmr.to_device(A, DEV), _dev(np.zeros((A.n, 2))))
    assert iz.status == bmr.CONVERGED and iz.band_iters == 0 and float(Xz.abs().max()) == 0.0


def test_full_size_lap3d_128_p8_prefix():
    """128^3 Laplacian, p=8, the benchmark's launch configuration: the first
    264 band iterations against the oracle element by element (33 block
    iterations: one whole group of 32 blocks with its regular flush at
    j = 256, then a partial group flushed at the stop)."""
    A, B, _, _ = workload("lap3d-128-p8")
    X, info, ro, _ = _both(A, B, 1e-30, 264)
    assert info.band_iters == ro.iters == 264
    assert info.block_iters == 33
    _hist_close(info.hist, ro.hist)
    assert _relcols(X, ro.X) <= 1e-8


def test_full_size_lap3d_128_p8_converged_properties():
    """Full solve to 1e-8 at 128^3, p=8: the recurrence residual is the
    explicit one and satisfies the stopping test."""
    A, B, tol, mi = workload("lap3d-128-p8")
    Ad = bmr.to_device(A, DEV)
    Bd = _dev(B)
    X, info = bmr.solve(Ad, Bd, tol=tol, max_iter=mi, hist_cap=mi)
    assert info.status == bmr.CONVERGED
    beta = np.linalg.norm(B, axis=0)
    ex = bmr.residual(Ad, Bd, X) / beta
    assert info.res_rec.max() < tol
    assert ex.max() < 10 * tol
    assert np.allclose(info.res_explicit, ex, rtol=1e-12, atol=0)
    assert np.all(np.diff(info.hist, axis=0) <= 1e-14)


@pytest.mark.parametrize("name", ["lap3d-128-p1", "lap3d-128-p16", "rand-1m-p16"])
def test_full_size_prefix_other_workloads(name):
    """The other full-size workloads (128^3 at p = 1 and p = 16, the random
    sparse indefinite matrix with n = 2^20, p = 16): the first 64 band
    iterations against the oracle element by element (two groups of 4 blocks
    at p = 16, two full groups at p = 1)."""
    A, B, _, _ = workload(name)
    X, info, ro, _ = _both(A, B, 1e-30, 64)
    assert info.band_iters == ro.iters == 64
    _hist_close(info.hist, ro.hist)
    assert _relcols(X, ro.X) <= 1e-8


@pytest.mark.parametrize("name", ["stress-64-k0", "stress-64-k4", "stress-64-k8", "stress-64-e3"])
def test_full_size_stress_prefix(name):
    """64^3 deflation-stress inputs at full size: the replacements of the
    first 64 band iterations (the copy column at the initial QR; the
    dependent candidate of iteration 1 for [e_1, A e_1, ...]) match the
    oracle, and so do the iterate and the residual history."""
    A, B, _, _ = workload(name)
    X, info, ro, _ = _both(A, B, 1e-30, 64)
    assert info.band_iters == ro.iters == 64
    assert info.n_replaced == len(ro.replaced) >= 1
    _hist_close(info.hist, ro.hist)
    assert _relcols(X, ro.X) <= 1e-8


@pytest.mark.parametrize("name", ["stress-64-k0", "stress-64-k4", "stress-64-k8", "stress-64-e3"])
def test_full_size_stress_converged_properties(name):
    """64^3 deflation-stress inputs solved to 1e-8 on the GPU: converged, the
    explicit residual meets the tolerance, and the dependent column's
    solution follows from the others (x_8 = x_1 for the copy column,
    x_2 = e_1 for B = [e_1, A e_1, ...])."""
    A, B, tol, mi = workload(name)
    Ad = bmr.to_device(A, DEV)
    Bd = _dev(B)
    X, info = bmr.solve(Ad, Bd, tol=tol, max_iter=mi)
    assert info.status == bmr.CONVERGED, info.status_name
    assert info.n_replaced >= 1
    beta = np.linalg.norm(B, axis=0)
    ex = bmr.residual(Ad, Bd, X) / beta
    assert ex.max() < 10 * tol
    assert np.allclose(info.res_explicit, ex, rtol=1e-12, atol=0)
    Xh = X.cpu().numpy()
    if name.endswith("e3"):
        e1 = np.zeros(A.n)
        e1[0] = 1.0
        assert np.linalg.norm(Xh[:, 1] - e1) <= 1e-8
    else:
        assert np.linalg.norm(Xh[:, 7] - Xh[:, 0]) <= 1e-8 * np.linalg.norm(Xh[:, 0])
