"""GPU tests of the relaxed-precision solver (BMR_PREC_RELAXED): one run of
block MINRES in binary64 until every recurrence residual is below
relax_tol (default 1e3 tol), then with binary32 Lanczos blocks and
arithmetic on the same band state, the search directions and X kept in
binary64.

Not in the paper, so the binary32 part has no oracle trajectory.  What pins
the results:
  * up to the switch the run is the FP64 solver, bitwise: its residual
    history rows equal those of the FP64 solve (which the parity tests
    compare with the oracle), and a switch level that is never reached gives
    the FP64 X bitwise;
  * every converged solve: the explicit residual, recomputed on the CPU in
    FP64, is within a small factor of tol (the recurrence is what stops, as
    for FP64; relaxation bounds the gap), and X is within
    (||r_i|| + ||r_i^64||) / sigma_min(A) of the FP64 solve's X (each lies
    within ||r|| / sigma_min of the exact solution, A symmetric; sigma_min
    from the stencil's closed-form eigenvalues);
  * the iteration count after the switch stays close to the FP64 count.
"""
import numpy as np
import pytest

from workloads import laplacian, rhs_normal, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1301_2102_amd as bmr  # noqa: E402

DEV = "cuda:0"


def _dev(B):
    return torch.from_numpy(np.ascontiguousarray(B)).to(DEV)


def _explicit(A, B, X):
    return (np.linalg.norm(B - A.to_scipy() @ X, axis=0) / np.linalg.norm(B, axis=0)).max()


def _sigma_min(dims, shift):
    """Smallest |eigenvalue| of the shifted Dirichlet Laplacian: the
    eigenvalues are sum_d (2 - 2 cos(k_d pi / (N_d + 1))) - shift."""
    lam = [2 - 2 * np.cos(np.arange(1, m + 1) * np.pi / (m + 1)) for m in dims]
    return np.abs(lam[0][:, None, None] + lam[1][None, :, None] + lam[2][None, None, :] - shift).min()


# systems on which the switch (at the end of a group of blocks after the
# residual first falls below 1e-5) comes well before convergence, from the
# oracle's iteration counts: e.g. 24^3, p = 8 needs 152 blocks to 1e-10 and
# crosses 1e-5 at block 112 (groups of 32 blocks)
CASES = [((24, 25, 26), 1), ((24, 25, 26), 2), ((20, 21, 22), 3), ((24, 25, 26), 5), ((24, 24, 24), 8),
         ((24, 24, 24), 12), ((24, 25, 26), 16)]


@pytest.mark.parametrize("dims,p", CASES)
def test_switch_then_converge(dims, p):
    """Each layout class of the block size (one lane per row, 4-, 8- and
    16-lane groups, paired rows): the FP64 prefix is bitwise the FP64 solve,
    the binary32 part converges with the explicit residual at tol."""
    A = laplacian(dims, 0.3)
    B = rhs_normal(A.n, p, seed=p)
    Ad, Bd = bmr.to_device(A, DEV), _dev(B)
    tol, cap = 1e-10, 40000
    X64, i64 = bmr.solve(Ad, Bd, tol=tol, max_iter=cap, hist_cap=cap, poll_every=4)
    X, info = bmr.solve(Ad, Bd, tol=tol, max_iter=cap, hist_cap=cap, poll_every=4, precision="relaxed",
                        relax_tol=1e-5)
    assert i64.status == 0 and info.status == 0, (i64.status_name, info.status_name)
    s = info.switch_iter
    assert 0 < s < info.band_iters, (s, info.band_iters)
    assert (s // p) % bmr.group_len(p) == 0 and s % p == 0
    assert np.array_equal(info.hist[:s], i64.hist[:s])
    assert info.band_iters <= 1.25 * i64.band_iters + 8 * p, (info.band_iters, i64.band_iters)
    Xh, X64h = X.cpu().numpy(), X64.cpu().numpy()
    S = A.to_scipy()
    r = np.linalg.norm(B - S @ Xh, axis=0)
    r64 = np.linalg.norm(B - S @ X64h, axis=0)
    beta = np.linalg.norm(B, axis=0)
    assert (r / beta).max() < 3 * tol, (r / beta).max()
    assert np.allclose(info.res_explicit, r / beta, rtol=1e-6, atol=1e-16)
    # both are within ||r|| / sigma_min of the exact solution
    err = np.linalg.norm(Xh - X64h, axis=0)
    assert np.all(err <= 1.01 * (r + r64) / _sigma_min(dims, 0.3)), (err, r, r64)


def test_unreached_switch_is_the_fp64_solve():
    """A switch level just above tol is never seen at a poll before the stop:
    the result is the FP64 solve's, bitwise."""
    A = laplacian((10, 11, 12), 0.3)
    B = rhs_normal(A.n, 4, seed=3)
    Ad, Bd = bmr.to_device(A, DEV), _dev(B)
    X64, i64 = bmr.solve(Ad, Bd, tol=1e-8, max_iter=5000)
    X, info = bmr.solve(Ad, Bd, tol=1e-8, max_iter=5000, precision="relaxed", relax_tol=1.000001e-8)
    assert info.switch_iter == 0
    assert info.band_iters == i64.band_iters
    assert torch.equal(X, X64)
    assert np.array_equal(info.res_explicit, i64.res_explicit)


def test_switch_with_accumulated_rotations_and_group_ends():
    """The switch lands on the end of a group of blocks whatever the poll
    batch; accumulated rotations carry across it.  32^3, p = 8 needs 288
    blocks to 1e-10 and crosses 1e-5 near block 219."""
    A = laplacian((32, 32, 32), 0.3)
    B = rhs_normal(A.n, 8, seed=0)
    Ad, Bd = bmr.to_device(A, DEV), _dev(B)
    grp = bmr.group_len(8)
    for poll in (1, 3, 8):
        X, info = bmr.solve(Ad, Bd, tol=1e-10, max_iter=40000, precision="relaxed", relax_tol=1e-5,
                            poll_every=poll, accumulate=True)
        assert info.status == 0, info.status_name
        assert info.switch_iter > 0 and (info.switch_iter // 8) % grp == 0, (poll, info.switch_iter)
        assert _explicit(A, B, X.cpu().numpy()) < 3e-10


def test_full_size_relaxed_to_1e10():
    """128^3, p = 8 to 1e-10: converged, explicit residual at tol (the CPU
    recomputes it on 4096 sampled rows and from the library's residual)."""
    A, B, _, mi = workload("lap3d-128-p8")
    Ad, Bd = bmr.to_device(A, DEV), _dev(B)
    X, info = bmr.solve(Ad, Bd, tol=1e-10, max_iter=400000, precision="relaxed")
    assert info.status == 0, info.status_name
    assert info.switch_iter > 0
    assert info.res_explicit.max() < 2e-10, info.res_explicit
    rows = np.random.default_rng(0).choice(A.n, 4096, replace=False)
    S = A.to_scipy()[rows]
    Xh = X.cpu().numpy()
    r_rows = B[rows] - S @ Xh
    R = (Bd - bmr.spmm(Ad, X)).cpu().numpy()
    assert np.allclose(R[rows], r_rows, rtol=0, atol=1e-12 * np.abs(B).max())
    assert (np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)).max() < 2e-10


def test_relaxed_without_bench_with_profile_and_short_history():
    """n_bench = 0 (no substitute vectors to round), the per-kernel timing
    flag (one block iteration in flight at a time, so the switch may come a
    group later) and a history shorter than the run: both converge with the
    explicit residual at tol, and their FP64 part is the same iteration."""
    A = laplacian((24, 24, 24), 0.3)
    B = rhs_normal(A.n, 8, seed=8)
    Ad, Bd = bmr.to_device(A, DEV), _dev(B)
    kw = dict(tol=1e-10, max_iter=40000, poll_every=4, precision="relaxed", relax_tol=1e-5, n_bench=0)
    X, info = bmr.solve(Ad, Bd, hist_cap=40000, **kw)
    Xp, infop = bmr.solve(Ad, Bd, hist_cap=100, profile=True, **kw)
    assert info.status == 0 and infop.status == 0
    assert info.switch_iter > 0 and infop.switch_iter > 0
    assert infop.hist.shape == (100, 8)
    assert np.array_equal(infop.hist, info.hist[:100])
    assert infop.kernel_ms["n_block_iters"] > 0
    for Y in (X, Xp):
        assert _explicit(A, B, Y.cpu().numpy()) < 3e-10
