"""GPU parity of the two variant modes against the oracle's, through the C
ABI: retained candidates (BMR_FLAG_RETAIN; Section 5.1, last paragraph;
reading R13) and accumulated block rotations (BMR_FLAG_ACCUMULATE;
Section 4's remark; reading R14).

Near-dependent inputs with the dependence tolerance 1e-3: the removed
candidate's remainder is about 1e-5 of its reference norm, so its direction
is known to about 1e-11 on both sides, and the usual bar applies: the same
stopping index and retained count, X to 1e-8, the first 50 residual norms to
1e-6 relative (+1e-13)."""
import numpy as np
import pytest

import oracle
from workloads import laplacian, rhs_e1_ae1, rhs_near_copy, rhs_near_e1_ae1, rhs_normal, rhs_stress, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1301_2102_amd as bmr  # noqa: E402

DEV = "cuda:0"


def _dev(B):
    return torch.from_numpy(np.ascontiguousarray(B)).to(DEV)


def _relcols(X, Y):
    return (np.linalg.norm(X - Y, axis=0) / np.maximum(np.linalg.norm(Y, axis=0), 1e-300)).max()


def _hist_close(hg, ho, rel=1e-6, abs_=1e-13):
    k = min(len(hg), len(ho), 50)
    d = np.abs(hg[:k] - ho[:k])
    assert np.all(d <= rel * ho[:k] + abs_), (np.max(d / np.maximum(ho[:k], 1e-300)), k)


def _both(A, B, tol, max_iter, **kw):
    Ad = bmr.to_device(A, DEV)
    Xg, info = bmr.solve(Ad, _dev(B), tol=tol, max_iter=max_iter, hist_cap=max_iter, retain=True, **kw)
    ro = oracle.solve(A.to_scipy(), B, tol=tol, max_iter=max_iter, retain=True, **kw)
    return Xg.cpu().numpy(), info, ro


def test_default_gamma_keeps_nothing_and_changes_nothing():
    """Copy column (exactly dependent): nothing is retained and the flag
    changes no bit of the result."""
    A = laplacian((16, 16, 16), 0.3)
    B = rhs_stress(A.n, 0, p=8, seed=0)
    Ad = bmr.to_device(A, DEV)
    X1, i1 = bmr.solve(Ad, _dev(B), tol=1e-8, max_iter=6000)
    X2, i2 = bmr.solve(Ad, _dev(B), tol=1e-8, max_iter=6000, retain=True)
    assert i1.n_replaced == i2.n_replaced >= 1 and i2.n_retained == 0
    assert i1.band_iters == i2.band_iters
    assert torch.equal(X1, X2)


@pytest.mark.parametrize("case", ["initial", "iteration"])
def test_retained_candidate_matches_oracle(case):
    A = laplacian((10, 11, 12), 0.3)
    B = rhs_near_copy(A.n, p=4) if case == "initial" else rhs_near_e1_ae1(A)
    p = B.shape[1]
    # a prefix spanning the retained vector's window and beyond
    X, info, ro = _both(A, B, 1e-30, 6 * p, gamma=1e-3)
    assert info.band_iters == ro.iters == 6 * p
    assert info.n_replaced == len(ro.replaced) == 1
    assert info.n_retained == len(ro.retained) == 1
    assert info.n_explicit_qr >= 2  # the blocks inside the window went column by column
    _hist_close(info.hist, ro.hist)
    assert _relcols(X, ro.X) <= 1e-8
    # converged: the oracle on row-permuted copies of these systems stops up
    # to two iterations apart (306 .. 308 for the in-iteration case) with X
    # within 6e-10, so both sides are compared at the smaller stopping index
    Xc, ic, rc = _both(A, B, 1e-10, 3000, gamma=1e-3)
    assert ic.status == rc.status == bmr.CONVERGED
    assert abs(ic.band_iters - rc.iters) <= 4, (ic.band_iters, rc.iters)
    jm = min(ic.band_iters, rc.iters)
    Xm, im, rm = _both(A, B, 1e-30, jm, gamma=1e-3)
    assert im.band_iters == rm.iters == jm
    assert im.n_retained == len(rm.retained) == 1
    assert _relcols(Xm, rm.X) <= 1e-8


# --------------------------------------------------------------------------
# Accumulated rotations (BMR_FLAG_ACCUMULATE; Section 4's remark; reading R14)
# --------------------------------------------------------------------------
def _both_acc(A, B, tol, max_iter):
    Ad = bmr.to_device(A, DEV)
    Xg, info = bmr.solve(Ad, _dev(B), tol=tol, max_iter=max_iter, hist_cap=max_iter, accumulate=True)
    ro = oracle.solve(A.to_scipy(), B, tol=tol, max_iter=max_iter, accumulate=True)
    return Xg.cpu().numpy(), info, ro, Ad


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 12, 16])
def test_accumulated_rotations_match_oracle(p):
    A = laplacian((10, 11, 12), 0.3)
    B = rhs_normal(A.n, p, seed=30 + p)
    X, info, ro, Ad = _both_acc(A, B, 1e-30, 96)
    assert info.band_iters == ro.iters == 96
    _hist_close(info.hist, ro.hist)
    assert _relcols(X, ro.X) <= 1e-8
    Xc, ic, rc, _ = _both_acc(A, B, 1e-9, 4000)
    assert ic.status == rc.status == bmr.CONVERGED
    assert ic.band_iters == rc.iters
    assert _relcols(Xc, rc.X) <= 1e-8
    # and the sequential GPU solve stops at the same index with the same X to rounding
    Xs, info_s = bmr.solve(Ad, _dev(B), tol=1e-9, max_iter=4000)
    assert info_s.band_iters == ic.band_iters
    assert _relcols(Xc, Xs.cpu().numpy()) <= 1e-10


def test_accumulated_rotations_through_replacement():
    A = laplacian((12, 12, 12), 0.3)
    B = rhs_e1_ae1(A, extra=2, seed=1)
    X, info, ro, _ = _both_acc(A, B, 1e-10, 3000)
    assert info.n_replaced == len(ro.replaced) >= 1 and info.n_explicit_qr >= 1
    assert info.status == ro.status == bmr.CONVERGED
    assert info.band_iters == ro.iters
    assert _relcols(X, ro.X) <= 1e-8


def test_full_size_accumulated_prefix():
    """128^3 p = 8, the benchmark's launch configuration, 264 band iterations
    (one whole group of 32 blocks and a partial one) with accumulated
    rotations against the oracle's."""
    A, B, _, _ = workload("lap3d-128-p8")
    X, info, ro, _ = _both_acc(A, B, 1e-30, 264)
    assert info.band_iters == ro.iters == 264
    _hist_close(info.hist, ro.hist)
    assert _relcols(X, ro.X) <= 1e-8
