"""GPU parity of the IC(0)-preconditioned solve against the oracle
(``oracle.precond``): the level-scheduled factorisation and triangular
solves, and whole split-preconditioned solves, through the C ABI.

Tolerances follow the unpreconditioned parity tests: the triangular solves
to 1e-12 relative (a handful of rounding steps per level), X to 1e-8 at the
same stopping index, the first 50 preconditioned residual norms to 1e-6
relative.  The absolute floor is 1e-12 instead of 1e-13: the preconditioned
recurrence falls below 1e-12 within 40 iterations on the small cases, and
there the two sides differ by the rounding of the triangular solves (4e-13
measured where the oracle's value is 1.6e-13)."""
import numpy as np
import pytest

import oracle
import oracle.precond as opc
from workloads import laplacian, random_symmetric, rhs_normal

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


def _diag_dominant(n, seed):
    import scipy.sparse as sp
    from workloads import Csr
    A = random_symmetric(n, draws=4, seed=seed).to_scipy().tolil()
    A.setdiag(0.0)
    A = sp.csr_matrix(A)
    A.data = -np.abs(A.data)
    d = np.asarray(abs(A).sum(axis=1)).ravel() + 0.5
    M = sp.csr_matrix(A + sp.diags(d))
    M.sort_indices()
    return Csr(M.shape[0], M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


@pytest.mark.parametrize("which", ["lap2d-32", "lap3d-24", "rand"])
@pytest.mark.parametrize("p", [1, 3, 8, 16])
def test_ic0_triangular_solves_match_oracle(which, p):
    if which == "lap2d-32":
        M = laplacian((32, 32), 0.0)
    elif which == "lap3d-24":
        M = laplacian((24, 23, 22), 0.0)
    else:
        M = _diag_dominant(4001, 7)
    C = opc.ichol0(M.to_scipy())
    ic = bmr.ic0_factor(bmr.to_device(M, DEV))
    V = np.random.default_rng(p).standard_normal((M.n, p))
    Vd = _dev(V)
    W1 = bmr.ic0_apply(ic, Vd).cpu().numpy()
    W2 = bmr.ic0_apply(ic, Vd, trans=True).cpu().numpy()
    assert _relcols(W1, opc.apply_cinv(C, V)) <= 1e-12
    assert _relcols(W2, opc.apply_cinvt(C, V)) <= 1e-12
    # in place
    Vi = _dev(V)
    bmr.ic0_apply(ic, Vi, W=Vi)
    assert np.array_equal(Vi.cpu().numpy(), W1)


def test_ic0_breakdown_reported():
    M = laplacian((6, 6), 7.0)  # indefinite: IC(0) has a negative pivot
    with pytest.raises(bmr.BmrError) as e:
        bmr.ic0_factor(bmr.to_device(M, DEV))
    assert e.value.status == bmr.IC0_BREAKDOWN


def _both(A, M, B, tol, max_iter, **kw):
    Ad = bmr.to_device(A, DEV)
    ic = bmr.ic0_factor(bmr.to_device(M, DEV))
    Xg, info = bmr.solve(Ad, _dev(B), tol=tol, max_iter=max_iter, hist_cap=max_iter, ic0=ic, **kw)
    ro = opc.solve(A.to_scipy(), M.to_scipy(), B, tol=tol, max_iter=max_iter, **kw)
    return Xg.cpu().numpy(), info, ro, Ad


def _hist_close(hg, ho, rel=1e-6, abs_=1e-12):
    k = min(len(hg), len(ho), 50)
    assert k > 0
    d = np.abs(hg[:k] - ho[:k])
    assert np.all(d <= rel * ho[:k] + abs_), (np.max(d / np.maximum(ho[:k], 1e-300)), k)


def test_precond_lap2d_32_p4_converged():
    """32 x 32 Laplacian shifted by -0.7 (indefinite), p = 4, IC(0) of the
    unshifted Laplacian, solved to 1e-8: the oracle's stopping index, X and
    residual history."""
    A = laplacian((32, 32), 0.7)
    M = laplacian((32, 32), 0.0)
    B = rhs_normal(A.n, 4, seed=0)
    X, info, ro, Ad = _both(A, M, B, 1e-8, 2000)
    assert info.status == ro.status == bmr.CONVERGED
    assert info.band_iters == ro.iters, (info.band_iters, ro.iters)
    assert _relcols(X, ro.X) <= 1e-8
    _hist_close(info.hist, ro.hist)
    # res_explicit is the unpreconditioned relative residual of the result
    ex = bmr.residual(Ad, _dev(B), _dev(X)) / np.linalg.norm(B, axis=0)
    assert np.allclose(info.res_explicit, ex, rtol=1e-10, atol=0)
    assert info.res_rec.max() < 1e-8


@pytest.mark.parametrize("p", [1, 2, 5, 8, 16])
def test_precond_block_sizes(p):
    A = laplacian((10, 11, 12), 0.3)
    M = laplacian((10, 11, 12), 0.0)
    B = rhs_normal(A.n, p, seed=20 + p)
    X, info, ro, _ = _both(A, M, B, 1e-30, 64)
    assert info.band_iters == ro.iters == 64
    _hist_close(info.hist, ro.hist)
    assert _relcols(X, ro.X) <= 1e-8
    Xc, ic, rc, _ = _both(A, M, B, 1e-9, 3000)
    assert ic.status == rc.status == bmr.CONVERGED
    assert ic.band_iters == rc.iters
    assert _relcols(Xc, rc.X) <= 1e-8


def test_precond_lap3d_64_p8_prefix():
    """64^3 Laplacian shifted by -0.3, p = 8, IC(0) of the unshifted
    Laplacian: the first 128 band iterations (16 block iterations) element by
    element against the oracle."""
    A = laplacian((64, 64, 64), 0.3)
    M = laplacian((64, 64, 64), 0.0)
    B = rhs_normal(A.n, 8, seed=0)
    X, info, ro, _ = _both(A, M, B, 1e-30, 128)
    assert info.band_iters == ro.iters == 128
    _hist_close(info.hist, ro.hist)
    assert _relcols(X, ro.X) <= 1e-8


def test_precond_lap3d_64_p8_converged():
    """The same 64^3 system solved to 1e-8 on the GPU: converged in fewer
    iterations than without the preconditioner, preconditioned recurrence
    below the tolerance, explicit residual consistent with it."""
    A = laplacian((64, 64, 64), 0.3)
    M = laplacian((64, 64, 64), 0.0)
    B = rhs_normal(A.n, 8, seed=0)
    Ad = bmr.to_device(A, DEV)
    ic = bmr.ic0_factor(bmr.to_device(M, DEV))
    Bd = _dev(B)
    X, info = bmr.solve(Ad, Bd, tol=1e-8, max_iter=40000, ic0=ic, hist_cap=40000)
    assert info.status == bmr.CONVERGED
    assert info.res_rec.max() < 1e-8
    assert np.all(np.diff(info.hist, axis=0) <= 1e-14)
    ex = bmr.residual(Ad, Bd, X) / np.linalg.norm(B, axis=0)
    assert np.allclose(info.res_explicit, ex, rtol=1e-10, atol=0)
    # the recurrence is the explicit preconditioned residual ||C^{-1}(b - A x)|| / ||C^{-1} b||
    # (C from the oracle), up to the rounding left after the stop
    C = opc.ichol0(M.to_scipy())
    Xh = X.cpu().numpy()
    pre = (np.linalg.norm(opc.apply_cinv(C, B - A.to_scipy() @ Xh), axis=0)
           / np.linalg.norm(opc.apply_cinv(C, B), axis=0))
    assert pre.max() < 1.5e-8, pre
    _, plain = bmr.solve(Ad, Bd, tol=1e-8, max_iter=400000)
    assert plain.status == bmr.CONVERGED and info.band_iters < plain.band_iters


@pytest.mark.parametrize("dims,sigma,p", [((32, 32), 0.7, 4), ((64, 64, 64), 0.3, 8)])
def test_precond_redblack_ordering(dims, sigma, p):
    """The same systems with the unknowns in red-black order (every stencil
    neighbour of a red point is black): IC(0) of the reordered Laplacian has
    two levels, so each triangular solve is two launches.  Against the
    oracle on the same reordered matrices: a 64-iteration prefix, and the
    converged 32 x 32 solve."""
    from workloads import permuted, redblack_order
    perm = redblack_order(dims)
    A = permuted(laplacian(dims, sigma), perm)
    M = permuted(laplacian(dims, 0.0), perm)
    B = rhs_normal(A.n, p, seed=1)
    X, info, ro, _ = _both(A, M, B, 1e-30, 64)
    assert info.band_iters == ro.iters == 64
    _hist_close(info.hist, ro.hist)
    assert _relcols(X, ro.X) <= 1e-8
    if len(dims) == 2:
        # the stop sits in the rounding floor here: the oracle on B perturbed
        # in its last bit stops anywhere in 328 .. 333 (331 unperturbed), with
        # X within 4.2e-10 at the smaller index; so both sides are compared at
        # the smaller stopping index
        Xc, ic, rc, _ = _both(A, M, B, 1e-8, 3000)
        assert ic.status == rc.status == bmr.CONVERGED
        assert abs(ic.band_iters - rc.iters) <= 8, (ic.band_iters, rc.iters)
        jm = min(ic.band_iters, rc.iters)
        Xm, im, rm, _ = _both(A, M, B, 1e-30, jm)
        assert im.band_iters == rm.iters == jm
        assert _relcols(Xm, rm.X) <= 1e-8
