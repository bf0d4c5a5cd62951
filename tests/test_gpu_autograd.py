"""GPU tests of the differentiable solve (adjoint block MINRES) and of the
pattern-gradient kernel, against the oracle's adjoint gradients (themselves
pinned by finite differences of dense solves) and against central finite
differences of GPU solves.

Finite differences of solves: the two perturbed solves run the same number of
band iterations (the base solve's count, tol set below reach), so the
difference quotient differentiates one smooth Krylov approximation; it then
agrees with the converged adjoint gradient to the solves' accuracy.
"""
import numpy as np
import pytest

import oracle
from workloads import laplacian, random_symmetric, theta_problem, diag_positions

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1301_2102_amd as bmr  # noqa: E402
from paper_1301_2102_amd.autograd import solve_diff  # noqa: E402

DEV = "cuda:0"


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("p", [1, 3, 8, 16])
@pytest.mark.parametrize("kind", ["lap", "rand"])
def test_pattern_grad_kernel_matches_oracle(p, kind):
    A = laplacian((11, 13, 9), 0.3) if kind == "lap" else random_symmetric(3001, draws=13, seed=5)
    rng = np.random.default_rng(p)
    Lam, X = rng.standard_normal((A.n, p)), rng.standard_normal((A.n, p))
    g = bmr.pattern_grad(bmr.to_device(A, DEV), _dev(Lam), _dev(X)).cpu().numpy()
    ref = oracle.pattern_grad(A.indptr, A.indices, Lam, X)
    assert np.allclose(g, ref, rtol=1e-13, atol=1e-13 * p)


class _Model:
    """val(theta, sigma) = L.val + scatter(theta - sigma) on the diagonal."""

    def __init__(self, t):
        self.t = t
        self.A = bmr.to_device(t.L, DEV)
        self.base = self.A.val.clone()
        self.diag = torch.from_numpy(diag_positions(t.L)).to(DEV)

    def val(self, theta, sigma):
        return self.base.index_add(0, self.diag, theta - sigma)

    def loss(self, theta, sigma, B, W, **kw):
        X = solve_diff(self.A, B, val=self.val(theta, sigma), **kw)
        return (W * X).sum()


def _grads(m, tol=1e-12, max_iter=200000):
    t = m.t
    theta = _dev(t.theta).requires_grad_()
    sigma = torch.tensor(t.sigma, dtype=torch.float64, device=DEV, requires_grad=True)
    B = _dev(t.B).requires_grad_()
    L = m.loss(theta, sigma, B, _dev(t.W), tol=tol, max_iter=max_iter)
    L.backward()
    return float(L), theta.grad.cpu().numpy(), float(sigma.grad), B.grad.cpu().numpy()


@pytest.mark.parametrize("p", [1, 8])
def test_autograd_matches_oracle_gradient(p):
    t = theta_problem((12, 12, 12), sigma=0.3, p=p, seed=2)
    _, dth, dsg, dB = _grads(_Model(t))
    g = oracle.loss_grad(t.matrix().to_scipy(), t.B, t.W, tol=1e-12, max_iter=50000)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)  # noqa: E731
    print(f"p={p}: theta {rel(dth, g.dtheta):.1e} sigma {abs(dsg - g.dsigma) / abs(g.dsigma):.1e} "
          f"B {rel(dB, g.dB):.1e}")
    assert rel(dth, g.dtheta) < 1e-7 and abs(dsg - g.dsigma) < 1e-7 * abs(g.dsigma) and rel(dB, g.dB) < 1e-7


def _fd_check(t, tol, h=1e-6, n_dir=2, rtol=1e-5, h_sigma=None, rtol_sigma=None):
    m = _Model(t)
    L0, dth, dsg, dB = _grads(m, tol=tol, max_iter=1_000_000)
    Bd, Wd = _dev(t.B), _dev(t.W)
    th = _dev(t.theta)
    sg = torch.tensor(t.sigma, dtype=torch.float64, device=DEV)

    def at(theta, sigma):
        return bmr.DeviceCsr(m.A.n, m.A.row_ptr, m.A.col_idx, m.val(theta, sigma).contiguous())

    # the base forward solve's iteration count (on A(theta, sigma)) fixes the
    # perturbed solves' count
    _, info = bmr.solve(at(th, sg), Bd, tol=tol, max_iter=1_000_000)
    assert info.status == bmr.CONVERGED
    j = info.band_iters

    def loss_fixed(theta, sigma, B):
        X, inf = bmr.solve(at(theta, sigma), B, tol=1e-300, max_iter=j)
        assert inf.band_iters == j
        return float((Wd * X).sum())

    rng = np.random.default_rng(11)
    for _ in range(n_dir):
        d = _dev(rng.standard_normal(t.L.n))
        fd = (loss_fixed(th + h * d, sg, Bd) - loss_fixed(th - h * d, sg, Bd)) / (2 * h)
        an = float(np.dot(dth, d.cpu().numpy()))
        print(f"theta direction: fd {fd:.8e} adjoint {an:.8e} rel {abs(fd - an) / abs(an):.1e}")
        assert abs(fd - an) <= rtol * abs(an), (fd, an)
    hs = h if h_sigma is None else h_sigma
    fd = (loss_fixed(th, sg + hs, Bd) - loss_fixed(th, sg - hs, Bd)) / (2 * hs)
    print(f"sigma: fd {fd:.8e} adjoint {dsg:.8e} rel {abs(fd - dsg) / abs(dsg):.1e}")
    assert abs(fd - dsg) <= (rtol if rtol_sigma is None else rtol_sigma) * abs(dsg), (fd, dsg)
    D = _dev(rng.standard_normal(t.B.shape))
    fd = (loss_fixed(th, sg, Bd + h * D) - loss_fixed(th, sg, Bd - h * D)) / (2 * h)
    an = float(np.sum(dB * D.cpu().numpy()))
    print(f"B direction: fd {fd:.8e} adjoint {an:.8e} rel {abs(fd - an) / abs(an):.1e}")
    assert abs(fd - an) <= rtol * abs(an), (fd, an)
    return j


def test_autograd_finite_differences_small():
    _fd_check(theta_problem((14, 12, 10), sigma=0.3, p=4, seed=3), tol=1e-11)


def test_unconverged_forward_raises():
    t = theta_problem((10, 10, 10), sigma=0.3, p=2, seed=0)
    m = _Model(t)
    theta = _dev(t.theta).requires_grad_()
    sigma = torch.tensor(t.sigma, dtype=torch.float64, device=DEV)
    with pytest.raises(bmr.BmrError):
        m.loss(theta, sigma, _dev(t.B), _dev(t.W), tol=1e-12, max_iter=10)


def test_full_size_theta_problem_96_finite_differences():
    """A(theta, sigma) = 96^3 Laplacian + diag(theta) - 0.3 I, p = 8, forward
    and adjoint to 1e-10; gradients in theta (random directions) and B
    against central differences (h = 1e-6) of GPU solves.

    This A has an eigenvalue about 2e-6 from zero (dL/dsigma is ~8e10): a
    shift of sigma by 1e-6 moves it by half its size, so the central
    difference in sigma carries a truncation error of order (h / lambda)^2
    (18% measured at h = 1e-6).  sigma is checked with h = 1e-8 instead.
    Tolerance: a difference quotient of solves and the adjoint gradient each
    carry the solves' relative error, up to kappa * tol ~ 6e6 * 1e-10 here,
    so 1e-3 (measured: 1e-7 to 2e-5)."""
    j = _fd_check(theta_problem((96, 96, 96), sigma=0.3, p=8, seed=0), tol=1e-10, n_dir=1, rtol=1e-3,
                  h_sigma=1e-8)
    print(f"96^3 p=8: {j} band iterations per solve")
