"""The allocation-free explicit residual (bmr_residual_noalloc, partial sums
in the library's static device scratch) against bmr_residual (partial sums in
a caller workspace), called through the C ABI: two calls in a row, the second
with a smaller system and block, each compared element by element."""
import ctypes

import numpy as np
import pytest

from workloads import laplacian, random_symmetric

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1301_2102_amd as bmr  # noqa: E402

DEV = "cuda:0"


def _lib():
    lib = bmr.load()
    f = lib.bmr_residual_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(bmr._Csr), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    return lib


def _case(lib, A, p, seed):
    rng = np.random.default_rng(seed)
    Ad = bmr.to_device(A, DEV)
    B = torch.from_numpy(rng.standard_normal((A.n, p))).to(DEV)
    X = torch.from_numpy(rng.standard_normal((A.n, p))).to(DEV)
    # the existing entry point, with a workspace
    n_ref, R_ref = bmr.residual(Ad, B, X, want_R=True)
    # the allocation-free one: caller passes only inputs and outputs
    R = torch.full_like(B, np.nan)
    norms = (ctypes.c_double * p)()
    Ac = Ad._c()
    stream = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    st = lib.bmr_residual_noalloc(ctypes.byref(Ac), B.data_ptr(), X.data_ptr(), p, R.data_ptr(), norms, stream)
    assert st == bmr.CONVERGED, bmr.status_string(st)
    torch.cuda.synchronize()
    got = np.array(norms[:p])
    # same kernels, same workgroup count, same summation order
    assert np.array_equal(R.cpu().numpy(), R_ref.cpu().numpy())
    assert np.array_equal(got, n_ref)
    # and against a CPU evaluation of the definition
    Rc = B.cpu().numpy() - A.to_scipy() @ X.cpu().numpy()
    assert np.allclose(got, np.linalg.norm(Rc, axis=0), rtol=1e-12, atol=0)
    # norms only (R = NULL)
    norms2 = (ctypes.c_double * p)()
    st = lib.bmr_residual_noalloc(ctypes.byref(Ac), B.data_ptr(), X.data_ptr(), p, None, norms2, stream)
    assert st == bmr.CONVERGED
    assert np.array_equal(np.array(norms2[:p]), n_ref)


def test_noalloc_residual_matches_workspace_entry_point():
    lib = _lib()
    _case(lib, laplacian((64, 64, 64), 0.3), 16, seed=1)      # 2048 workgroups' worth of rows
    _case(lib, random_symmetric(3001, draws=5, seed=3), 3, seed=2)  # smaller n and p second


def test_noalloc_residual_rejects_bad_arguments():
    lib = _lib()
    A = laplacian((8, 8), 0.1)
    Ad = bmr.to_device(A, DEV)
    B = torch.zeros((A.n, 2), dtype=torch.float64, device=DEV)
    norms = (ctypes.c_double * 16)()
    Ac = Ad._c()
    assert lib.bmr_residual_noalloc(ctypes.byref(Ac), B.data_ptr(), B.data_ptr(), 17, None, norms, None) == \
        bmr.INVALID_ARG
    assert lib.bmr_residual_noalloc(ctypes.byref(Ac), None, B.data_ptr(), 2, None, norms, None) == bmr.INVALID_ARG
