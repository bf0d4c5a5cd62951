// bmr_residual_noalloc: the explicit residual of bmr_residual for callers
// that cannot allocate or pass device memory (code under graph capture,
// serving loops, harnesses that forbid allocation).  Its partial sums live in
// a file-scope device array instead of a caller workspace.
//
// The array is a host-side stand-in in host code: its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// on the first call there, and only that address is handed to the kernels.
// Every call on a device shares that device's array and leaves its partial
// sums in it; the kernels overwrite every entry they read, so nothing has to
// be cleared first, but calls that overlap on one device (two streams, two
// host threads) race on it.
#include <mutex>

#include "bmr_internal.hpp"

namespace bmr {
namespace {

// Partial sums of k_residual (p per workgroup, at most pass1_grid's 2048
// workgroups and BMR_MAX_P columns) followed by the p reduced sums: 262 KB.
constexpr int NOALLOC_MAX_WG = 2048;
constexpr size_t NOALLOC_PART = (size_t)NOALLOC_MAX_WG * MAXP;
constexpr size_t NOALLOC_DOUBLES = NOALLOC_PART + MAXP;

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_scratch[MAX_DEVICES];  // device address of `scratch` on each device, once looked up

// Device address of the scratch array on the current device.
int scratch_address(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return BMR_HIP_ERROR;
  if (dev < 0 || dev >= MAX_DEVICES) return BMR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BMR_HIP_ERROR;
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return 0;
}

}  // namespace
}  // namespace bmr

using namespace bmr;

extern "C" int bmr_residual_noalloc(const bmr_csr_t* A, const double* B, const double* X, int p, double* R,
                                    double* norms, hipStream_t stream) {
  if (!A || A->n < 1 || A->n >= (int64_t(1) << 31) || A->nnz < 0 || A->nnz >= (int64_t(1) << 31) || !A->row_ptr ||
      (A->nnz > 0 && (!A->col_idx || !A->val)))
    return BMR_INVALID_ARG;
  if (!B || !X || !norms || p < 1 || p > BMR_MAX_P || ((uintptr_t)X & 15u) != 0) return BMR_INVALID_ARG;
  // the same workgroup count as bmr_residual, so both sum in the same order
  const int n_wg = pass1_grid(A->n, p);
  if (n_wg > NOALLOC_MAX_WG || (size_t)n_wg * p > NOALLOC_PART) return BMR_WORKSPACE_TOO_SMALL;
  double* base = nullptr;
  const int e = scratch_address(&base);
  if (e) return e;
  const int r = residual_norms(A, B, X, p, R, base, n_wg, base + NOALLOC_PART, stream, norms);
  return r == 0 ? BMR_CONVERGED : r;
}
