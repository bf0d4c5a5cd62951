// Incomplete Cholesky IC(0) preconditioner on the device: the numeric
// factorisation and the block triangular solves, both level-scheduled.
//
// C is lower triangular with the pattern of the lower triangle of M.  Row i
// of C needs the finished rows j < i of its pattern, so the rows fall into
// levels (level(i) = 1 + the largest level of those rows, 0 without any):
// the rows of one level are independent and one launch handles one level.
// The backward solve with C^T runs the same levels in reverse order: row i
// of C^T needs the rows j > i with C(j, i) != 0, all of a higher level.
//
// Storage (device, inside the caller's IC(0) buffer): the strictly lower
// part of C in CSR (row pointers, columns ascending, values), its transpose
// (the strictly upper part of C^T) in CSR with the position of each entry in
// the lower arrays, the diagonal, and the rows sorted by level.
//
// Factorisation of row i (the row recurrence of Cholesky with every entry
// outside the pattern dropped):
//     C(i,j) = (M(i,j) - sum_{k<j} C(i,k) C(j,k)) / C(j,j),  j < i in the pattern, ascending,
//     C(i,i) = sqrt(M(i,i) - sum_{k<i} C(i,k)^2),
// the sums over the columns k the rows i and j share (a merge of the two
// sorted column lists).  A pivot that is not positive marks a breakdown.
#include <math.h>

#include "bmr_internal.hpp"

namespace bmr {
namespace {

constexpr int WG = 256;

// One thread per row of the level.
__global__ __launch_bounds__(WG) void k_ic0_level(const int32_t* __restrict__ rows, int lo, int hi,
                                                  const int32_t* __restrict__ lrp, const int32_t* __restrict__ lci,
                                                  const int32_t* __restrict__ lmap, const int32_t* __restrict__ dmap,
                                                  const double* __restrict__ mval, double* __restrict__ lval,
                                                  double* __restrict__ diag, int* __restrict__ fail) {
  const int r = lo + blockIdx.x * WG + threadIdx.x;
  if (r >= hi) return;
  const int i = rows[r];
  const int s = lrp[i], e = lrp[i + 1];
  double sq = 0.0;
  for (int q = s; q < e; ++q) {
    const int j = lci[q];
    double t = mval[lmap[q]];
    // shared columns k < j of rows i (entries s .. q-1) and j (all of row j)
    int a = s, b = lrp[j];
    const int bend = lrp[j + 1];
    while (a < q && b < bend) {
      const int ka = lci[a], kb = lci[b];
      if (ka == kb) {
        t -= lval[a] * lval[b];
        ++a;
        ++b;
      } else if (ka < kb) {
        ++a;
      } else {
        ++b;
      }
    }
    const double v = t / diag[j];
    lval[q] = v;
    sq += v * v;
  }
  const double d = mval[dmap[i]] - sq;
  if (d > 0.0 && isfinite(d)) {
    diag[i] = sqrt(d);
  } else {
    diag[i] = 1.0;  // keeps later levels finite; the factorisation is reported as failed
    atomicOr(fail, 1);
  }
}

// Values of the transposed (strictly upper) part from the lower one, and
// both parts divided by the pivot of the row each entry multiplies (used by
// the one-launch solves of two-level factors).
__global__ void k_ic0_upper(const int32_t* __restrict__ upos, const int32_t* __restrict__ lci,
                            const int32_t* __restrict__ uci, const double* __restrict__ lval,
                            const double* __restrict__ diag, double* __restrict__ uval,
                            double* __restrict__ lval_s, double* __restrict__ uval_s, int64_t nnz) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const double u = lval[upos[e]];
    uval[e] = u;
    uval_s[e] = u / diag[uci[e]];
    lval_s[e] = lval[e] / diag[lci[e]];
  }
}

// One level of a triangular solve with p right-hand sides (row-interleaved):
//     y_i = (rhs_i - sum_{e in row i} val_e y_{col_e}) / diag_i
// for the rows of the level, in the order of the row's entries.  rhs may be
// y itself (each row reads its own right-hand side before writing it, and
// reads only rows of earlier levels).  LPR lanes per row, each holding CPL
// adjacent columns; the halt flag of the solver state (when given) turns the
// launch into a no-op once the iteration has stopped.
template <int P>
struct TrsvShape {
  static constexpr int CPL = (P % 2 == 0) ? 2 : 1;
  static constexpr int LPR = (P + CPL - 1) / CPL <= 1 ? 1 : (P + CPL - 1) / CPL <= 2 ? 2 : (P + CPL - 1) / CPL <= 4 ? 4
                             : (P + CPL - 1) / CPL <= 8 ? 8 : 16;
  static constexpr int RPB = WG / LPR;  // rows per workgroup
};

template <int P>
__global__ __launch_bounds__(WG) void k_trsv_level(const int32_t* __restrict__ rows, int lo, int hi,
                                                   const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                   const double* __restrict__ va, const double* __restrict__ diag,
                                                   const double* rhs, double* y, const DevState* __restrict__ st) {
  if (st && st->halt) return;
  using S = TrsvShape<P>;
  constexpr int CPL = S::CPL, LPR = S::LPR;
  const int r = lo + blockIdx.x * S::RPB + threadIdx.x / LPR;
  const int c0 = (threadIdx.x % LPR) * CPL;
  if (r >= hi || c0 >= P) return;
  const int64_t i = rows[r];
  double acc[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) acc[k] = 0.0;
  const int s = rp[i], e = rp[i + 1];
  for (int q = s; q < e; ++q) {
    const int64_t j = ci[q];
    const double v = va[q];
#pragma unroll
    for (int k = 0; k < CPL; ++k)
      if (c0 + k < P) acc[k] = fma(v, y[j * P + c0 + k], acc[k]);
  }
  const double d = diag[i];
#pragma unroll
  for (int k = 0; k < CPL; ++k)
    if (c0 + k < P) y[i * P + c0 + k] = (rhs[i * P + c0 + k] - acc[k]) / d;
}

}  // namespace

hipError_t launch_ic0_factor(const Ic0View& v, const double* mval, int* fail, hipStream_t s) {
  for (int l = 0; l < v.n_levels; ++l) {
    const int lo = v.level_ptr[l], hi = v.level_ptr[l + 1];
    if (hi <= lo) continue;
    const int grid = (hi - lo + WG - 1) / WG;
    hipLaunchKernelGGL(k_ic0_level, dim3(grid), dim3(WG), 0, s, v.level_rows, lo, hi, v.lrp, v.lci, v.lmap, v.dmap,
                       mval, v.lval, v.diag, fail);
  }
  if (v.nnz_l > 0) {
    const int64_t g = std::min<int64_t>(8192, (v.nnz_l + WG - 1) / WG);
    hipLaunchKernelGGL(k_ic0_upper, dim3((int)g), dim3(WG), 0, s, v.upos, v.lci, v.uci, (const double*)v.lval,
                       (const double*)v.diag, v.uval, v.lval_s, v.uval_s, v.nnz_l);
  }
  return hipGetLastError();
}

hipError_t launch_ic0_solve(const Ic0View& v, int p, bool trans, const double* rhs, double* y, const DevState* st,
                            hipStream_t s) {
  if (v.n_levels == 2 && rhs != y)  // one launch (two-level factor, out of place)
    return launch_trisolve2(p, trans ? v.urp : v.lrp, trans ? v.uci : v.lci, trans ? v.uval_s : v.lval_s, v.diag, v.n,
                            rhs, y, st, s);
  const int32_t* rp = trans ? v.urp : v.lrp;
  const int32_t* ci = trans ? v.uci : v.lci;
  const double* va = trans ? v.uval : v.lval;
#define LT(P)                                                                                                    \
  {                                                                                                              \
    constexpr int RPB = TrsvShape<P>::RPB;                                                                       \
    for (int q = 0; q < v.n_levels; ++q) {                                                                       \
      const int l = trans ? v.n_levels - 1 - q : q;                                                              \
      const int lo = v.level_ptr[l], hi = v.level_ptr[l + 1];                                                    \
      if (hi <= lo) continue;                                                                                    \
      hipLaunchKernelGGL(k_trsv_level<P>, dim3((hi - lo + RPB - 1) / RPB), dim3(WG), 0, s, v.level_rows, lo, hi, \
                         rp, ci, va, (const double*)v.diag, rhs, y, st);                                         \
    }                                                                                                            \
  }
  switch (p) {
    case 1: LT(1) break;
    case 2: LT(2) break;
    case 3: LT(3) break;
    case 4: LT(4) break;
    case 5: LT(5) break;
    case 6: LT(6) break;
    case 7: LT(7) break;
    case 8: LT(8) break;
    case 9: LT(9) break;
    case 10: LT(10) break;
    case 11: LT(11) break;
    case 12: LT(12) break;
    case 13: LT(13) break;
    case 14: LT(14) break;
    case 15: LT(15) break;
    case 16: LT(16) break;
    default: return hipErrorInvalidValue;
  }
#undef LT
  return hipGetLastError();
}

}  // namespace bmr
