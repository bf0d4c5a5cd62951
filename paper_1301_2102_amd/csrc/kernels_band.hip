// Reduction of the pass-1 partial sums and the band kernel: one workgroup
// that turns the p x p Gram products of a block iteration into the new block
// of the band Hessenberg matrix, reduces its p columns by Givens rotations,
// updates the rotated right-hand-side window S-hat, records the residual
// recurrence and decides whether to stop (Sections 3-5, Algorithm 7.1).
//
// Block iteration k covers band iterations j = (k-1)p + l + 1, l = 0..p-1.
// With V_k = [u_{(k-1)p+1} .. u_{kp}], the columns of H-bar touched by block
// k are (eq. (2.6) with the symmetry of Section 7):
//     rows of block k-1:  h_{(k-2)p+r+1, j} = B_{k-1}(l, r),  r >= l
//     rows of block k:    A_k(r, l)
//     rows of block k+1:  B_k(r, l),  r <= l
// A_k(r, l) for r >= l is the inner product of u_{(k-1)p+r+1} with the
// candidate of column l (the modified Gram-Schmidt coefficient in exact
// arithmetic), and the entries above the diagonal are taken from below by
// symmetry; B_k is the triangular factor of the remainder
// W' = W - V_k A_k = V_{k+1} B_k, obtained by Cholesky from the Gram
// products of pass 1.  When a pivot falls below tau * ||A u_j|| the Gram
// route cannot resolve the dependence test (Section 5) and the host runs the
// new-block QR column by column instead.
#include <math.h>

#include "bmr_internal.hpp"

namespace bmr {
namespace {

__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ part, int n_wg, double* __restrict__ red,
                                                DevState* __restrict__ st, int check_halt) {
  if (check_halt && st->halt) return;
  const int e = blockIdx.x;
  const double* src = part + (size_t)e * n_wg;
  double s = 0.0;
  for (int i = threadIdx.x; i < n_wg; i += 256) s += src[i];
  __shared__ double sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) red[e] = sh[0];
}

// Givens pair zeroing b against a: r = hypot(a, b), c = a / r, s = b / r;
// the identity when b is exactly zero.
__device__ inline void givens(double a, double b, double& c, double& s) {
  if (b == 0.0) {
    c = 1.0;
    s = 0.0;
  } else {
    const double r = hypot(a, b);
    c = a / r;
    s = b / r;
  }
}

__device__ void halt_with(DevState* st, int status, int reason) {
  st->status = status;
  st->reason = reason;
  st->halt = 1;
  st->k2 = 0;
}

// Phase A: A_k, Gram of the remainder, Cholesky -> B_k and bench coefficients.
// Returns false when the column-wise QR must take over.
__device__ bool phase_a(const double* __restrict__ red, DevState* __restrict__ st) {
#pragma clang fp contract(off)
  const int p = st->p, nb = st->nb, taken = st->taken;
  const double* G = red + off_G(p);
  const double* Q = red + off_Q(p);
  const double* Pm = red + off_P(p);
  const double* a2 = red + off_a(p);
  const double* Wg = red + off_Wg(p);
  const double* Vg = red + off_Vg(p, nb);
  double* Ak = st->Ak;
  double* Bk = st->Bk;
  for (int r = 0; r < p; ++r)
    for (int c = 0; c < p; ++c) Ak[r * MAXP + c] = (r >= c) ? G[r * p + c] : G[c * p + r];
  for (int c = 0; c < p; ++c) st->araw[c] = sqrt(a2[c]);
  // Gamma = Q - Ak^T G - G^T Ak + Ak^T Pm Ak   (Gram of W - V_k A_k)
  double T1[MAXP * MAXP], T2[MAXP * MAXP], Gam[MAXP * MAXP];
  for (int l = 0; l < p; ++l)
    for (int m = 0; m < p; ++m) {
      double t = 0.0, u = 0.0;
      for (int r = 0; r < p; ++r) {
        t += Ak[r * MAXP + l] * G[r * p + m];
        u += Pm[l * p + r] * Ak[r * MAXP + m];
      }
      T1[l * MAXP + m] = t;  // (Ak^T G)(l, m)
      T2[l * MAXP + m] = u;  // (Pm Ak)(l, m)
    }
  for (int l = 0; l < p; ++l)
    for (int m = 0; m < p; ++m) {
      double t = 0.0;
      for (int r = 0; r < p; ++r) t += Ak[r * MAXP + l] * T2[r * MAXP + m];
      Gam[l * MAXP + m] = Q[l * p + m] - T1[l * MAXP + m] - T1[m * MAXP + l] + t;
    }
  // Cholesky, row-oriented like the column-by-column Gram-Schmidt it replaces
  for (int c = 0; c < MAXP * MAXP; ++c) Bk[c] = 0.0;
  for (int l = 0; l < p; ++l) {
    for (int r = 0; r < l; ++r) {
      double t = 0.5 * (Gam[r * MAXP + l] + Gam[l * MAXP + r]);
      for (int q = 0; q < r; ++q) t -= Bk[q * MAXP + r] * Bk[q * MAXP + l];
      Bk[r * MAXP + l] = t / Bk[r * MAXP + r];
    }
    double d = Gam[l * MAXP + l];
    for (int q = 0; q < l; ++q) d -= Bk[q * MAXP + l] * Bk[q * MAXP + l];
    const double thr = st->tau_fb * st->araw[l];
    if (!(d > 0.0) || !(sqrt(d) >= thr) || !isfinite(d)) return false;
    Bk[l * MAXP + l] = sqrt(d);
  }
  // bench: coefficients of V_{k+1}^T g_b = B_k^{-T} (W^T g_b - A_k^T V_k^T g_b)
  for (int b = 0; b < MAXB; ++b)
    for (int l = 0; l < MAXP; ++l) st->bcoef[b * MAXP + l] = 0.0;
  for (int b = taken; b < nb; ++b) {
    double cf[MAXP];
    for (int l = 0; l < p; ++l) {
      double gw = Wg[l * nb + b];
      for (int r = 0; r < p; ++r) gw -= Ak[r * MAXP + l] * Vg[r * nb + b];
      for (int r = 0; r < l; ++r) gw -= Bk[r * MAXP + l] * cf[r];
      cf[l] = gw / Bk[l * MAXP + l];
      st->bcoef[b * MAXP + l] = cf[l];
    }
  }
  for (int c = 0; c < MAXP * MAXP; ++c) {
    st->P2A[c] = Ak[c];
    st->P2B[c] = Bk[c];
  }
  return true;
}

// Phase B: Givens QR of the p new columns of H-bar, S-hat window, residuals,
// stopping test, coefficients of the search directions and of the X update.
__device__ void phase_b(DevState* __restrict__ st, double* __restrict__ hist) {
#pragma clang fp contract(off)
  const int p = st->p;
  const int64_t k = st->k;
  const int64_t j0 = st->j;
  const double* Bprev = st->Bprev;
  const double* Ak = st->Ak;
  const double* Bk = st->Bk;
  double col[4 * MAXP];
  double S2[2 * MAXP][MAXP];
  double nrot[MAXP][MAXP][2];
  for (int r = 0; r < p; ++r)
    for (int c = 0; c < p; ++c) {
      S2[r][c] = st->Shat[r * MAXP + c];
      S2[p + r][c] = 0.0;
    }
  int lstar = p;
  int finished = 0, status = STATUS_RUNNING;
  for (int l = 0; l < p; ++l) {
    if (l >= st->lcap) {  // the column-wise QR ran out of substitutes at column l
      status = st->cap_status;
      finished = 1;
      lstar = l;
      break;
    }
    const int64_t j = j0 + l + 1;
    for (int r = 0; r < 4 * MAXP; ++r) col[r] = 0.0;
    for (int r = l; r < p; ++r) col[p + r] = Bprev[l * MAXP + r];
    for (int r = 0; r < p; ++r) col[2 * p + r] = Ak[r * MAXP + l];
    for (int r = 0; r <= l; ++r) col[3 * p + r] = Bk[r * MAXP + l];
    // rotations of columns j-2p .. j-1 (blocks k-2, k-1 and the first l of block k)
    if (k - 2 >= 1) {
      const int rb = (int)((k - 2) % 3);
      for (int i = l; i < p; ++i)
        for (int t = 1; t <= p; ++t) {
          const double c = st->rot[rb][i][t - 1][0], s = st->rot[rb][i][t - 1][1];
          const double a = col[i], b = col[i + t];
          col[i] = c * a + s * b;
          col[i + t] = -s * a + c * b;
        }
    }
    if (k - 1 >= 1) {
      const int rb = (int)((k - 1) % 3);
      for (int i = 0; i < p; ++i)
        for (int t = 1; t <= p; ++t) {
          const double c = st->rot[rb][i][t - 1][0], s = st->rot[rb][i][t - 1][1];
          const double a = col[p + i], b = col[p + i + t];
          col[p + i] = c * a + s * b;
          col[p + i + t] = -s * a + c * b;
        }
    }
    for (int i = 0; i < l; ++i)
      for (int t = 1; t <= p; ++t) {
        const double c = nrot[i][t - 1][0], s = nrot[i][t - 1][1];
        const double a = col[2 * p + i], b = col[2 * p + i + t];
        col[2 * p + i] = c * a + s * b;
        col[2 * p + i + t] = -s * a + c * b;
      }
    // new rotations: zero the p subdiagonal entries of column j
    const int piv = 2 * p + l;
    for (int t = 1; t <= p; ++t) {
      double c, s;
      givens(col[piv], col[piv + t], c, s);
      nrot[l][t - 1][0] = c;
      nrot[l][t - 1][1] = s;
      if (s != 0.0) {
        col[piv] = hypot(col[piv], col[piv + t]);
        col[piv + t] = 0.0;
        for (int q = 0; q < p; ++q) {
          const double a = S2[l][q], b = S2[l + t][q];
          S2[l][q] = c * a + s * b;
          S2[l + t][q] = -s * a + c * b;
        }
      }
    }
    if (!(col[piv] != 0.0)) {
      halt_with(st, isfinite(col[piv]) ? BMR_SINGULAR_R : BMR_NONFINITE, REASON_ERROR);
      st->j = j - 1;
      return;
    }
    for (int r = 0; r < p; ++r) {
      st->Ra[r * MAXP + l] = (r >= l) ? col[r] : 0.0;
      st->Rb[r * MAXP + l] = col[p + r];
      st->Rc[r * MAXP + l] = (r <= l) ? col[2 * p + r] : 0.0;
    }
    for (int q = 0; q < p; ++q) st->Z[l * MAXP + q] = S2[l][q];
    // recurrence residual rho_j^{(i)} = ||S-hat(j+1:j+p, i)|| (eq. (3.5))
    double worst = 0.0;
    int bad = 0;
    for (int q = 0; q < p; ++q) {
      double ss = 0.0;
      for (int t = 1; t <= p; ++t) ss += S2[l + t][q] * S2[l + t][q];
      const double rho = sqrt(ss);
      const double ratio = st->beta[q] > 0.0 ? rho / st->beta[q] : 0.0;
      if (!isfinite(ratio)) bad = 1;
      st->rho[q] = ratio;
      if (j <= st->hist_cap) hist[(j - 1) * p + q] = ratio;
      worst = fmax(worst, ratio);
    }
    if (bad) {
      halt_with(st, BMR_NONFINITE, REASON_ERROR);
      st->j = j - 1;
      return;
    }
    if (worst < st->tol) {
      status = BMR_CONVERGED;
      finished = 1;
    } else if (j >= st->max_iter) {
      status = BMR_MAX_ITER;
      finished = 1;
    }
    if (finished) {
      lstar = l + 1;
      break;
    }
  }
  if (finished && lstar == 0) {
    halt_with(st, status, REASON_FINISHED);
    return;
  }
  st->lstar = lstar;
  st->k2 = k;
  if (finished) {
    st->j = j0 + lstar;
    st->status = status;
    st->reason = REASON_FINISHED;
    st->halt = 1;
    return;
  }
  const int rk = (int)(k % 3);
  for (int i = 0; i < p; ++i)
    for (int t = 0; t < p; ++t) {
      st->rot[rk][i][t][0] = nrot[i][t][0];
      st->rot[rk][i][t][1] = nrot[i][t][1];
    }
  for (int c = 0; c < MAXP * MAXP; ++c) st->Bprev[c] = Bk[c];
  for (int r = 0; r < p; ++r)
    for (int c = 0; c < p; ++c) st->Shat[r * MAXP + c] = S2[p + r][c];
  st->j = j0 + p;
  st->k = k + 1;
}

// mode 0: phase A then phase B.  mode 1: the host has supplied B_k (column-
// wise QR) and already formed V_{k+1}; run phase B with pass 2 told to keep
// V_{k+1} as it is.
__global__ __launch_bounds__(64) void k_band(int mode, const double* __restrict__ red, double* __restrict__ hist,
                                            DevState* __restrict__ st) {
  if (threadIdx.x != 0) return;
  if (st->halt) {
    st->k2 = 0;
    return;
  }
  if (mode == 0) {
    if (!phase_a(red, st)) {
      st->reason = REASON_EXPLICIT_QR;
      st->halt = 1;
      st->k2 = 0;
      return;
    }
  } else {
    for (int c = 0; c < MAXP * MAXP; ++c) {
      st->P2A[c] = 0.0;
      st->P2B[c] = ((c / MAXP) == (c % MAXP)) ? 1.0 : 0.0;
    }
    for (int c = 0; c < MAXB * MAXP; ++c) st->bcoef[c] = 0.0;
  }
  phase_b(st, hist);
}

}  // namespace

hipError_t launch_reduce(const double* part, int n_wg, int n_ent, double* red, DevState* st, int check_halt,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(n_ent), dim3(256), 0, s, part, n_wg, red, st, check_halt);
  return hipGetLastError();
}

hipError_t launch_band(int mode, const double* red, double* hist, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_band, dim3(1), dim3(64), 0, s, mode, red, hist, st);
  return hipGetLastError();
}

}  // namespace bmr
