// Column-wise QR of a block of p columns on the device: the initial QR of
// F_0 = B (eq. (3.2)) and the new-block QR of a block iteration whose Gram
// route the band kernel rejected.  Each column is orthogonalised by classical
// Gram-Schmidt applied twice against the columns before it; its remainder
// norm is compared with gamma times a reference norm (||b_i|| at set-up,
// ||A u_j|| in the loop; the dependence test of Section 5), and a dependent
// column is replaced by the next vector of the substitutes bench, normalised
// (Section 5.1); then every unused bench vector takes one Gram-Schmidt step
// against the new column.
//
// With retained candidates (Section 5.1, last paragraph; a candidate removed
// in place of basis vector u_m is kept and the new basis vectors
// u_{m+1} .. u_{m+2p} take one Gram-Schmidt step against it), each column
// also takes those steps after its CGS2, in the order the candidates were
// kept, and a dependent column whose norm is above the retention floor is
// saved, normalised, before a substitute replaces it.  The coefficients of
// these steps are not recorded in the triangular factor.
//
// Every step is a fixed sequence of launches on the caller's stream:
//   dots    partial sums over n, one per workgroup (entry-major),
//   decide  one workgroup adds the partial sums in a fixed order and takes
//           the step's decision (coefficients, dependence, substitute,
//           exhaustion) into the device state,
//   apply   the column update with the coefficients from the state.
// Steps that a decision made unnecessary (the bench norm of an independent
// column, everything after the bench ran out) return at once.  The host
// therefore enqueues the whole QR without waiting for any of its results.
// Products and sums are FP64 for both storage types.
#include <math.h>

#include "bmr_internal.hpp"

namespace bmr {
namespace {

constexpr int WG = 256;
constexpr int MAXQ = MAXP > MAXB ? MAXP : MAXB;  // sums per dots launch

// Step kinds.  ST_KEPT + q: the step of a new column against retained
// candidate q; ST_SUBK + q: the same for a substitute (whose window includes
// the candidate's own index); ST_MGSV + r, ST_MGSD + q: the modified
// Gram-Schmidt step of the retained mode against column r of V_k or column
// q of the new block.
enum {
  ST_CGS = 0, ST_NORM = 1, ST_BENCH = 2, ST_BORTH = 3, ST_SAVE = 4, ST_RENORM = 5, ST_SYM = 6,
  ST_KEPT = 8, ST_SUBK = 12, ST_MGSV = 16, ST_MGSD = 32
};

// Basis index of column l of the block being orthogonalised: u_{l+1} at
// set-up, u_{kp+l+1} for the new block of block iteration k.
__device__ inline int64_t basis_index(int mode, int l, int p, const DevState* st) {
  return (mode == QR_LOOP ? st->k * p : 0) + l + 1;
}

// Whether step `step` of column l still has work: the QR is active, and the
// bench norm is wanted only for a dependent column, the bench update only
// while unused bench vectors remain, the copy of a kept candidate only when
// one was kept, the second normalisation only after a substitute was
// projected; the steps against retained candidate q (kept_live) only inside
// its window, and for a substitute only when the column was substituted.
__device__ inline bool step_live(int step, int nb, const DevState* st) {
  if (!st->qr_active) return false;
  if (step == ST_BENCH) return st->qr_need_bench != 0;
  if (step == ST_BORTH) return st->taken < nb;
  if (step == ST_SAVE) return st->qr_keep != 0;
  if (step == ST_RENORM) return st->qr_hit != 0;
  return true;
}
__device__ inline bool kept_live(int q, bool subst, int mode, int l, int p, const DevState* st) {
  if (!st->qr_active || q >= st->n_kept) return false;
  if (subst && st->qr_src == 0) return false;
  const int64_t m = basis_index(mode, l, p, st), mk = st->kept_m[q];
  return (subst ? mk : mk + 1) <= m && m <= mk + 2 * p;
}

// Decode a step kind: the base kind, and q (retained candidate or column).
__device__ inline int step_base(int step, int& q) {
  if (step >= ST_MGSD) { q = step - ST_MGSD; return ST_MGSD; }
  if (step >= ST_MGSV) { q = step - ST_MGSV; return ST_MGSV; }
  if (step >= ST_SUBK) { q = step - ST_SUBK; return ST_SUBK; }
  if (step >= ST_KEPT) { q = step - ST_KEPT; return ST_KEPT; }
  q = 0;
  return step;
}
__device__ inline bool live(int step, int q, int mode, int l, int p, int nb, const DevState* st) {
  if (step == ST_KEPT || step == ST_SUBK) return kept_live(q, step == ST_SUBK, mode, l, p, st);
  if (step == ST_MGSV || step == ST_MGSD || step == ST_SYM) return st->qr_active != 0;
  return step_live(step, nb, st);
}

// Number of sums of a dots step.
__device__ inline int step_sums(int step, int l, int nb) {
  return step == ST_CGS ? l : step == ST_BORTH ? nb : 1;
}

__global__ void k_qr_begin(int mode, int p, DevState* __restrict__ st) {
  const int t = threadIdx.x;
  for (int e = t; e < MAXP * MAXP; e += blockDim.x) st->qr_R[e] = 0.0;
  if (mode == QR_LOOP && t < MAXP) st->qr_ref[t] = t < p ? st->araw[t] : 0.0;
  if (t == 0) {
    st->qr_active = 1;
    st->qr_keep = 0;
    st->qr_hit = 0;
    st->qr_need_bench = 0;
    st->qr_src = 0;
    st->qr_b = 0;
    st->qr_div = 1.0;
    st->qr_lcap = p;
    st->qr_error = 0;
  }
}

// W <- W - V_k A_k (the part of the new block's orthogonalisation against
// V_k that pass 2 would have applied), column by column in FP64, rounded
// once.  One thread per row.
template <typename T>
__global__ __launch_bounds__(WG) void k_qr_sub(int p, T* __restrict__ W, const T* __restrict__ Vk, int64_t n,
                                               const DevState* __restrict__ st) {
  const int64_t stride = (int64_t)gridDim.x * WG;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
    double v[MAXP];
#pragma unroll
    for (int q = 0; q < MAXP; ++q) v[q] = q < p ? (double)Vk[i * p + q] : 0.0;
#pragma unroll
    for (int l = 0; l < MAXP; ++l) {
      if (l < p) {
        double y = (double)W[i * p + l];
#pragma unroll
        for (int q = 0; q < MAXP; ++q)
          if (q < p) y = fma(-st->Ak[q * MAXP + l], v[q], y);
        W[i * p + l] = (T)y;
      }
    }
  }
}

// Partial sums of one step, part[e * n_wg + workgroup]:
//   CGS    e < l:   D(:, e) . D(:, l)
//   NORM   e = 0:   D(:, l) . D(:, l)
//   BENCH  e = 0:   g_b . g_b for the next unused bench vector b = taken
//   BORTH  e < nb:  g_e . D(:, l)  (entries below `taken` are not used)
//   KEPT, SUBK  e = 0:  r_q . D(:, l) for retained candidate q
//   RENORM e = 0:   D(:, l) . D(:, l)
//   MGSV, MGSD e = 0:  V_k(:, q) . D(:, l),  D(:, q) . D(:, l)
template <typename T>
__global__ __launch_bounds__(WG) void k_qr_dots(int step, int mode, int l, int p, const T* __restrict__ D,
                                                const T* __restrict__ Vk, const T* __restrict__ bench,
                                                const T* __restrict__ ret, int nb, int64_t n,
                                                double* __restrict__ part, int n_wg,
                                                const DevState* __restrict__ st) {
  int q;
  step = step_base(step, q);
  if (!live(step, q, mode, l, p, nb, st)) return;
  if (step == ST_RENORM) step = ST_NORM;
  const int m = step_sums(step, l, nb);
  const int b = st->taken;
  double acc[MAXQ];
#pragma unroll
  for (int e = 0; e < MAXQ; ++e) acc[e] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * WG;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
    if (step == ST_BENCH) {
      const double y = (double)bench[i * nb + b];
      acc[0] = fma(y, y, acc[0]);
    } else if (step == ST_KEPT || step == ST_SUBK) {
      acc[0] = fma((double)ret[i * nb + q], (double)D[i * p + l], acc[0]);
    } else if (step == ST_MGSV) {
      acc[0] = fma((double)Vk[i * p + q], (double)D[i * p + l], acc[0]);
    } else if (step == ST_MGSD) {
      acc[0] = fma((double)D[i * p + q], (double)D[i * p + l], acc[0]);
    } else {
      const double y = (double)D[i * p + l];
      if (step == ST_NORM) {
        acc[0] = fma(y, y, acc[0]);
      } else if (step == ST_CGS) {
#pragma unroll
        for (int e = 0; e < MAXP; ++e)
          if (e < m) acc[e] = fma((double)D[i * p + e], y, acc[e]);
      } else {
#pragma unroll
        for (int e = 0; e < MAXB; ++e)
          if (e < m) acc[e] = fma((double)bench[i * nb + e], y, acc[e]);
      }
    }
  }
  // wavefront sums by shuffles, then the four wavefronts in order
  __shared__ double sh[WG / 64][MAXQ];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int e = 0; e < MAXQ; ++e) {
    if (e < m) {
      double a = acc[e];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
      if (lane == 0) sh[wave][e] = a;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < m) {
    const int e = threadIdx.x;
    part[(size_t)e * n_wg + blockIdx.x] = (sh[0][e] + sh[1][e]) + (sh[2][e] + sh[3][e]);
  }
}

// The sums of one step (one wavefront per entry, fixed order) and its
// decision, taken by thread 0 into the state.
__global__ __launch_bounds__(WG) void k_qr_decide(int step, int mode, int l, int p, int nb,
                                                  const double* __restrict__ part, int n_wg,
                                                  DevState* __restrict__ st) {
  int q;
  step = step_base(step, q);
  if (!live(step, q, mode, l, p, nb, st)) return;
  const int m = step_sums(step == ST_RENORM ? ST_NORM : step, l, nb);
  __shared__ double sum[MAXQ];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = wave; e < m; e += WG / 64) {
    const double* src = part + (size_t)e * n_wg;
    double s = 0.0;
    for (int i = lane; i < n_wg; i += 64) s += src[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) sum[e] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (step == ST_CGS) {
    for (int r = 0; r < l; ++r) {
      st->qr_coef[r] = sum[r];
      st->qr_R[r * MAXP + l] += sum[r];
    }
  } else if (step == ST_KEPT) {
    st->qr_coef[0] = sum[0];
  } else if (step == ST_SUBK) {
    st->qr_coef[0] = sum[0];
    st->qr_hit = 1;
  } else if (step == ST_RENORM) {
    st->qr_div = sqrt(sum[0]);
  } else if (step == ST_MGSV) {  // coefficient of u_{(k-1)p+q+1}, q >= l
    st->qr_coef[0] = sum[0];
    st->qr_M[q * MAXP + l] = sum[0];
  } else if (step == ST_MGSD) {  // coefficient of the new block's column q < l
    st->qr_coef[0] = sum[0];
    st->qr_R[q * MAXP + l] = sum[0];
  } else if (step == ST_NORM) {
    const double eta = sqrt(sum[0]);
    st->qr_keep = 0;
    st->qr_hit = 0;
    if (!isfinite(eta)) {
      st->qr_error = 1;
      st->qr_active = 0;
      st->qr_lcap = l;
      return;
    }
    if (eta <= st->gamma * st->qr_ref[l]) {  // dependent: a substitute is needed
      // kept only when a substitute can take its place (every keep then takes
      // a bench vector, so at most nb are kept: the slots of the n x nb array)
      if (st->retain && eta > RETAIN_FLOOR * st->qr_ref[l] && st->taken < nb && st->n_kept < nb) {
        // kept, normalised, in the next slot (the copy is the next apply step)
        const int q = st->n_kept;
        st->qr_keep = 1;
        st->qr_keep_slot = q;
        st->kept_m[q] = basis_index(mode, l, p, st);
        st->n_kept = q + 1;
        st->qr_div = eta;
      }
      st->qr_R[l * MAXP + l] = 0.0;
      if (st->taken < nb) {
        st->qr_need_bench = 1;
      } else {
        st->qr_active = 0;
        st->qr_lcap = l;
      }
    } else {
      st->qr_R[l * MAXP + l] = eta;
      st->qr_need_bench = 0;
      st->qr_src = 0;
      st->qr_div = eta;
    }
  } else if (step == ST_BENCH) {
    const int b = st->taken;
    const double gn = sqrt(sum[0]);
    st->qr_need_bench = 0;
    if (gn > st->gamma * st->bench_norm0[b]) {
      st->qr_src = 1;
      st->qr_b = b;
      st->qr_div = gn;
      st->taken = b + 1;
      st->n_replaced += 1;
    } else {  // the bench vector has no direction left outside the basis
      st->qr_active = 0;
      st->qr_lcap = l;
    }
  } else {
    for (int b = 0; b < nb; ++b) st->qr_coef[b] = sum[b];
  }
}

// The column update of a step, in FP64 and rounded to T once:
//   CGS    D(:, l) -= sum_{r<l} coef_r D(:, r)
//   NORM   D(:, l) = source / div, source the column itself or bench vector qr_b
//   BORTH  g_b -= coef_b D(:, l) for every unused bench vector b
//   KEPT   D(:, l) -= coef r_q
//   SAVE   r_slot = D(:, l) / div (the dependent candidate, before a substitute replaces it)
//   SUBK   as KEPT, for a substitute
//   RENORM D(:, l) /= div
//   SYM    D(:, l) -= sum_{r<l} M(l, r) V_k(:, r) (the coefficients of the block's
//          earlier candidates, by symmetry), one column after the other
//   MGSV, MGSD  D(:, l) -= coef V_k(:, q),  D(:, l) -= coef D(:, q)
template <typename T>
__global__ __launch_bounds__(WG) void k_qr_apply(int step, int mode, int l, int p, T* __restrict__ D,
                                                 const T* __restrict__ Vk, T* __restrict__ bench,
                                                 T* __restrict__ ret, int nb, int64_t n,
                                                 const DevState* __restrict__ st) {
  int q;
  step = step_base(step, q);
  if (!live(step, q, mode, l, p, nb, st)) return;
  const int64_t stride = (int64_t)gridDim.x * WG;
  const int64_t i0 = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (step == ST_KEPT || step == ST_SUBK) {
    const double c = st->qr_coef[0];
    for (int64_t i = i0; i < n; i += stride)
      D[i * p + l] = (T)fma(-c, (double)ret[i * nb + q], (double)D[i * p + l]);
  } else if (step == ST_RENORM) {
    const double div = st->qr_div;
    for (int64_t i = i0; i < n; i += stride) D[i * p + l] = (T)((double)D[i * p + l] / div);
  } else if (step == ST_SYM) {
    for (int64_t i = i0; i < n; i += stride) {
      double y = (double)D[i * p + l];
#pragma unroll
      for (int r = 0; r < MAXP; ++r)
        if (r < l) y = fma(-st->qr_M[l * MAXP + r], (double)Vk[i * p + r], y);
      D[i * p + l] = (T)y;
    }
  } else if (step == ST_MGSV || step == ST_MGSD) {
    const double c = st->qr_coef[0];
    const T* src = step == ST_MGSV ? Vk : D;
    for (int64_t i = i0; i < n; i += stride)
      D[i * p + l] = (T)fma(-c, (double)src[i * p + q], (double)D[i * p + l]);
  } else if (step == ST_SAVE) {
    const int slot = st->qr_keep_slot;
    const double div = st->qr_div;
    for (int64_t i = i0; i < n; i += stride) ret[i * nb + slot] = (T)((double)D[i * p + l] / div);
  } else if (step == ST_CGS) {
    for (int64_t i = i0; i < n; i += stride) {
      double y = (double)D[i * p + l];
#pragma unroll
      for (int r = 0; r < MAXP; ++r)
        if (r < l) y = fma(-st->qr_coef[r], (double)D[i * p + r], y);
      D[i * p + l] = (T)y;
    }
  } else if (step == ST_NORM) {
    const bool from_bench = st->qr_src != 0;
    const int b = st->qr_b;
    const double div = st->qr_div;
    for (int64_t i = i0; i < n; i += stride) {
      const double y = from_bench ? (double)bench[i * nb + b] : (double)D[i * p + l];
      D[i * p + l] = (T)(y / div);
    }
  } else {
    const int taken = st->taken;
    for (int64_t i = i0; i < n; i += stride) {
      const double u = (double)D[i * p + l];
#pragma unroll
      for (int b = 0; b < MAXB; ++b)
        if (b >= taken && b < nb) bench[i * nb + b] = (T)fma(-st->qr_coef[b], u, (double)bench[i * nb + b]);
    }
  }
}

// End of a QR in the loop: B_k and the column cap to the state and the
// device loop resumes (or stops with an error after a non-finite norm).
__global__ void k_qr_end(int p, int mgs, DevState* __restrict__ st) {
  const int t = threadIdx.x;
  for (int e = t; e < MAXP * MAXP; e += blockDim.x) st->Bk[e] = st->qr_R[e];
  if (mgs)  // A_k from the modified Gram-Schmidt coefficients, symmetric
    for (int e = t; e < MAXP * MAXP; e += blockDim.x) {
      const int r = e / MAXP, c = e % MAXP;
      st->Ak[e] = (r < p && c < p) ? st->qr_M[(r > c ? r : c) * MAXP + (r > c ? c : r)] : 0.0;
    }
  __syncthreads();
  if (t == 0) {
    st->n_explicit += 1;
    st->lcap = st->qr_lcap;
    st->cap_status = BMR_BENCH_EXHAUSTED;
    if (st->qr_error) {
      st->status = BMR_NONFINITE;
      st->reason = REASON_ERROR;
      st->halt = 1;
    } else {
      st->halt = 0;
      st->reason = REASON_NONE;
    }
  }
}

}  // namespace

int colqr_grid(int64_t n) {
  int64_t g = (n + WG - 1) / WG;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename T>
hipError_t launch_colqr(int p, int mode, T* D, const T* Vk, T* bench, int nb, int64_t n, double* part, int n_wg,
                        DevState* st, hipStream_t s, T* ret) {
  if (p < 1 || p > MAXP || nb < 0 || nb > MAXB || n_wg < 1) return hipErrorInvalidValue;
  const int g = colqr_grid(n);
  if (g > n_wg) return hipErrorInvalidValue;  // the partial sums hold n_wg per entry
  auto step = [&](int kind, int l) {
    hipLaunchKernelGGL(k_qr_dots<T>, dim3(g), dim3(WG), 0, s, kind, mode, l, p, (const T*)D, Vk, (const T*)bench,
                       (const T*)ret, nb, n, part, g, (const DevState*)st);
    hipLaunchKernelGGL(k_qr_decide, dim3(1), dim3(WG), 0, s, kind, mode, l, p, nb, (const double*)part, g, st);
  };
  auto apply = [&](int kind, int l) {
    hipLaunchKernelGGL(k_qr_apply<T>, dim3(g), dim3(WG), 0, s, kind, mode, l, p, D, Vk, bench, ret, nb, n,
                       (const DevState*)st);
  };
  // With retained candidates a new block follows the oracle's order:
  // the block's earlier candidates' coefficients by symmetry, then one
  // modified Gram-Schmidt step per band vector (the rest of V_k, then the
  // new block's earlier columns).  Otherwise W - V_k A_k with A_k from the
  // Gram products, then CGS2 within the new block.
  const bool mgs = mode == QR_LOOP && ret != nullptr;
  hipLaunchKernelGGL(k_qr_begin, dim3(1), dim3(WG), 0, s, mode, p, st);
  if (mode == QR_LOOP && !mgs)
    hipLaunchKernelGGL(k_qr_sub<T>, dim3(g), dim3(WG), 0, s, p, D, Vk, n, (const DevState*)st);
  for (int l = 0; l < p; ++l) {
    if (mgs) {
      if (l > 0) apply(ST_SYM, l);
      for (int r = l; r < p; ++r) {
        step(ST_MGSV + r, l);
        apply(ST_MGSV + r, l);
      }
      for (int q = 0; q < l; ++q) {
        step(ST_MGSD + q, l);
        apply(ST_MGSD + q, l);
      }
    } else {
      for (int pass = 0; l > 0 && pass < 2; ++pass) {
        step(ST_CGS, l);
        apply(ST_CGS, l);
      }
    }
    if (ret) {  // the retained candidates, in the order they were kept
      for (int q = 0; q < nb; ++q) {
        step(ST_KEPT + q, l);
        apply(ST_KEPT + q, l);
      }
    }
    step(ST_NORM, l);
    if (ret) apply(ST_SAVE, l);  // a kept candidate is copied before a substitute replaces it
    step(ST_BENCH, l);
    apply(ST_NORM, l);
    if (ret) {  // a substitute is kept out of the retained candidates, then normalised again
      for (int q = 0; q < nb; ++q) {
        step(ST_SUBK + q, l);
        apply(ST_SUBK + q, l);
      }
      step(ST_RENORM, l);
      apply(ST_RENORM, l);
    }
    if (nb > 0) {
      step(ST_BORTH, l);
      apply(ST_BORTH, l);
    }
  }
  if (mode == QR_LOOP) hipLaunchKernelGGL(k_qr_end, dim3(1), dim3(WG), 0, s, p, (int)mgs, st);
  return hipGetLastError();
}

template hipError_t launch_colqr<double>(int, int, double*, const double*, double*, int, int64_t, double*, int,
                                         DevState*, hipStream_t, double*);
template hipError_t launch_colqr<float>(int, int, float*, const float*, float*, int, int64_t, double*, int,
                                        DevState*, hipStream_t, float*);

}  // namespace bmr
