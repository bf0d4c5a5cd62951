// CSR block operator kernels for gfx950:
//   - pass 1 of a block iteration: W = A V_k - V_{k-1} B_{k-1}^T together with
//     the per-workgroup partial Gram products the band kernel needs,
//   - the plain block product W = A V,
//   - the explicit residual R = B - A X with column norms.
//
// Layout: every n x p block is row-interleaved (element (i, c) at i*p + c), so
// the p values one matrix entry multiplies are one contiguous 8p-byte segment.
// A group of LPR = next_pow2(p) lanes owns one row: lane c holds column c.
// The lanes of a group load up to LPR (column, value) pairs of the row at once
// and pass them round with cross-lane shuffles, so each row of A is read once
// for all p columns.  Workgroups get contiguous row ranges, and the logical
// workgroup id is remapped so that each of the 8 XCDs (whose L2 caches are
// private) walks one contiguous slab of rows: the stencil neighbours of a row
// then sit in the same L2.
#include "bmr_internal.hpp"

namespace bmr {
namespace {

constexpr int WG = 256;

template <int P>
struct Lanes {
  static constexpr int LPR = P <= 1 ? 1 : P <= 2 ? 2 : P <= 4 ? 4 : P <= 8 ? 8 : 16;
  static constexpr int RPW = 64 / LPR;        // rows per wavefront
  static constexpr int RPG = (WG / 64) * RPW; // rows per workgroup step
};

__device__ inline int logical_wg(int n_wg) {
  const int w = blockIdx.x;
  return (w % 8) * (n_wg / 8) + (w / 8);
}

__device__ inline double shfl_d(double x, int src, int width) { return __shfl(x, src, width); }

// acc = sum over the entries of `row` of val * V[col*P + c], in CSR order.
// All LPR lanes of a group call this with the same row and `valid` flag.
template <int P, int LPR>
__device__ inline double gather_row(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                    const double* __restrict__ va, const double* __restrict__ V, int64_t row,
                                    bool valid, int c) {
  int s = 0, e = 0;
  if (valid) {
    s = rp[row];
    e = rp[row + 1];
  }
  double acc = 0.0;
  if constexpr (LPR == 1) {
    for (int q = s; q < e; ++q) acc = fma(va[q], V[(int64_t)ci[q] * P], acc);
  } else {
    for (int base = s; base < e; base += LPR) {
      const int idx = base + c;
      int col = 0;
      double v = 0.0;
      if (idx < e) {
        col = ci[idx];
        v = va[idx];
      }
      const int cnt = min(LPR, e - base);
      for (int q = 0; q < cnt; ++q) {
        const int cq = __shfl(col, q, LPR);
        const double vq = shfl_d(v, q, LPR);
        if (c < P) acc = fma(vq, V[(int64_t)cq * P + c], acc);
      }
    }
  }
  return acc;
}

// Sum x over the groups of a wavefront (lanes with equal c); the result is
// valid in every lane.
template <int LPR>
__device__ inline double group_sum(double x) {
#pragma unroll
  for (int o = LPR; o < 64; o <<= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <int P>
__global__ __launch_bounds__(WG) void k_pass1(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                              const double* __restrict__ va, int64_t n, double* __restrict__ Vbase,
                                              size_t slot, const double* __restrict__ bench,
                                              double* __restrict__ part, int n_wg, DevState* __restrict__ st) {
  if (st->halt) return;
  constexpr int LPR = Lanes<P>::LPR, RPW = Lanes<P>::RPW, RPG = Lanes<P>::RPG;
  const int64_t k = st->k;
  const double* __restrict__ V = Vbase + (size_t)(k % 3) * slot;
  const double* __restrict__ Vp = Vbase + (size_t)((k + 2) % 3) * slot;  // V_{k-1}
  double* __restrict__ W = Vbase + (size_t)((k + 1) % 3) * slot;         // becomes V_{k+1}
  const int nb = st->nb, taken = st->taken;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / LPR, c = lane % LPR;

  double bp[P];  // row c of B_{k-1}
#pragma unroll
  for (int r = 0; r < P; ++r) bp[r] = (c < P) ? st->Bprev[c * MAXP + r] : 0.0;

  double aG[P], aQ[P], aP[P], aA = 0.0, aWg[MAXB], aVg[MAXB], aGg[MAXB * MAXB];
#pragma unroll
  for (int r = 0; r < P; ++r) aG[r] = aQ[r] = aP[r] = 0.0;
#pragma unroll
  for (int b = 0; b < MAXB; ++b) aWg[b] = aVg[b] = 0.0;
#pragma unroll
  for (int b = 0; b < MAXB * MAXB; ++b) aGg[b] = 0.0;

  const int L = logical_wg(n_wg);
  const int64_t chunk = ((n + n_wg - 1) / n_wg + RPG - 1) / RPG * RPG;
  const int64_t r0 = (int64_t)L * chunk;
  const int64_t r1 = min(n, r0 + chunk);

  for (int64_t base = r0; base < r1; base += RPG) {
    const int64_t row = base + wave * RPW + grp;
    const bool valid = row < r1;
    const double a = gather_row<P, LPR>(rp, ci, va, V, row, valid, c);
    double v = 0.0, vp = 0.0;
    if (valid && c < P) {
      v = V[row * P + c];
      vp = Vp[row * P + c];
    }
    // known coefficients by symmetry: column c loses sum_{r >= c} B_{k-1}(c, r) V_{k-1}(:, r)
    double w = a;
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const double vr = shfl_d(vp, r, LPR);
      if (r >= c) w = fma(-bp[r], vr, w);
    }
    if (valid && c < P) W[row * P + c] = w;
    aA = fma(a, a, aA);
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const double vr = shfl_d(v, r, LPR);
      const double wr = shfl_d(w, r, LPR);
      aG[r] = fma(vr, w, aG[r]);
      aQ[r] = fma(wr, w, aQ[r]);
      aP[r] = fma(vr, v, aP[r]);
    }
    if (taken < nb) {
      double g[MAXB];
#pragma unroll
      for (int b = 0; b < MAXB; ++b) g[b] = (b >= taken && b < nb && valid) ? bench[row * nb + b] : 0.0;
#pragma unroll
      for (int b = 0; b < MAXB; ++b) {
        aWg[b] = fma(w, g[b], aWg[b]);
        aVg[b] = fma(v, g[b], aVg[b]);
      }
      if (c == 0) {
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
#pragma unroll
          for (int b2 = 0; b2 < MAXB; ++b2) aGg[b * MAXB + b2] = fma(g[b], g[b2], aGg[b * MAXB + b2]);
      }
    }
  }

  // ---- workgroup reduction: deterministic order --------------------------
  constexpr int NEMAX = n_entries(MAXP, MAXB);
  __shared__ double sred[WG / 64][NEMAX];
  const int ne = n_entries(P, nb);
#pragma unroll
  for (int r = 0; r < P; ++r) {
    aG[r] = group_sum<LPR>(aG[r]);
    aQ[r] = group_sum<LPR>(aQ[r]);
    aP[r] = group_sum<LPR>(aP[r]);
  }
  aA = group_sum<LPR>(aA);
  if (taken < nb) {
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      aWg[b] = group_sum<LPR>(aWg[b]);
      aVg[b] = group_sum<LPR>(aVg[b]);
    }
#pragma unroll
    for (int b = 0; b < MAXB * MAXB; ++b) aGg[b] = group_sum<LPR>(aGg[b]);
  }
  if (grp == 0 && c < P) {
    double* s = sred[wave];
#pragma unroll
    for (int r = 0; r < P; ++r) {
      s[off_G(P) + r * P + c] = aG[r];
      s[off_Q(P) + r * P + c] = aQ[r];
      s[off_P(P) + r * P + c] = aP[r];
    }
    s[off_a(P) + c] = aA;
    for (int b = 0; b < nb; ++b) {
      s[off_Wg(P) + c * nb + b] = aWg[b];
      s[off_Vg(P, nb) + c * nb + b] = aVg[b];
    }
    if (c == 0)
      for (int b = 0; b < nb; ++b)
        for (int b2 = 0; b2 < nb; ++b2) s[off_gg(P, nb) + b * nb + b2] = aGg[b * MAXB + b2];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ne; e += WG) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < WG / 64; ++q) t += sred[q][e];
    part[(size_t)e * n_wg + L] = t;
  }
}

template <int P>
__global__ __launch_bounds__(WG) void k_spmm(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                             const double* __restrict__ va, int64_t n, const double* __restrict__ V,
                                             double* __restrict__ W, int n_wg) {
  constexpr int LPR = Lanes<P>::LPR, RPW = Lanes<P>::RPW, RPG = Lanes<P>::RPG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / LPR, c = lane % LPR;
  const int L = logical_wg(n_wg);
  const int64_t chunk = ((n + n_wg - 1) / n_wg + RPG - 1) / RPG * RPG;
  const int64_t r0 = (int64_t)L * chunk;
  const int64_t r1 = min(n, r0 + chunk);
  for (int64_t base = r0; base < r1; base += RPG) {
    const int64_t row = base + wave * RPW + grp;
    const bool valid = row < r1;
    const double a = gather_row<P, LPR>(rp, ci, va, V, row, valid, c);
    if (valid && c < P) W[row * P + c] = a;
  }
}

template <int P>
__global__ __launch_bounds__(WG) void k_residual(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const double* __restrict__ va, int64_t n,
                                                 const double* __restrict__ Bm, const double* __restrict__ X,
                                                 double* __restrict__ R, double* __restrict__ part, int n_wg) {
  constexpr int LPR = Lanes<P>::LPR, RPW = Lanes<P>::RPW, RPG = Lanes<P>::RPG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / LPR, c = lane % LPR;
  const int L = logical_wg(n_wg);
  const int64_t chunk = ((n + n_wg - 1) / n_wg + RPG - 1) / RPG * RPG;
  const int64_t r0 = (int64_t)L * chunk;
  const int64_t r1 = min(n, r0 + chunk);
  double acc = 0.0;
  for (int64_t base = r0; base < r1; base += RPG) {
    const int64_t row = base + wave * RPW + grp;
    const bool valid = row < r1;
    const double ax = gather_row<P, LPR>(rp, ci, va, X, row, valid, c);
    if (valid && c < P) {
      const double r = Bm[row * P + c] - ax;
      if (R) R[row * P + c] = r;
      acc = fma(r, r, acc);
    }
  }
  acc = group_sum<LPR>(acc);
  __shared__ double s[WG / 64][LPR];
  if (grp == 0) s[wave][c] = acc;
  __syncthreads();
  if (threadIdx.x < P) {
    double t = 0.0;
    for (int q = 0; q < WG / 64; ++q) t += s[q][threadIdx.x];
    part[(size_t)threadIdx.x * n_wg + L] = t;
  }
}

}  // namespace

int pass1_grid(int64_t n, int p) {
  const int lpr = p <= 1 ? 1 : p <= 2 ? 2 : p <= 4 ? 4 : p <= 8 ? 8 : 16;
  const int64_t rpg = (WG / 64) * (64 / lpr);
  const int64_t steps = (n + rpg - 1) / rpg;
  int64_t g = (steps + 3) / 4;  // at least ~4 steps per workgroup when large
  if (g > 2048) g = 2048;
  if (g < 8) g = 8;
  return (int)((g + 7) / 8 * 8);
}

#define BMR_DISPATCH_P(p, MACRO) \
  switch (p) {                   \
    case 1: MACRO(1); break;     \
    case 2: MACRO(2); break;     \
    case 3: MACRO(3); break;     \
    case 4: MACRO(4); break;     \
    case 5: MACRO(5); break;     \
    case 6: MACRO(6); break;     \
    case 7: MACRO(7); break;     \
    case 8: MACRO(8); break;     \
    case 9: MACRO(9); break;     \
    case 10: MACRO(10); break;   \
    case 11: MACRO(11); break;   \
    case 12: MACRO(12); break;   \
    case 13: MACRO(13); break;   \
    case 14: MACRO(14); break;   \
    case 15: MACRO(15); break;   \
    case 16: MACRO(16); break;   \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_pass1(int p, const bmr_csr_t& A, double* Vbase, size_t slot, double* bench, double* part, int n_wg,
                        DevState* st, hipStream_t s) {
#define L1(P)                                                                                         \
  hipLaunchKernelGGL(k_pass1<P>, dim3(n_wg), dim3(WG), 0, s, A.row_ptr, A.col_idx, A.val, A.n, Vbase, \
                     slot, bench, part, n_wg, st)
  BMR_DISPATCH_P(p, L1)
#undef L1
  return hipGetLastError();
}

hipError_t launch_spmm(int p, const bmr_csr_t& A, const double* V, double* W, hipStream_t s) {
  const int n_wg = pass1_grid(A.n, p);
#define L2(P) hipLaunchKernelGGL(k_spmm<P>, dim3(n_wg), dim3(WG), 0, s, A.row_ptr, A.col_idx, A.val, A.n, V, W, n_wg)
  BMR_DISPATCH_P(p, L2)
#undef L2
  return hipGetLastError();
}

hipError_t launch_residual(int p, const bmr_csr_t& A, const double* Bm, const double* X, double* R, double* part,
                           int n_wg, hipStream_t s) {
#define L3(P)                                                                                                  \
  hipLaunchKernelGGL(k_residual<P>, dim3(n_wg), dim3(WG), 0, s, A.row_ptr, A.col_idx, A.val, A.n, Bm, X, R, \
                     part, n_wg)
  BMR_DISPATCH_P(p, L3)
#undef L3
  return hipGetLastError();
}

}  // namespace bmr
