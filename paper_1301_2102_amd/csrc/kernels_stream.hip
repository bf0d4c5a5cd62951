// Row-streaming kernels of a block iteration and the column kernels of the
// column-wise QR path.
//
// Pass 2 touches every row once and keeps each row's p values in registers
// (one lane per row): it finishes the orthogonalisation of the candidates,
//     W' = W - V_k A_k,  V_{k+1} = W' B_k^{-1}          (forward substitution),
// updates the substitute bench against V_{k+1} (Section 5.1), forms the
// search directions of the block (eq. (4.1)),
//     M_k = (V_k - M_{k-2} R_a - M_{k-1} R_b) R_c^{-1},
// and adds them to the iterate (eq. (4.2)), X += M_k(:, 1:l*) Z_k(1:l*, :).
// The iterate is updated once per group of three blocks (k = 3, 6, 9, ...,
// and at the block where the iteration stops): pass 2 of block k reads
// M_{k-2} and M_{k-1} for the recurrence anyway, so it adds the pending
// products M_{k-2} Z_{k-2} and M_{k-1} Z_{k-1} before M_k Z_k in the same
// order as block-by-block updates would (the stored X is exact), and X is
// read and written a third as often.
// Every per-row operation runs in the order of the one-vector-per-iteration
// algorithm, so that only the inner products differ in rounding.
// The p x p coefficient blocks come from the band kernel through the device
// state and are staged in LDS once per workgroup, rounded to the storage type
// T (double, or float in the inner solve of the mixed-precision solver, whose
// row arithmetic then runs in FP32).
#include "bmr_internal.hpp"

namespace bmr {
namespace {

constexpr int WG = 256;

// Wavefronts per SIMD that pass 2 asks the compiler to fit: one lane holds
// several p-wide rows, and without a bound the compiler spends up to 256
// registers on them at large p (one wavefront per SIMD).
constexpr int pass2_waves(int p, int esz) { return p <= 8 ? 1 : (esz == 8 && p >= 12 ? 3 : 4); }

template <int P, typename T>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(pass2_waves(P, sizeof(T))))) void k_pass2(T* __restrict__ Vbase, T* __restrict__ Mbase, size_t slot,
                                              T* __restrict__ X, T* __restrict__ bench, int64_t n,
                                              const DevState* __restrict__ st) {
  const int64_t k = st->k2;
  if (k == 0) return;
  // X is updated at the last block of each group of three and at the block
  // where the iteration stops; f0 is the first block of the group.
  const bool finishing = st->reason == REASON_FINISHED;
  const bool upd_x = finishing || (k % 3 == 0);
  const int64_t f0 = k - (k - 1) % 3;
  __shared__ T sA[P * P], sB[P * P], sRa[P * P], sRb[P * P], sRc[P * P], sBc[MAXB * P];
  __shared__ T sZ[3][P * P];  // Z of blocks k-2, k-1, k
  for (int e = threadIdx.x; e < P * P; e += WG) {
    const int r = e / P, c = e % P, o = r * MAXP + c;
    sA[e] = (T)st->P2A[o];
    sB[e] = (T)st->P2B[o];
    sRa[e] = (T)st->Ra[o];
    sRb[e] = (T)st->Rb[o];
    sRc[e] = (T)st->Rc[o];
    for (int d = 0; d < 3; ++d) sZ[d][e] = (T)st->Z[(k + 1 + d) % 3][o];
  }
  for (int e = threadIdx.x; e < MAXB * P; e += WG) sBc[e] = (T)st->bcoef[(e / P) * MAXP + (e % P)];
  __syncthreads();
  const int lstar = st->lstar, nb = st->nb, taken = st->taken;
  const T* __restrict__ V = Vbase + (size_t)(k % 3) * slot;
  T* __restrict__ Wn = Vbase + (size_t)((k + 1) % 3) * slot;
  const T* __restrict__ Mm2 = Mbase + (size_t)((k + 1) % 3) * slot;  // M_{k-2}
  const T* __restrict__ Mm1 = Mbase + (size_t)((k + 2) % 3) * slot;  // M_{k-1}
  T* __restrict__ Mk = Mbase + (size_t)(k % 3) * slot;

  const int64_t stride = (int64_t)gridDim.x * WG;
  for (int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x; row < n; row += stride) {
    // re-read the coefficients from LDS in every row rather than holding
    // 6p^2 of them in registers for the whole loop
    asm volatile("" ::: "memory");
    T v[P], w[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
      v[c] = V[row * P + c];
      w[c] = Wn[row * P + c];
    }
    // finish the band orthogonalisation: column l loses sum_r A_k(r, l) u_r,
    // then the earlier new vectors of its own block
#pragma unroll
    for (int l = 0; l < P; ++l) {
#pragma unroll
      for (int r = 0; r < P; ++r) w[l] = fma(-v[r], sA[r * P + l], w[l]);
    }
#pragma unroll
    for (int l = 0; l < P; ++l) {
#pragma unroll
      for (int r = 0; r < l; ++r) w[l] = fma(-w[r], sB[r * P + l], w[l]);
      w[l] = w[l] / sB[l * P + l];
    }
#pragma unroll
    for (int c = 0; c < P; ++c) Wn[row * P + c] = w[c];
    // keep the unused substitutes orthogonal to the new basis vectors
    for (int b = taken; b < nb; ++b) {
      T g = bench[row * nb + b];
#pragma unroll
      for (int l = 0; l < P; ++l) g = fma(-w[l], sBc[b * P + l], g);
      bench[row * nb + b] = g;
    }
    asm volatile("" ::: "memory");
    // search directions of the block
    T mk[P], m2[P], m1[P];
    {
#pragma unroll
      for (int c = 0; c < P; ++c) {
        m2[c] = Mm2[row * P + c];
        m1[c] = Mm1[row * P + c];
        mk[c] = T(0);
      }
#pragma unroll
      for (int l = 0; l < P; ++l) {
        if (l < lstar) {
          T m = v[l];
#pragma unroll
          for (int r = 0; r < P; ++r)
            if (r >= l) m = fma(-sRa[r * P + l], m2[r], m);
#pragma unroll
          for (int r = 0; r < P; ++r) m = fma(-sRb[r * P + l], m1[r], m);
#pragma unroll
          for (int r = 0; r < l; ++r) m = fma(-sRc[r * P + l], mk[r], m);
          mk[l] = m / sRc[l * P + l];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < P; ++c) Mk[row * P + c] = mk[c];
    asm volatile("" ::: "memory");
    // progressive update of the iterate: the pending blocks of the group,
    // oldest first (M_{k-2}, M_{k-1} are complete blocks, M_k has l* columns)
    if (upd_x) {
      // for p > 8 a few columns at a time, so that the row of X does not
      // sit in registers next to the three rows of M
      constexpr int XC = P <= 8 ? P : (P % 4 == 0 ? 4 : (P % 2 == 0 ? 2 : 1));
#pragma unroll
      for (int c0 = 0; c0 < P; c0 += XC) {
        T x[XC];
#pragma unroll
        for (int c = 0; c < XC; ++c) x[c] = X[row * P + c0 + c];
        if (f0 <= k - 2) {
#pragma unroll
          for (int l = 0; l < P; ++l)
#pragma unroll
            for (int c = 0; c < XC; ++c) x[c] = fma(m2[l], sZ[0][l * P + c0 + c], x[c]);
        }
        if (f0 <= k - 1) {
#pragma unroll
          for (int l = 0; l < P; ++l)
#pragma unroll
            for (int c = 0; c < XC; ++c) x[c] = fma(m1[l], sZ[1][l * P + c0 + c], x[c]);
        }
#pragma unroll
        for (int l = 0; l < P; ++l) {
          if (l < lstar) {
#pragma unroll
            for (int c = 0; c < XC; ++c) x[c] = fma(mk[l], sZ[2][l * P + c0 + c], x[c]);
          }
        }
#pragma unroll
        for (int c = 0; c < XC; ++c) X[row * P + c0 + c] = x[c];
      }
    }
  }
}

template <typename T>
__global__ void k_fill(T* __restrict__ x, size_t count, T v) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) x[i] = v;
}

// SplitMix64 (S. Vigna's public-domain reference): the (c+1)-th output of the
// stream seeded with `seed` is mix(seed + (c+1) * golden).  Entry i of bench
// vector b uses counter c = b*n + i; the top 53 bits map to [-1, 1).
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void k_bench_init(T* __restrict__ bench, int64_t n, int nb, uint64_t seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    for (int b = 0; b < nb; ++b) {
      const uint64_t bits = splitmix64_at(seed, (uint64_t)b * (uint64_t)n + (uint64_t)i) >> 11;
      bench[i * nb + b] = (T)(2.0 * ((double)bits * 0x1.0p-53) - 1.0);
    }
}

// part[wg*(m+1) + r] = sum_i X[i*ldx + r] * Y[i*ldy + yc] (r < m); part[wg*(m+1) + m] = sum_i Y^2
// (products and sums in FP64 for both storage types)
template <typename T>
__global__ __launch_bounds__(WG) void k_coldots(const T* Y, int ldy, int yc, const T* X, int ldx, int m, int64_t n,
                                                double* __restrict__ part) {
  double acc[MAXP + 1];
#pragma unroll
  for (int r = 0; r <= MAXP; ++r) acc[r] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * WG;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
    const double y = Y[i * ldy + yc];
#pragma unroll
    for (int r = 0; r < MAXP; ++r)
      if (r < m) acc[r] = fma((double)X[i * ldx + r], y, acc[r]);
    acc[MAXP] = fma(y, y, acc[MAXP]);
  }
  __shared__ double sh[WG];
  for (int r = 0; r <= m; ++r) {
    const double a = (r < m) ? acc[r] : acc[MAXP];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * (m + 1) + r] = sh[0];
    __syncthreads();
  }
}

// D[i*ldd + dc] = (S[i*lds + sc] - sum_{r<m} coef[r] * X[i*ldx + r]) / div,
// evaluated in FP64 and rounded to T once.  D may be the same column as S (in
// place) and X may be other columns of the same block, so none of the
// pointers is restrict-qualified.
template <typename T>
__global__ void k_colop(T* D, int ldd, int dc, const T* S, int lds, int sc, const T* X, int ldx, int m, ColCoef coef,
                        double div, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double y = S[i * lds + sc];
    for (int r = 0; r < m; ++r) y = fma(-coef.c[r], (double)X[i * ldx + r], y);
    D[i * ldd + dc] = (T)(y / div);
  }
}

// dst[i] = src[i] rounded to float (round to nearest even)
__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = (float)src[i];
}

// x[i] += d[i] in FP64 (the refinement step X += D of the mixed-precision solver)
__global__ void k_add_f32(double* __restrict__ x, const float* __restrict__ d, size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) x[i] += (double)d[i];
}

// Gradient of a loss of X = A^{-1} B with respect to the stored entries of A,
// symmetrised: for entry e = (i, j), g_e = -(Lam_i . X_j + Lam_j . X_i) / 2,
// with Lam the adjoint solution.  One lane per row i; its own rows of Lam and
// X stay in registers, the rows j of its entries are gathered.
template <int P>
__global__ __launch_bounds__(WG) void k_pattern_grad(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                     const double* __restrict__ Lam, const double* __restrict__ X,
                                                     double* __restrict__ g, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * WG;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
    double li[P], xi[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
      li[c] = Lam[i * P + c];
      xi[c] = X[i * P + c];
    }
    const int s = rp[i], e = rp[i + 1];
    for (int q = s; q < e; ++q) {
      const int64_t j = ci[q];
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        a = fma(li[c], X[j * P + c], a);
        b = fma(Lam[j * P + c], xi[c], b);
      }
      g[q] = -0.5 * (a + b);
    }
  }
}

// dst[i] = src[i] (FP64 block copy)
__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = src[i];
}

}  // namespace

int coldots_grid(int64_t n) {
  int64_t g = (n + WG - 1) / WG;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (int)g;
}

static int stream_grid(int64_t n) {
  int64_t g = (n + WG - 1) / WG;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
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

template <typename T>
hipError_t launch_pass2(int p, T* Vbase, T* Mbase, size_t slot, T* X, T* bench, int64_t n, DevState* st,
                        hipStream_t s) {
  const int g = stream_grid(n);
#define L4(P) hipLaunchKernelGGL((k_pass2<P, T>), dim3(g), dim3(WG), 0, s, Vbase, Mbase, slot, X, bench, n, st)
  BMR_DISPATCH_P(p, L4)
#undef L4
  return hipGetLastError();
}

static unsigned flat_grid(size_t count) {
  size_t g = (count + WG - 1) / WG;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T>
hipError_t launch_fill(T* x, size_t count, T v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<T>, dim3(flat_grid(count)), dim3(WG), 0, s, x, count, v);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bench_init(T* bench, int64_t n, int nb, uint64_t seed, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bench_init<T>, dim3(stream_grid(n)), dim3(WG), 0, s, bench, n, nb, seed);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coldots(const T* Y, int ldy, int yc, const T* X, int ldx, int m, int64_t n, double* part, int n_wg,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_coldots<T>, dim3(n_wg), dim3(WG), 0, s, Y, ldy, yc, X, ldx, m, n, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_colop(T* D, int ldd, int dc, const T* S, int lds, int sc, const T* X, int ldx, int m, ColCoef coef,
                        double div, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_colop<T>, dim3(stream_grid(n)), dim3(WG), 0, s, D, ldd, dc, S, lds, sc, X, ldx, m, coef, div,
                     n);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3(flat_grid(count)), dim3(WG), 0, s, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_add_f32(double* x, const float* d, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_f32, dim3(flat_grid(count)), dim3(WG), 0, s, x, d, count);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(flat_grid(count)), dim3(WG), 0, s, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_pattern_grad(int p, const bmr_csr_t& A, const double* Lam, const double* X, double* g,
                               hipStream_t s) {
  const int grid = stream_grid(A.n);
#define L5(P) \
  hipLaunchKernelGGL(k_pattern_grad<P>, dim3(grid), dim3(WG), 0, s, A.row_ptr, A.col_idx, Lam, X, g, A.n)
  BMR_DISPATCH_P(p, L5)
#undef L5
  return hipGetLastError();
}

#define BMR_INSTANTIATE(T)                                                                                          \
  template hipError_t launch_pass2<T>(int, T*, T*, size_t, T*, T*, int64_t, DevState*, hipStream_t);               \
  template hipError_t launch_fill<T>(T*, size_t, T, hipStream_t);                                                  \
  template hipError_t launch_bench_init<T>(T*, int64_t, int, uint64_t, hipStream_t);                               \
  template hipError_t launch_coldots<T>(const T*, int, int, const T*, int, int, int64_t, double*, int, hipStream_t); \
  template hipError_t launch_colop<T>(T*, int, int, const T*, int, int, const T*, int, int, ColCoef, double, int64_t, \
                                      hipStream_t);
BMR_INSTANTIATE(double)
BMR_INSTANTIATE(float)
#undef BMR_INSTANTIATE

}  // namespace bmr
