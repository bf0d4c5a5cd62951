// Row-streaming kernels of a block iteration and the column kernels of the
// column-wise QR path.
//
// Pass 2 touches every row once and keeps each row's p values in registers
// (one lane per row; in FP64 the rows travel between HBM and the lanes
// through an LDS tile, so that every load and store instruction covers
// whole cache lines): it finishes the orthogonalisation of the candidates,
//     W' = W - V_k A_k,  V_{k+1} = W' B_k^{-1}          (forward substitution),
// and updates the substitute bench against V_{k+1} (Section 5.1).  The
// search directions of eq. (4.1) and the iterate update of eq. (4.2) are
// applied once per group of s blocks (and at the block where the iteration
// stops): with M_k = V_k C_k + M_{k-1} D_k + M_{k-2} E_k, the group's
// contribution sum_k M_k Z_k to X, and the two search-direction blocks the
// next group starts from, are combinations of the group's Lanczos blocks
// V_{g+1} .. V_{g+s} and of M_g, M_{g-1}, with p x p coefficients that the
// band kernel forms by a backward recurrence.  Per block iteration this
// reads and writes three n x p blocks (W, V_k in, V_{k+1} out) instead of
// six, plus (s + 6) blocks once per group.
// The p x p coefficient blocks come from the band kernel through the device
// state and are staged in LDS once per workgroup, rounded to the storage type
// T (double, or float in the inner solve of the mixed-precision solver, whose
// row arithmetic then runs in FP32); the FP64 flush for p <= 8 reads them
// from the state with scalar loads instead.
#include "bmr_internal.hpp"

namespace bmr {
namespace {

constexpr int WG = 256;

// Wavefronts per SIMD that pass 2 asks the compiler to fit: one lane holds
// several p-wide rows (and a row of the staging tile), and without a bound
// the compiler spends up to 256 registers on them at large p (one wavefront
// per SIMD); the bounds below are the tightest that do not spill.
constexpr int pass2_waves(int p, int esz) {
  return esz == 8 ? (p >= 14 ? 2 : p >= 10 ? 3 : 4) : 4;
}

// Ordering of LDS accesses between the lanes of one wavefront (the LDS
// executes a wavefront's accesses in issue order).
__device__ inline void lane_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wavefront's 64 consecutive p-wide rows (64p elements from src, the first
// `count` of them valid) into one row per lane: load instruction k reads the
// contiguous elements 64k .. 64k+63, so every instruction consumes whole
// cache lines and the loads can carry the non-temporal hint, and the tile
// (rows padded to p+1 elements) turns them into rows in LDS.  One lane per
// row loading its own p values instead issues p loads that each touch a
// strip of the tile's lines: 3.7 against 6.0 TB/s for two such streams in
// and one out, caches cold.
template <int P, typename T>
__device__ __attribute__((always_inline)) inline void rows_in(const T* __restrict__ src, int count, T* tile,
                                                               int lane, T (&x)[P]) {
  T t[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int e = 64 * k + lane;
    t[k] = e < count ? __builtin_nontemporal_load(src + e) : T(0);
  }
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int e = 64 * k + lane;
    tile[(e / P) * (P + 1) + e % P] = t[k];
  }
  lane_sync();
#pragma unroll
  for (int c = 0; c < P; ++c) x[c] = tile[lane * (P + 1) + c];
  lane_sync();
}

// The inverse of rows_in: one row per lane out to 64 consecutive rows.  NT:
// non-temporal stores, for blocks no kernel reads soon; V_{k+1} keeps
// ordinary stores, which leave it in the memory-side cache for the gathers
// of the next pass 1.
template <int P, bool NT, typename T>
__device__ __attribute__((always_inline)) inline void rows_out(T* __restrict__ dst, int count, T* tile, int lane,
                                                                const T (&x)[P]) {
#pragma unroll
  for (int c = 0; c < P; ++c) tile[lane * (P + 1) + c] = x[c];
  lane_sync();
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int e = 64 * k + lane;
    if (e < count) {
      const T y = tile[(e / P) * (P + 1) + e % P];
      if constexpr (NT) {
        __builtin_nontemporal_store(y, dst + e);
      } else {
        dst[e] = y;
      }
    }
  }
  lane_sync();
}

template <int P, typename T>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(pass2_waves(P, sizeof(T))))) void k_pass2(
    T* __restrict__ Vbase, size_t slot, T* __restrict__ bench, int64_t n, const DevState* __restrict__ st) {
  const int64_t k = st->k2;
  if (k == 0) return;
  constexpr int R = ring_len(P);
  __shared__ T sA[P * P], sB[P * P], sBc[MAXB * P];
  for (int e = threadIdx.x; e < P * P; e += WG) {
    const int r = e / P, c = e % P, o = r * MAXP + c;
    sA[e] = (T)st->P2A[o];
    sB[e] = (T)st->P2B[o];
  }
  for (int e = threadIdx.x; e < MAXB * P; e += WG) sBc[e] = (T)st->bcoef[(e / P) * MAXP + (e % P)];
  __syncthreads();
  const int nb = st->nb, taken = st->taken;
  const T* __restrict__ V = Vbase + (size_t)(k % R) * slot;
  T* __restrict__ Wn = Vbase + (size_t)((k + 1) % R) * slot;
  if constexpr (sizeof(T) == 8) {
    __shared__ T stile[WG / 64][64 * (P + 1)];
    const int lane = threadIdx.x & 63;
    T* tile = stile[threadIdx.x >> 6];

    // each wavefront takes 64 consecutive rows per step
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t row0 = (int64_t)blockIdx.x * WG + (threadIdx.x & ~63); row0 < n; row0 += stride) {
      // re-read the coefficients from LDS in every row rather than holding
      // them in registers for the whole loop
      asm volatile("" ::: "memory");
      const int count = (int)((n - row0 < 64 ? n - row0 : 64) * P);
      const int64_t row = row0 + lane;
      T v[P], w[P];
      rows_in<P>(V + row0 * P, count, tile, lane, v);
      rows_in<P>(Wn + row0 * P, count, tile, lane, w);
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
      rows_out<P, false>(Wn + row0 * P, count, tile, lane, w);
      // keep the unused substitutes orthogonal to the new basis vectors
      if (row < n) {
        for (int b = taken; b < nb; ++b) {
          T gv = bench[row * nb + b];
#pragma unroll
          for (int l = 0; l < P; ++l) gv = fma(-w[l], sBc[b * P + l], gv);
          bench[row * nb + b] = gv;
        }
      }
    }
  } else {
    // FP32: one row per lane.  Its rows are half as wide, and the staged form
    // (4-byte elements, twice the instructions) was slower: 40.1 -> 45.8 us
    // at p = 8, against 90.0 -> 76.0 us in FP64.
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x; row < n; row += stride) {
      asm volatile("" ::: "memory");
      T v[P], w[P];
#pragma unroll
      for (int c = 0; c < P; ++c) {
        v[c] = V[row * P + c];
        w[c] = Wn[row * P + c];
      }
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
      for (int b = taken; b < nb; ++b) {
        T gv = bench[row * nb + b];
#pragma unroll
        for (int l = 0; l < P; ++l) gv = fma(-w[l], sBc[b * P + l], gv);
        bench[row * nb + b] = gv;
      }
    }
  }
}

// The search directions of a group of m blocks g+1 .. g+m (g + m = kexp)
// into X, and the two search-direction blocks the next group starts from:
//     X += sum_t V_{g+1+t} Y[0][t] + M_g Y[0][M_g] + M_{g-1} Y[0][M_{g-1}],
//     M_{g+m-1}, M_{g+m} likewise with Y[1], Y[2] (in place of M_{g-1}, M_g).
// One row per lane; each input row is read once and feeds all three outputs.
// The flush holds three p-wide accumulators per lane; for p > 8 it asks for
// three wavefronts per SIMD (unbounded, p = 16 took all 256 registers).
constexpr int flush_waves(int p) { return p <= 8 ? 1 : 3; }

// rows_in for U blocks at once: every load is issued before the first
// transpose, so that a lane has U p-wide rows in flight.
template <int P, int U, typename T>
__device__ __attribute__((always_inline)) inline void rows_in_batch(const T* const (&src)[U], const bool (&use)[U],
                                                                     int count, T* tile, int lane, T (&x)[U][P]) {
  T t[U][P];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int e = 64 * k + lane;
      t[u][k] = (use[u] && e < count) ? __builtin_nontemporal_load(src[u] + e) : T(0);
    }
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int e = 64 * k + lane;
      tile[(e / P) * (P + 1) + e % P] = t[u][k];
    }
    lane_sync();
#pragma unroll
    for (int c = 0; c < P; ++c) x[u][c] = tile[lane * (P + 1) + c];
    lane_sync();
  }
}

// TV: storage type of the Lanczos blocks in the ring; T: that of the search
// directions and X (FP32 blocks with FP64 search directions and X after the
// switch of BMR_PREC_RELAXED).
template <int P, typename T, typename TV = T>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(flush_waves(P)))) void k_flush(
    const TV* __restrict__ Vbase, T* __restrict__ Mbase, size_t slot, T* __restrict__ X, int64_t n, int64_t kexp,
    const DevState* __restrict__ st) {
  if (st->flush_block != kexp || st->flush_len == 0) return;
  constexpr int S = group_len(P), R = ring_len(P);
  const int m = st->flush_len;
  const bool keep_m = st->flush_keep != 0;
  const int64_t g = kexp - m;
  T* __restrict__ Ma = Mbase;         // M_{g-1}, then M_{g+m-1}
  T* __restrict__ Mb = Mbase + slot;  // M_g, then M_{g+m}
  constexpr bool SAME = sizeof(TV) == sizeof(T);
  if constexpr (sizeof(T) == 8 && SAME && P <= 8) {
    // FP64, p <= 8: the rows move through the LDS tile as in pass 2, and the
    // wave-uniform coefficients are read from the state record (scalar
    // loads) rather than staged in LDS, which leaves the tile as the only
    // LDS use and keeps the occupancy.  Two input blocks are in flight.
    __shared__ T stile[WG / 64][64 * (P + 1)];
    const int lane = threadIdx.x & 63;
    T* tile = stile[threadIdx.x >> 6];
    const double* __restrict__ Yg = &st->Y[0][0][0];
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t row0 = (int64_t)blockIdx.x * WG + (threadIdx.x & ~63); row0 < n; row0 += stride) {
      asm volatile("" ::: "memory");
      const int count = (int)((n - row0 < 64 ? n - row0 : 64) * P);
      T acc[3][P];
      rows_in<P>(X + row0 * P, count, tile, lane, acc[0]);
#pragma unroll
      for (int c = 0; c < P; ++c) acc[1][c] = acc[2][c] = T(0);
      constexpr int U = 2;
      for (int i0 = 0; i0 < m + 2; i0 += U) {
        const T* srcs[U];
        bool use[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u;
          use[u] = i < m + 2;
          srcs[u] = (i < m ? Vbase + (size_t)((g + 1 + i) % R) * slot : (i == m ? Mb : Ma)) + row0 * P;
        }
        T x[U][P];
        rows_in_batch<P, U>(srcs, use, count, tile, lane, x);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u;
          if (i < m + 2) {
            const int bs = i < m ? i : MAXS + (i - m);  // block of Y
#pragma unroll
            for (int r = 0; r < P; ++r)
#pragma unroll
              for (int o = 0; o < 3; ++o)
#pragma unroll
                for (int c = 0; c < P; ++c)
                  acc[o][c] = fma(x[u][r], Yg[((size_t)o * (MAXS + 2) + bs) * (MAXP * MAXP) + r * MAXP + c],
                                  acc[o][c]);
          }
        }
      }
      rows_out<P, true>(X + row0 * P, count, tile, lane, acc[0]);
      if (keep_m) {
        rows_out<P, true>(Ma + row0 * P, count, tile, lane, acc[1]);
        rows_out<P, true>(Mb + row0 * P, count, tile, lane, acc[2]);
      }
    }
    return;
  }
  __shared__ T sY[3][S + 2][P * P];  // input blocks: V_{g+1+t} at t < m, M_g at S, M_{g-1} at S + 1
  for (int e = threadIdx.x; e < 3 * (S + 2) * P * P; e += WG) {
    const int o = e / ((S + 2) * P * P), b = (e / (P * P)) % (S + 2), rc = e % (P * P);
    const int src = b < S ? b : MAXS + (b - S);
    sY[o][b][rc] = (b < m || b >= S) ? (T)st->Y[o][src][(rc / P) * MAXP + rc % P] : T(0);
  }
  __syncthreads();
  // FP64 and p > 8: each wavefront's 64 rows of every block move through an
  // LDS tile (coalesced non-temporal loads and stores, as in pass 2): p = 16
  // 0.420 -> 0.395 ms per block iteration with pass 2.  p <= 8: one row per
  // lane; there the tile's LDS would cost a workgroup per CU (3 -> 2) and the
  // staged form was slower (pass 2 + flush 0.114 -> 0.125 ms at p = 8).
  // FP32 keeps one row per lane, as in its pass 2.
  if constexpr (P > 8 && sizeof(T) == 8 && SAME) {
    __shared__ T stile[WG / 64][64 * (P + 1)];
    const int lane = threadIdx.x & 63;
    T* tile = stile[threadIdx.x >> 6];
    // each wavefront takes 64 consecutive rows per step; its rows of every
    // block move through the LDS tile as in pass 2
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t row0 = (int64_t)blockIdx.x * WG + (threadIdx.x & ~63); row0 < n; row0 += stride) {
      asm volatile("" ::: "memory");
      const int count = (int)((n - row0 < 64 ? n - row0 : 64) * P);
      T acc[3][P];
      rows_in<P>(X + row0 * P, count, tile, lane, acc[0]);
#pragma unroll
      for (int c = 0; c < P; ++c) acc[1][c] = acc[2][c] = T(0);
      // inputs i = 0 .. m + 1: V_{g+1+i} (i < m), M_g, M_{g-1}, one block at
      // a time (registers)
      for (int i = 0; i < m + 2; ++i) {
        const T* src = i < m ? Vbase + (size_t)((g + 1 + i) % R) * slot : (i == m ? Mb : Ma);
        T x[P];
        rows_in<P>(src + row0 * P, count, tile, lane, x);
        const int b = i < m ? i : S + (i - m);
#pragma unroll
        for (int r = 0; r < P; ++r)
#pragma unroll
          for (int o = 0; o < 3; ++o)
#pragma unroll
            for (int c = 0; c < P; ++c) acc[o][c] = fma(x[r], sY[o][b][r * P + c], acc[o][c]);
      }
      rows_out<P, true>(X + row0 * P, count, tile, lane, acc[0]);
      if (keep_m) {
        rows_out<P, true>(Ma + row0 * P, count, tile, lane, acc[1]);
        rows_out<P, true>(Mb + row0 * P, count, tile, lane, acc[2]);
      }
    }
  } else {
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x; row < n; row += stride) {
      asm volatile("" ::: "memory");
      T acc[3][P];
#pragma unroll
      for (int c = 0; c < P; ++c) {
        acc[0][c] = X[row * P + c];
        acc[1][c] = acc[2][c] = T(0);
      }
      // inputs i = 0 .. m + 1: V_{g+1+i} (i < m), M_g, M_{g-1}.  For p <= 8
      // the loads of four input rows are issued before their FMAs, so that a
      // lane has several loads in flight (0.71 -> 0.63 ms per group at 128^3,
      // p = 8); at larger p one row at a time keeps the registers in bounds.
      constexpr int U = P <= 8 ? 4 : 1;
      for (int i0 = 0; i0 < m + 2; i0 += U) {
        T x[U][P];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u;
          if (i < m) {
            const TV* __restrict__ src = Vbase + (size_t)((g + 1 + i) % R) * slot;
#pragma unroll
            for (int c = 0; c < P; ++c) x[u][c] = (T)src[row * P + c];
          } else if (i < m + 2) {
            const T* __restrict__ src = i == m ? Mb : Ma;
#pragma unroll
            for (int c = 0; c < P; ++c) x[u][c] = src[row * P + c];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u;
          if (i < m + 2) {
            const int b = i < m ? i : S + (i - m);
#pragma unroll
            for (int r = 0; r < P; ++r)
#pragma unroll
              for (int o = 0; o < 3; ++o)
#pragma unroll
                for (int c = 0; c < P; ++c) acc[o][c] = fma(x[u][r], sY[o][b][r * P + c], acc[o][c]);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < P; ++c) X[row * P + c] = acc[0][c];
      if (keep_m) {
#pragma unroll
        for (int c = 0; c < P; ++c) {
          Ma[row * P + c] = acc[1][c];
          Mb[row * P + c] = acc[2][c];
        }
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
  // wavefront sums by shuffles, then the four wavefronts in order; every
  // index into acc is a constant after unrolling (no scratch)
  __shared__ double sh[WG / 64][MAXP + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r <= MAXP; ++r) {
    if (r < m || r == MAXP) {
      double a = acc[r];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
      if (lane == 0) sh[wave][r] = a;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x <= m) {
    const int r = (int)threadIdx.x < m ? (int)threadIdx.x : MAXP;
    part[(size_t)blockIdx.x * (m + 1) + threadIdx.x] = (sh[0][r] + sh[1][r]) + (sh[2][r] + sh[3][r]);
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
hipError_t launch_pass2(int p, T* Vbase, size_t slot, T* bench, int64_t n, DevState* st, hipStream_t s) {
  const int g = stream_grid(n);
#define L4(P) hipLaunchKernelGGL((k_pass2<P, T>), dim3(g), dim3(WG), 0, s, Vbase, slot, bench, n, st)
  BMR_DISPATCH_P(p, L4)
#undef L4
  return hipGetLastError();
}

template <typename T>
hipError_t launch_flush(int p, const T* Vbase, T* Mbase, size_t slot, T* X, int64_t n, int64_t k, const DevState* st,
                        hipStream_t s) {
  if (!Vbase || !Mbase || !X || !st) return hipErrorInvalidValue;
  const int g = stream_grid(n);
#define L5(P) hipLaunchKernelGGL((k_flush<P, T>), dim3(g), dim3(WG), 0, s, Vbase, Mbase, slot, X, n, k, st)
  BMR_DISPATCH_P(p, L5)
#undef L5
  return hipGetLastError();
}

hipError_t launch_flush_vf(int p, const float* Vbase, double* Mbase, size_t slot, double* X, int64_t n, int64_t k,
                           const DevState* st, hipStream_t s) {
  if (!Vbase || !Mbase || !X || !st) return hipErrorInvalidValue;
  const int g = stream_grid(n);
#define L5(P) \
  hipLaunchKernelGGL((k_flush<P, double, float>), dim3(g), dim3(WG), 0, s, Vbase, Mbase, slot, X, n, k, st)
  BMR_DISPATCH_P(p, L5)
#undef L5
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
  if (!x) return hipErrorInvalidValue;
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

hipError_t launch_to_f32(const double* src, float* dst, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (!src || !dst) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_to_f32, dim3(flat_grid(count)), dim3(WG), 0, s, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_add_f32(double* x, const float* d, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (!x || !d) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_add_f32, dim3(flat_grid(count)), dim3(WG), 0, s, x, d, count);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (!src || !dst) return hipErrorInvalidValue;
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
  template hipError_t launch_pass2<T>(int, T*, size_t, T*, int64_t, DevState*, hipStream_t);                        \
  template hipError_t launch_flush<T>(int, const T*, T*, size_t, T*, int64_t, int64_t, const DevState*, hipStream_t); \
  template hipError_t launch_fill<T>(T*, size_t, T, hipStream_t);                                                  \
  template hipError_t launch_bench_init<T>(T*, int64_t, int, uint64_t, hipStream_t);                               \
  template hipError_t launch_coldots<T>(const T*, int, int, const T*, int, int, int64_t, double*, int, hipStream_t);
BMR_INSTANTIATE(double)
BMR_INSTANTIATE(float)
#undef BMR_INSTANTIATE

}  // namespace bmr
