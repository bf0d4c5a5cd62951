// Reduction of the pass-1 partial sums and the band kernel: one workgroup of
// two wavefronts that turns the p x p Gram products of a block iteration into the new block
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
//
// Work split: lane l owns column l of the block (its 4p band entries, kept
// in LDS, with a window of p+1 of them in registers) and column l of the
// S-hat window.  A second wavefront applies the rotations of the two
// previous blocks while the first is in phase A; the p rotations of each
// column of the block are generated together (lane t makes rotation t from a
// prefix sum of squares) and applied by the lanes owning the columns to its
// right.
#include <math.h>

#include "bmr_internal.hpp"

namespace bmr {
namespace {

// One wavefront per entry: each lane keeps four partial sums, with up to
// sixteen loads in flight, then the wavefront adds its lanes by shuffles.
// The order of the additions is fixed, so the result is reproducible.
__global__ __launch_bounds__(64) void k_reduce(const double* __restrict__ part, int n_wg, double* __restrict__ red,
                                               DevState* __restrict__ st, int check_halt) {
  if (check_halt && st->halt) return;
  const int e = blockIdx.x;
  const double* src = part + (size_t)e * n_wg;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = threadIdx.x;
#pragma unroll 4
  for (; i + 192 < n_wg; i += 256) {
    s0 += src[i];
    s1 += src[i + 64];
    s2 += src[i + 128];
    s3 += src[i + 192];
  }
  for (; i < n_wg; i += 64) s0 += src[i];
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) red[e] = s;
}

// Most of the band kernel runs on one wavefront.  Its barriers there only
// have to order LDS accesses between the lanes of that wavefront, which the
// LDS executes in issue order; __syncthreads() would add a workgroup-scope
// fence, which waits for every outstanding global store (the R rows, Z, the
// residuals and the history written as the loop goes) on each call.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Barrier of the band kernel's two wavefronts that orders their LDS accesses
// only: the global stores still in flight are not waited for.
__device__ inline void wg_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Givens rotation of the pair (x, y).  In a sweep x passes through p
// rotations in a row, so the products with y are formed first and x enters
// each result through a single fused multiply-add.
__device__ inline void rotate(double c, double s, double& x, double& y) {
  const double a = x, b = y;
  x = fma(c, a, s * b);
  y = fma(-s, a, c * b);
}

// Cross-lane moves inside a row of 16 lanes by DPP, which reads the other
// lane's register directly instead of going through the LDS.  Controls:
// 0xB1 and 0x4E swap neighbours at distance 1 and 2 inside each group of 4,
// 0x141 mirrors each half row, 0x140 the row, 0x110 + o shifts the row
// right by o (lanes below o receive 0).
template <int CTRL>
__device__ inline int dpp_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ inline double dpp_double(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_int<CTRL>((int)b), hi = dpp_int<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// largest value over the 16 lanes of each row, in every lane of the row
__device__ inline double row_max(double v) {
  v = fmax(v, dpp_double<0xB1>(v));
  v = fmax(v, dpp_double<0x4E>(v));
  v = fmax(v, dpp_double<0x141>(v));
  return fmax(v, dpp_double<0x140>(v));
}

// the value of lane (l - o) of the same row in lane l, 0 where l - o falls
// outside it; o is a constant power of two below 16 after unrolling
template <typename T>
__device__ inline T row_shr(T v, int o) {
  if constexpr (sizeof(T) == 8) {
    switch (o) {
      case 1: return dpp_double<0x111>(v);
      case 2: return dpp_double<0x112>(v);
      case 4: return dpp_double<0x114>(v);
      default: return dpp_double<0x118>(v);
    }
  } else {
    switch (o) {
      case 1: return dpp_int<0x111>(v);
      case 2: return dpp_int<0x112>(v);
      case 4: return dpp_int<0x114>(v);
      default: return dpp_int<0x118>(v);
    }
  }
}

// lane l's value, the same in every lane
__device__ inline double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ void halt_with(DevState* st, int status, int reason) {
  st->status = status;
  st->reason = reason;
  st->halt = 1;
  st->k2 = 0;
}

template <int P>
struct BandShared {
  double Ak[P][P], Bk[P][P], Bp[P][P];
  union {
    struct {  // phase A
      double G[P * P], Q[P * P], Pm[P * P];
      double T1[P][P], T2[P][P], Gam[P][P];
    };
    struct {  // phase B: R rows of blocks k-2, k-1, k in the block's columns, Z_k, C, D, E
      double Ra[P][P], Rb[P][P], Rc[P][P], Zk[P][P], C[P][P], D[P][P], E[P][P];
      double Tr[3][3][P][P];                 // backward recurrences of the three outputs (ring of 3)
      double gs[4][group_len(P)][P][P];      // the group's C, D, E, Z at the flush
    };
  };
  double araw[P], beta[P];
  double Wg[P * MAXB], Vg[P * MAXB];  // W^T g_b and V_k^T g_b (bench inner products)
  double rot[2][P][P][2];  // rotations of blocks k-2 and k-1
  double nrot[P][P][2];    // rotations of block k
  double Qb[2][2 * P][2 * P + 1];  // accumulated rotations of blocks k-2 and k-1 (accumulating mode)
  double col[P][4 * P + 1];  // column l of H-bar, rows of blocks k-2 .. k+1
  double s2[P][2 * P + 1];   // column q of the S-hat window (p live + p new rows)
};

// Scalars of the state the band kernel reads, loaded once at its start.
struct BandCtl {
  int64_t k, j0, max_iter, hist_cap;
  int halt, lcap, cap_status, taken;
  double tol, tau_fb;
  bool force_qr;  // a retained candidate still applies to the new block's basis vectors
};

// Every global input of the band kernel, loaded into registers before the
// first of them is used.  A single wavefront would otherwise wait for each
// load in turn, and, since loads and stores share one counter, for every
// store issued before it.  The rotations of all three ring slots are read so
// that no load waits for k.
template <int P>
struct BandLoads {
  static constexpr int N = (P * P + 63) / 64;      // entries of a p x p matrix per lane
  static constexpr int NW = (P * MAXB + 63) / 64;  // entries of W^T g (or V^T g) per lane
  double bprev[N], rot[3][2][N], shat[N], m0[N], m1[N], m2[N], wg[NW], vg[NW];
  double a, beta;
};

template <int P>
__device__ __attribute__((always_inline)) inline void load_band(int mode, int nb, const double* __restrict__ red, const DevState* __restrict__ st,
                                 BandCtl& c, BandLoads<P>& L) {
  using BL = BandLoads<P>;
  const int tid = threadIdx.x;
  c.halt = st->halt;
  c.k = st->k;
  c.j0 = st->j;
  c.max_iter = st->max_iter;
  c.hist_cap = st->hist_cap;
  c.lcap = st->lcap;
  c.cap_status = st->cap_status;
  c.taken = st->taken;
  c.tol = st->tol;
  c.tau_fb = st->tau_fb;
  // the new block holds u_{kp+1} .. u_{kp+p}; a candidate kept in place of
  // u_m applies to u_{m+1} .. u_{m+2p}
  c.force_qr = false;
  for (int q = 0; q < st->n_kept; ++q) c.force_qr |= st->kept_m[q] + 2 * P >= c.k * P + 1;
#pragma unroll
  for (int x = 0; x < BL::N; ++x) {
    const int e = tid + 64 * x;
    const bool ok = e < P * P;
    const int r = ok ? e / P : 0, cc = ok ? e % P : 0, o = r * MAXP + cc;
    L.bprev[x] = ok ? st->Bprev[o] : 0.0;
    L.shat[x] = ok ? st->Shat[o] : 0.0;
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      L.rot[sl][0][x] = ok ? st->rot[sl][r][cc][0] : 1.0;
      L.rot[sl][1][x] = ok ? st->rot[sl][r][cc][1] : 0.0;
    }
    if (mode == 0) {  // Gram products of pass 1
      const int ei = ok ? e : 0;
      L.m0[x] = ok ? red[off_G(P) + ei] : 0.0;
      L.m1[x] = ok ? red[off_Q(P) + ei] : 0.0;
      L.m2[x] = ok ? red[off_P(P) + ei] : 0.0;
    } else {  // A_k and B_k from the column-wise QR
      L.m0[x] = ok ? st->Ak[o] : 0.0;
      L.m1[x] = ok ? st->Bk[o] : 0.0;
      L.m2[x] = 0.0;
    }
  }
#pragma unroll
  for (int x = 0; x < BL::NW; ++x) {
    const int e = tid + 64 * x;
    const bool ok = mode == 0 && e < P * nb;
    const int ei = ok ? e : 0;
    L.wg[x] = ok ? red[off_Wg(P) + ei] : 0.0;
    L.vg[x] = ok ? red[off_Vg(P, nb) + ei] : 0.0;
  }
  const int lane = tid < P ? tid : 0;
  L.a = (mode == 0 && tid < P) ? red[off_a(P) + lane] : 0.0;
  L.beta = tid < P ? st->beta[lane] : 0.0;
}

// Phase A: A_k (phase_a_ak), then the Gram of the remainder, Cholesky ->
// B_k, bench coefficients (phase_a).  Returns false (the same in every lane)
// when the column-wise QR must take over.  Leaves A_k and B_k in shared
// memory.
template <int P>
__device__ void phase_a_ak(BandShared<P>& sh) {
  const int tid = threadIdx.x;
  for (int e = tid; e < P * P; e += 64) {
    const int r = e / P, c = e % P;
    sh.Ak[r][c] = (r >= c) ? sh.G[r * P + c] : sh.G[c * P + r];
  }
  wave_sync();
}

template <int P>
__device__ bool phase_a(int nb, int taken, double tau_fb, DevState* __restrict__ st, BandShared<P>& sh) {
  const int tid = threadIdx.x;
  for (int e = tid; e < P * P; e += 64) {
    const int l = e / P, m = e % P;
    double t = 0.0, u = 0.0;
    for (int r = 0; r < P; ++r) {
      t += sh.Ak[r][l] * sh.G[r * P + m];
      u += sh.Pm[l * P + r] * sh.Ak[r][m];
    }
    sh.T1[l][m] = t;  // (A_k^T G)(l, m)
    sh.T2[l][m] = u;  // (Pm A_k)(l, m)
  }
  wave_sync();
  // Gram of W - V_k A_k:  Q - A_k^T G - G^T A_k + A_k^T Pm A_k
  for (int e = tid; e < P * P; e += 64) {
    const int l = e / P, m = e % P;
    double t = 0.0;
    for (int r = 0; r < P; ++r) t += sh.Ak[r][l] * sh.T2[r][m];
    sh.Gam[l][m] = sh.Q[l * P + m] - sh.T1[l][m] - sh.T1[m][l] + t;
  }
  wave_sync();
  // symmetric working copy in T2 (off-diagonal entries averaged)
  for (int e = tid; e < P * P; e += 64) {
    const int l = e / P, m = e % P;
    sh.T2[l][m] = (l == m) ? sh.Gam[l][l] : 0.5 * (sh.Gam[l][m] + sh.Gam[m][l]);
    sh.Bk[l][m] = 0.0;
  }
  wave_sync();
  // right-looking Cholesky T2 = B_k^T B_k; each entry sees its subtractions
  // in the same order as the row-oriented recurrence.  Every lane forms the
  // pivot test and the entries of row l of B_k it needs itself, so a column
  // costs one exchange through LDS.
  constexpr int N = (P * P + 63) / 64;
#pragma unroll 1
  for (int l = 0; l < P; ++l) {
    const double d = sh.T2[l][l];
    const double thr = tau_fb * sh.araw[l];
    double tr[N], tc[N];
#pragma unroll
    for (int x = 0; x < N; ++x) {
      const int e = tid + 64 * x, r = (e / P) % P, c = e % P;
      tr[x] = sh.T2[l][r];
      tc[x] = sh.T2[l][c];
    }
    const bool ok = (d > 0.0) && isfinite(d) && (sqrt(d) >= thr);
    if (!ok) return false;
    const double piv = sqrt(d), inv = 1.0 / piv;
#pragma unroll
    for (int x = 0; x < N; ++x) {
      const int e = tid + 64 * x, r = e / P, c = e % P;
      if (e < P * P) {
        const double bc = tc[x] * inv;  // B_k(l, c)
        if (r == l && c >= l) sh.Bk[l][c] = (c == l) ? piv : bc;
        if (r > l && c > l) sh.T2[r][c] -= (tr[x] * inv) * bc;
      }
    }
    wave_sync();
  }
  // bench: V_{k+1}^T g_b = B_k^{-T} (W^T g_b - A_k^T V_k^T g_b), one lane per
  // vector; lane b writes row b of the coefficients (zeros for used vectors)
  if (tid < MAXB) {
    const int b = tid;
    const bool live = b >= taken && b < nb;
    const double* Wg = sh.Wg;
    const double* Vg = sh.Vg;
    double cf[P];
#pragma unroll
    for (int l = 0; l < P; ++l) {
      double c = 0.0;
      if (live) {
        double gw = Wg[l * nb + b];
        for (int r = 0; r < P; ++r) gw -= sh.Ak[r][l] * Vg[r * nb + b];
#pragma unroll
        for (int r = 0; r < l; ++r) gw -= sh.Bk[r][l] * cf[r];
        c = gw / sh.Bk[l][l];
      }
      cf[l] = c;
      st->bcoef[b * MAXP + l] = c;
    }
    for (int l = P; l < MAXP; ++l) st->bcoef[b * MAXP + l] = 0.0;
  }
  for (int e = tid; e < P * P; e += 64) {
    const int r = e / P, c = e % P;
    st->Ak[r * MAXP + c] = sh.Ak[r][c];
    st->Bk[r * MAXP + c] = sh.Bk[r][c];
    st->P2A[r * MAXP + c] = sh.Ak[r][c];
    st->P2B[r * MAXP + c] = sh.Bk[r][c];
  }
  if (tid < P) st->araw[tid] = sh.araw[tid];
  wave_sync();
  return true;
}

// The inputs, from the registers they were loaded into, to LDS: B_{k-1},
// the rotations of blocks k-2 and k-1 (ring slots (k-2) mod 3 and (k-1) mod 3;
// the identity before block 1), the S-hat window, the column norms of B, and
// either phase A's Gram products (mode 0) or A_k and B_k (mode 1).
template <int P>
__device__ __attribute__((always_inline)) inline void store_band_inputs(int mode, int nb, const BandCtl& ctl,
                                                                        const BandLoads<P>& L, BandShared<P>& sh) {
  const int tid = threadIdx.x;
  const int64_t k = ctl.k;
  const int s0 = (int)((k + 1) % 3), s1 = (int)((k + 2) % 3);  // (k-2) mod 3, (k-1) mod 3 for k >= 1
  const bool have0 = k - 2 >= 1, have1 = k - 1 >= 1;
#pragma unroll
  for (int x = 0; x < BandLoads<P>::N; ++x) {
    const int e = tid + 64 * x;
    if (e < P * P) {
      const int r = e / P, c = e % P;
      sh.Bp[r][c] = L.bprev[x];
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const double r0 = L.rot[0][w][x], r1 = L.rot[1][w][x], r2 = L.rot[2][w][x];
        const double v0 = s0 == 0 ? r0 : s0 == 1 ? r1 : r2;
        const double v1 = s1 == 0 ? r0 : s1 == 1 ? r1 : r2;
        const double id = w == 0 ? 1.0 : 0.0;
        sh.rot[0][r][c][w] = have0 ? v0 : id;
        sh.rot[1][r][c][w] = have1 ? v1 : id;
      }
      // S-hat window, column-major per lane: p live rows, then p zero rows
      sh.s2[c][r] = L.shat[x];
      sh.s2[c][P + r] = 0.0;
      if (mode == 0) {  // phase A's Gram products
        sh.G[e] = L.m0[x];
        sh.Q[e] = L.m1[x];
        sh.Pm[e] = L.m2[x];
      } else {  // A_k and B_k of the column-wise QR
        sh.Ak[r][c] = L.m0[x];
        sh.Bk[r][c] = L.m1[x];
      }
    }
  }
#pragma unroll
  for (int x = 0; x < BandLoads<P>::NW; ++x) {
    const int e = tid + 64 * x;
    if (mode == 0 && e < P * nb) {
      sh.Wg[e] = L.wg[x];
      sh.Vg[e] = L.vg[x];
    }
  }
  if (tid < P) {
    sh.beta[tid] = L.beta;
    if (mode == 0) sh.araw[tid] = sqrt(L.a);
  }
  wave_sync();
}

// Search directions of block k in the grouped form (eq. (4.1)):
//     M_k = V_k C_k + M_{k-1} D_k + M_{k-2} E_k,
//     C_k = R_c^{-1},  D_k = -R_b C_k,  E_k = -R_a C_k,
// on the leading l* columns (zero beyond), stored with Z_k (rows beyond l*
// zero) at the block's position t in the group.  At the group's last block,
// or when the iteration stops, the coefficients of the flush kernel follow
// from the backward recurrence over the group's m blocks
//     T_t = src_t + D_{t+1} T_{t+1} + E_{t+2} T_{t+2}   (t = m-1 .. 0),
// T_t being the total weight with which M_{g+1+t} enters the output
// (src_t = Z_t for X; the identity at t = m-2 or m-1, zero otherwise, for
// the search-direction blocks M_{g+m-1} and M_{g+m} the next group starts
// from):
//     Y[o][t] = C_t T_t,  Y[o][M_g] = D_0 T_0 + E_1 T_1,  Y[o][M_{g-1}] = E_0 T_0.
// Expanding the recurrence this way changes only the rounding of X.
template <int P>
__device__ void search_coefficients(DevState* __restrict__ st, BandShared<P>& sh, int64_t k, int lstar,
                                    bool finishing) {
  constexpr int S = group_len(P);
  const int tid = threadIdx.x;
  const int t = (int)((k - 1) % S);
  // C = R_c^{-1} (upper triangular) on the leading l* columns: lane q forms
  // row q in registers (entries left of the diagonal are 0 and add nothing)
  if (tid < P) {
    const int q = tid;
    double crow[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      double a = (q == i) ? 1.0 : 0.0;
#pragma unroll
      for (int r = 0; r < i; ++r) a = fma(-crow[r], sh.Rc[r][i], a);
      crow[i] = (i < lstar && q <= i) ? a / sh.Rc[i][i] : 0.0;
      sh.C[q][i] = crow[i];
    }
  }
  wave_sync();
  constexpr int NQ = (P * P + 63) / 64;
#pragma unroll
  for (int x = 0; x < NQ; ++x) {
    const int e = tid + 64 * x;
    if (e < P * P) {
      const int q = e / P, i = e % P;
      double d = 0.0, f = 0.0;
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const bool use = i < lstar && r <= i;
        const double cri = sh.C[r][i];
        d = use ? fma(-sh.Rb[q][r], cri, d) : d;
        f = use ? fma(-sh.Ra[q][r], cri, f) : f;
      }
      const double z = (q < lstar) ? sh.Zk[q][i] : 0.0;
      sh.D[q][i] = d;
      sh.E[q][i] = f;
      sh.Zk[q][i] = z;
      st->gC[t][q * MAXP + i] = sh.C[q][i];
      st->gD[t][q * MAXP + i] = d;
      st->gE[t][q * MAXP + i] = f;
      st->gZ[t][q * MAXP + i] = z;
    }
  }
  wave_sync();
  if (!finishing && t != S - 1) return;
  // stage the group's coefficients in LDS: positions u < t from the earlier
  // band kernels of the group, in batches whose loads are all in flight
  // before the first is stored (a single wavefront would otherwise wait for
  // each load in turn), and position t from this one
  {
    constexpr int EL = (P * P + 63) / 64;             // elements per lane and matrix
    constexpr int BATCH = 32 / (4 * EL) > 0 ? 32 / (4 * EL) : 1;
#pragma unroll 1
    for (int u0 = 0; u0 < t; u0 += BATCH) {
      double buf[BATCH][4][EL];
#pragma unroll
      for (int du = 0; du < BATCH; ++du)
#pragma unroll
        for (int w = 0; w < 4; ++w)
#pragma unroll
          for (int x = 0; x < EL; ++x) {
            const int u = u0 + du, e = tid + 64 * x;
            const double* src = w == 0 ? st->gC[u] : w == 1 ? st->gD[u] : w == 2 ? st->gE[u] : st->gZ[u];
            buf[du][w][x] = (u < t && e < P * P) ? src[(e / P) * MAXP + e % P] : 0.0;
          }
#pragma unroll
      for (int du = 0; du < BATCH; ++du)
#pragma unroll
        for (int w = 0; w < 4; ++w)
#pragma unroll
          for (int x = 0; x < EL; ++x) {
            const int u = u0 + du, e = tid + 64 * x;
            if (u < t && e < P * P) sh.gs[w][u][e / P][e % P] = buf[du][w][x];
          }
    }
  }
  for (int e = tid; e < P * P; e += 64) {
    const int r = e / P, c = e % P;
    sh.gs[0][t][r][c] = sh.C[r][c];
    sh.gs[1][t][r][c] = sh.D[r][c];
    sh.gs[2][t][r][c] = sh.E[r][c];
    sh.gs[3][t][r][c] = sh.Zk[r][c];
  }
  wave_sync();
  auto cC = [&](int u, int r, int c) { return sh.gs[0][u][r][c]; };
  auto cD = [&](int u, int r, int c) { return sh.gs[1][u][r][c]; };
  auto cE = [&](int u, int r, int c) { return sh.gs[2][u][r][c]; };
  auto cZ = [&](int u, int r, int c) { return sh.gs[3][u][r][c]; };
  const int m = t + 1;
  // the three outputs' recurrences run side by side (one element of each
  // per lane and step), which hides the latency of their dependent chains
  constexpr int NE = 3 * P * P, IT = (NE + 63) / 64;
#pragma unroll 1
  for (int u = m - 1; u >= 0; --u) {
    const int s0 = u % 3, s1 = (u + 1) % 3, s2 = (u + 2) % 3;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + 64 * it;
      if (e < NE) {
        const int o = e / (P * P), q = (e / P) % P, c = e % P;
        double v = (o == 0) ? cZ(u, q, c) : ((u == m - 3 + o && q == c) ? 1.0 : 0.0);
        if (u + 1 < m)
          for (int i = 0; i < P; ++i) v += cD(u + 1, q, i) * sh.Tr[o][s1][i][c];
        if (u + 2 < m)
          for (int i = 0; i < P; ++i) v += cE(u + 2, q, i) * sh.Tr[o][s2][i][c];
        sh.Tr[o][s0][q][c] = v;
      }
    }
    wave_sync();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + 64 * it;
      if (e < NE) {
        const int o = e / (P * P), q = (e / P) % P, c = e % P;
        double y = 0.0;
        for (int r = q; r < P; ++r) y += cC(u, q, r) * sh.Tr[o][s0][r][c];
        st->Y[o][u][q * MAXP + c] = y;
      }
    }
    wave_sync();
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = tid + 64 * it;
    if (e < NE) {
      const int o = e / (P * P), q = (e / P) % P, c = e % P;
      double yb = 0.0, ya = 0.0;
      for (int i = 0; i < P; ++i) {
        yb += cD(0, q, i) * sh.Tr[o][0][i][c];
        ya += cE(0, q, i) * sh.Tr[o][0][i][c];
      }
      if (m >= 2)
        for (int i = 0; i < P; ++i) yb += cE(1, q, i) * sh.Tr[o][1][i][c];
      st->Y[o][MAXS][q * MAXP + c] = yb;
      st->Y[o][MAXS + 1][q * MAXP + c] = ya;
    }
  }
  wave_sync();
  if (tid == 0) {
    st->flush_len = m;
    st->flush_keep = finishing ? 0 : 1;
    st->flush_block = k;
  }
}

// Rotations of the two previous blocks applied to rows 0 .. 3p-1 of the
// block's columns, which hold only B_{k-1} and A_k: the band kernel's second
// wavefront runs this while the first is still in phase A.
template <int P>
__device__ void prev_rotations(BandShared<P>& sh) {
  const int lane = threadIdx.x & 63;
  // column l of H-bar over the rows of blocks k-2 .. k (zero, B_{k-1}, A_k)
  for (int e = lane; e < 3 * P * P; e += 64) {
    const int l = e / (3 * P), r = e % (3 * P);
    double v = 0.0;
    if (r >= P && r < 2 * P) v = (r - P >= l) ? sh.Bp[l][r - P] : 0.0;
    if (r >= 2 * P) v = sh.Ak[r - 2 * P][l];
    sh.col[l][r] = v;
  }
  wave_sync();
  // Rotations of blocks k-2 and k-1.  Rotation (b, i) mixes row bp+i of a
  // column with the p rows below it, so lane l sweeps a window of p+1 rows
  // down its column in registers: the top row is final once its rotations
  // are applied and leaves the window, one untouched row enters at the
  // bottom.  The rotations of block k-2 reach column l only from row l on.
  // The next step's rotations and row are loaded ahead.  Row 3p, which
  // enters the window after the last step, belongs to block k+1 and is not
  // written yet: it is read but never used.
  if (lane < P) {
    const int l = lane;
    double cw[P + 1];
#pragma unroll
    for (int t = 0; t <= P; ++t) cw[t] = sh.col[l][t];
    double rc[P], rs[P];
#pragma unroll
    for (int t = 0; t < P; ++t) {
      rc[t] = sh.rot[0][0][t][0];
      rs[t] = sh.rot[0][0][t][1];
    }
    double nxt = sh.col[l][P + 1];
    // unrolled so that a step's chain of p rotations overlaps the next
    // step's, which needs only the first rotated row of this one
#pragma unroll 4
    for (int base = 0; base < 2 * P; ++base) {
      const bool live = base >= P || base >= l;
      double c[P], sn[P];
#pragma unroll
      for (int t = 0; t < P; ++t) {
        c[t] = rc[t];
        sn[t] = rs[t];
      }
      const double enter = nxt;
      const int ahead = base + 1 < 2 * P ? base + 1 : base;
#pragma unroll
      for (int t = 0; t < P; ++t) {
        rc[t] = sh.rot[ahead / P][ahead % P][t][0];
        rs[t] = sh.rot[ahead / P][ahead % P][t][1];
      }
      nxt = sh.col[l][ahead + 1 + P];
      double x = cw[0], y[P];
#pragma unroll
      for (int t = 0; t < P; ++t) y[t] = cw[t + 1];
#pragma unroll
      for (int t = 0; t < P; ++t) rotate(c[t], sn[t], x, y[t]);
      sh.col[l][base] = live ? x : cw[0];
#pragma unroll
      for (int t = 0; t < P; ++t) cw[t] = live ? y[t] : cw[t + 1];
      cw[P] = enter;
    }
#pragma unroll
    for (int t = 0; t < P; ++t) sh.col[l][2 * P + t] = cw[t];
  }
}

// Phase B: Givens QR of the p new columns of H-bar, S-hat window, residuals,
// stopping test, coefficients of the search directions and of the X update.
// Runs on the first wavefront after the rotations of the previous blocks.
// The same rows in the accumulating form (Section 4's remark on keeping the
// action of a block of reflectors as one matrix): the p^2 rotations of block
// k-1 are multiplied into one orthogonal 2p x 2p matrix Q_{k-1} over the rows
// of blocks k-1 and k (lane q forms column q; it is also kept in the state
// for the next block), and the new block's columns take Q_{k-2} (formed by
// the previous block's kernel) and Q_{k-1} as matrix products.  Q_{k-2}
// also holds the rotations of block k-2's first columns, which the
// sequential form skips for the columns to their right: they act on rows
// that are still zero there, so only the rounding changes.
template <int P>
__device__ void prev_rotations_acc(BandShared<P>& sh, DevState* __restrict__ st, int64_t k) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < 3 * P * P; e += 64) {
    const int l = e / (3 * P), r = e % (3 * P);
    double v = 0.0;
    if (r >= P && r < 2 * P) v = (r - P >= l) ? sh.Bp[l][r - P] : 0.0;
    if (r >= 2 * P) v = sh.Ak[r - 2 * P][l];
    sh.col[l][r] = v;
  }
  const bool have0 = k - 2 >= 1, have1 = k - 1 >= 1;
  if (lane < 2 * P) {
    const int q = lane;
    double qc[2 * P];
#pragma unroll
    for (int r = 0; r < 2 * P; ++r) qc[r] = r == q ? 1.0 : 0.0;
    if (have1) {
#pragma unroll 1
      for (int i = 0; i < P; ++i)
#pragma unroll
        for (int t = 0; t < P; ++t) rotate(sh.rot[1][i][t][0], sh.rot[1][i][t][1], qc[i], qc[i + t + 1]);
    }
    double (*Qk1)[2 * MAXP] = st->Qacc[(k + 1) & 1];  // slot of block k-1
    const double (*Qk2)[2 * MAXP] = st->Qacc[k & 1];  // slot of block k-2
#pragma unroll
    for (int r = 0; r < 2 * P; ++r) {
      sh.Qb[1][r][q] = qc[r];
      Qk1[r][q] = qc[r];
      sh.Qb[0][r][q] = have0 ? Qk2[r][q] : (r == q ? 1.0 : 0.0);
    }
  }
  wave_sync();
  // rows [0, 2p) by Q_{k-2}, then rows [p, 3p) by Q_{k-1}; each lane forms
  // up to NO outputs in registers before any is written back
  constexpr int NO = (2 * P * P + 63) / 64;
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    if (w == 0 ? !have0 : !have1) continue;
    const int off = w * P;
    double o[NO];
#pragma unroll
    for (int x = 0; x < NO; ++x) {
      const int e = lane + 64 * x;
      double a = 0.0;
      if (e < 2 * P * P) {
        const int l = e / (2 * P), r = e % (2 * P);
#pragma unroll
        for (int t = 0; t < 2 * P; ++t) a = fma(sh.Qb[w][r][t], sh.col[l][off + t], a);
      }
      o[x] = a;
    }
    wave_sync();
#pragma unroll
    for (int x = 0; x < NO; ++x) {
      const int e = lane + 64 * x;
      if (e < 2 * P * P) sh.col[e / (2 * P)][off + e % (2 * P)] = o[x];
    }
    wave_sync();
  }
}

template <int P>
__device__ void phase_b(const BandCtl ctl, DevState* __restrict__ st, double* __restrict__ hist, BandShared<P>& sh) {
  const int tid = threadIdx.x;
  const int64_t k = ctl.k;
  const int64_t j0 = ctl.j0;
  const int lcap = ctl.lcap, cap_status = ctl.cap_status;
  const double tol = ctl.tol;
  const int64_t max_iter = ctl.max_iter, hist_cap = ctl.hist_cap;
  // rows 3p .. 4p-1 of column l (block k+1: B_k), then a row read ahead past
  // the last column and never used; the rows above come from prev_rotations
  for (int e = tid; e < P * (P + 1); e += 64) {
    const int l = e / (P + 1), r = e % (P + 1);
    sh.col[l][3 * P + r] = (r < P && r <= l) ? sh.Bk[r][l] : 0.0;
  }
  wave_sync();
  // Each column of the block has two windows of p+1 rows that the column's
  // rotations sweep down: one of H-bar, held by lane q of the first row of
  // 16 lanes (rows 2p+i .. 3p+i at column i), and one of S-hat, held by lane
  // 16+q of the second row (rows i .. i+p; rows p and beyond start at 0).
  // Both rows apply the same rotations in the same instructions.
  const bool hlane = tid < P, slane = tid >= 16 && tid < 16 + P;
  const int q = hlane ? tid : slane ? tid - 16 : 0;
  double win[P + 1];
#pragma unroll
  for (int t = 0; t <= P; ++t) win[t] = hlane ? sh.col[q][2 * P + t] : slane ? sh.s2[q][t] : 0.0;
  wave_sync();

  // 1 / ||b_q|| of the S-hat lane's column (0 for a zero right-hand side)
  const double binv = (slane && sh.beta[q] > 0.0) ? 1.0 / sh.beta[q] : 0.0;
  int lstar = P, finished = 0, status = STATUS_RUNNING;
#pragma unroll 1
  for (int i = 0; i < P; ++i) {
    if (i >= lcap) {  // the column-wise QR ran out of substitutes at column i
      status = cap_status;
      finished = 1;
      lstar = i;
      break;
    }
    const int64_t j = j0 + i + 1;
    const int piv = 2 * P + i;
    // everything this column reads from the other lanes, in one batch: the
    // pivot column i (rows piv .. piv+p) and its rows q, p+q, 2p+q for R;
    // then the row entering this lane's window
    const double x0 = sh.col[i][piv];
    const double y = (tid < P) ? sh.col[i][piv + 1 + tid] : 0.0;
    const double ra = sh.col[i][q], rb = sh.col[i][P + q], rcv = sh.col[i][2 * P + q];
    const double enter = hlane ? sh.col[q][piv + 1 + P] : 0.0;
    // New rotations zero the p subdiagonal entries y_1..y_p of column j
    // against its diagonal x_0.  Rotation t leaves
    //     x_t = sqrt(x_0^2 + y_1^2 + ... + y_t^2)
    // on the diagonal (x_0 itself while y_1..y_t are all zero, the identity
    // rotations of givens()), and is c_t = x_{t-1} / x_t, s_t = y_t / x_t.
    // Lane t-1 forms x_t from a prefix sum of squares over the lanes,
    // scaled by a power of two near the column's largest magnitude, so the
    // p rotations come out at once instead of through p dependent hypot
    // calls.
    double m = row_max(fabs(y));
    m = fmax(m, fabs(x0));
    // power-of-two scale: exact, and keeps the squares in range
    int ex = 0;
    if (m > 0.0 && isfinite(m)) (void)frexp(m, &ex);
    const double inv = ldexp(1.0, -ex), scl = ldexp(1.0, ex);
    double ps = (y * inv) * (y * inv);
    int nz = (y != 0.0) ? 1 : 0;
#pragma unroll
    for (int o = 1; o < P; o <<= 1) {  // inclusive scan; lanes below o add 0
      ps += row_shr(ps, o);
      nz |= row_shr(nz, o);
    }
    const double xs = x0 * inv;
    const double xt = nz ? scl * sqrt(xs * xs + ps) : x0;
    double xprev = row_shr(xt, 1);
    if (tid == 0) xprev = x0;
    if (tid < P) {
      const bool ident = (y == 0.0);
      const double rinv = 1.0 / xt;
      sh.nrot[i][tid][0] = ident ? 1.0 : xprev * rinv;
      sh.nrot[i][tid][1] = ident ? 0.0 : y * rinv;
    }
    const double pivot = lane_value(xt, P - 1);  // the new diagonal entry
    if (!(pivot != 0.0)) {
      if (tid == 0) {
        halt_with(st, isfinite(pivot) ? BMR_SINGULAR_R : BMR_NONFINITE, REASON_ERROR);
        st->j = j - 1;
      }
      return;
    }
    wave_sync();
    if (hlane) {  // column j of R: rows of blocks k-2, k-1 and k (lane q writes row q of each)
      sh.Ra[q][i] = (q >= i) ? ra : 0.0;
      sh.Rb[q][i] = rb;
      sh.Rc[q][i] = (q < i) ? rcv : (q == i) ? pivot : 0.0;
    }
    double ratio = 0.0;
    // the rotations of column i reach the later columns of the block and
    // every column of S-hat
    if ((hlane && q > i) || slane) {
      double c[P], sn[P];
#pragma unroll
      for (int t = 0; t < P; ++t) {
        c[t] = sh.nrot[i][t][0];
        sn[t] = sh.nrot[i][t][1];
      }
      double x = win[0], yy[P];
#pragma unroll
      for (int t = 0; t < P; ++t) yy[t] = win[t + 1];
#pragma unroll
      for (int t = 0; t < P; ++t) rotate(c[t], sn[t], x, yy[t]);
#pragma unroll
      for (int t = 0; t < P; ++t) win[t] = yy[t];
      win[P] = enter;
      if (hlane) {
        sh.col[q][piv] = x;
#pragma unroll
        for (int t = 0; t < P; ++t) sh.col[q][piv + 1 + t] = yy[t];
      } else {
        // recurrence residual rho_j^{(q)} = ||S-hat(j+1:j+p, q)|| (eq. (3.5)),
        // the squares summed pairwise
        double sq[P];
#pragma unroll
        for (int t = 0; t < P; ++t) sq[t] = yy[t] * yy[t];
#pragma unroll
        for (int w = 1; w < P; w <<= 1)
#pragma unroll
          for (int t = 0; t + w < P; t += 2 * w) sq[t] += sq[t + w];
        ratio = binv > 0.0 ? sqrt(sq[0]) * binv : 0.0;
        sh.Zk[i][q] = x;
        st->rho[q] = ratio;
        if (j <= hist_cap) hist[(j - 1) * P + q] = ratio;
      }
    }
    // stopping test over the columns (the S-hat lanes, in the second row):
    // the largest ratio, with a non-finite ratio counted as +inf; every lane
    // takes lane 16's decision
    const double worst = lane_value(row_max(isfinite(ratio) ? ratio : INFINITY), 16);
    const int f = (worst == INFINITY) ? 2 : (worst < tol) ? 1 : (j >= max_iter) ? 3 : 0;
    if (f == 2) {
      if (tid == 0) {
        halt_with(st, BMR_NONFINITE, REASON_ERROR);
        st->j = j - 1;
      }
      return;
    }
    if (f) {
      status = (f == 1) ? BMR_CONVERGED : BMR_MAX_ITER;
      finished = 1;
      lstar = i + 1;
      break;
    }
    wave_sync();
  }
  // S-hat rows p .. 2p-1, carried to the next block
  if (!finished && slane) {
#pragma unroll
    for (int t = 0; t < P; ++t) sh.s2[q][P + t] = win[t];
  }
  wave_sync();
  search_coefficients<P>(st, sh, k, lstar, finished);
  // A finished block (lstar = 0 included) still goes through pass 2, which
  // applies the X updates the earlier blocks of its group left pending.
  if (finished) {
    if (tid == 0) {
      st->lstar = lstar;
      st->k2 = k;
      st->j = j0 + lstar;
      st->status = status;
      st->reason = REASON_FINISHED;
      st->halt = 1;
    }
    return;
  }
  const int rk = (int)(k % 3);
  for (int e = tid; e < P * P; e += 64) {
    const int i = e / P, t = e % P;
    st->rot[rk][i][t][0] = sh.nrot[i][t][0];
    st->rot[rk][i][t][1] = sh.nrot[i][t][1];
    st->Bprev[i * MAXP + t] = sh.Bk[i][t];
    st->Shat[i * MAXP + t] = sh.s2[t][P + i];
  }
  if (tid == 0) {
    st->lstar = P;
    st->k2 = k;
    st->j = j0 + P;
    st->k = k + 1;
  }
}

// mode 0: phase A then phase B.  mode 1: the host has supplied B_k (column-
// wise QR) and already formed V_{k+1}; run phase B with pass 2 told to keep
// V_{k+1} as it is.  nb: bench vectors (the state's nb).
//
// Two wavefronts: the first loads the inputs and runs phase A; the second
// applies the rotations of the previous blocks meanwhile (they need only
// B_{k-1} and A_k).  The first then runs phase B alone.  Both wavefronts
// reach both barriers on every path that gets past the halt test.
template <int P>
__global__ __launch_bounds__(128) void k_band(int mode, int nb, const double* __restrict__ red,
                                             double* __restrict__ hist, DevState* __restrict__ st) {
  __shared__ BandShared<P> sh;
  const bool first = threadIdx.x < 64;
  BandCtl ctl;
  BandLoads<P> L;
  if (first) load_band<P>(mode, nb, red, st, ctl, L);
  else ctl.halt = st->halt;
  if (ctl.halt) {  // the same in both wavefronts: nothing writes it meanwhile
    if (threadIdx.x == 0) st->k2 = 0;
    return;
  }
  if (first) {
    store_band_inputs<P>(mode, nb, ctl, L, sh);
    if (mode == 0) phase_a_ak<P>(sh);
  }
  wg_lds_sync();  // B_{k-1}, A_k and the rotations are in LDS
  bool ok = true;
  if (first) {
    if (mode == 0) {
      ok = !ctl.force_qr && phase_a<P>(nb, ctl.taken, ctl.tau_fb, st, sh);
      if (!ok && threadIdx.x == 0) {
        for (int e = 0; e < P * P; ++e) st->Ak[(e / P) * MAXP + (e % P)] = sh.Ak[e / P][e % P];
        for (int c = 0; c < P; ++c) st->araw[c] = sh.araw[c];
        st->reason = REASON_EXPLICIT_QR;
        st->halt = 1;
        st->k2 = 0;
      }
    } else {
      for (int e = threadIdx.x; e < P * P; e += 64) {
        const int r = e / P, c = e % P;
        st->P2A[r * MAXP + c] = 0.0;
        st->P2B[r * MAXP + c] = (r == c) ? 1.0 : 0.0;
      }
      for (int e = threadIdx.x; e < MAXB * MAXP; e += 64) st->bcoef[e] = 0.0;
    }
  } else if (st->accumulate) {
    prev_rotations_acc<P>(sh, st, st->k);
  } else {
    prev_rotations<P>(sh);
  }
  wg_lds_sync();  // rows 0 .. 3p-1 of the columns rotated, B_k in LDS
  if (first && ok) phase_b<P>(ctl, st, hist, sh);
}

}  // namespace

hipError_t launch_reduce(const double* part, int n_wg, int n_ent, double* red, DevState* st, int check_halt,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(n_ent), dim3(64), 0, s, part, n_wg, red, st, check_halt);
  return hipGetLastError();
}

hipError_t launch_band(int p, int mode, int nb, const double* red, double* hist, DevState* st, hipStream_t s) {
  if (nb < 0 || nb > MAXB) return hipErrorInvalidValue;
#define LB(P) hipLaunchKernelGGL(k_band<P>, dim3(1), dim3(128), 0, s, mode, nb, red, hist, st)
  switch (p) {
    case 1: LB(1); break;
    case 2: LB(2); break;
    case 3: LB(3); break;
    case 4: LB(4); break;
    case 5: LB(5); break;
    case 6: LB(6); break;
    case 7: LB(7); break;
    case 8: LB(8); break;
    case 9: LB(9); break;
    case 10: LB(10); break;
    case 11: LB(11); break;
    case 12: LB(12); break;
    case 13: LB(13); break;
    case 14: LB(14); break;
    case 15: LB(15); break;
    case 16: LB(16); break;
    default: return hipErrorInvalidValue;
  }
#undef LB
  return hipGetLastError();
}

}  // namespace bmr
