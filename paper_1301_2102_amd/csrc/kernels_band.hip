// Reduction of the pass-1 partial sums and the band kernel: one wavefront
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
//
// Work split inside the wavefront: lane l owns column l of the block (its
// 4p band entries, kept in LDS) and column l of the S-hat window.  The
// rotations of the two previous blocks are applied by all lanes at once; the
// p rotations of each column of the block are generated together (lane t
// makes rotation t from a prefix sum of squares) and applied by the lanes
// owning the columns to its right.
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

// The band kernel runs as a single wavefront (64 lanes).  Its barriers only
// have to order LDS accesses between the lanes of that wavefront, which the
// LDS executes in issue order; __syncthreads() would add a workgroup-scope
// fence, which waits for every outstanding global store (the R rows, Z, the
// residuals and the history written as the loop goes) on each call.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline void rotate(double c, double s, double& x, double& y) {
  const double a = x, b = y;
  x = c * a + s * b;
  y = -s * a + c * b;
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
  double col[P][4 * P + 1];  // column l of H-bar, rows of blocks k-2 .. k+1
  double s2[P][2 * P + 1];   // column q of the S-hat window (p live + p new rows)
  double piv;
  int flag;
};

// Phase A: A_k, Gram of the remainder, Cholesky -> B_k, bench coefficients.
// Returns false (the same in every lane) when the column-wise QR must take
// over.  Leaves A_k and B_k in shared memory.
template <int P>
__device__ bool phase_a(const double* __restrict__ red, DevState* __restrict__ st, BandShared<P>& sh) {
  const int tid = threadIdx.x;
  const int nb = st->nb, taken = st->taken;
  for (int e = tid; e < P * P; e += 64) {
    sh.G[e] = red[off_G(P) + e];
    sh.Q[e] = red[off_Q(P) + e];
    sh.Pm[e] = red[off_P(P) + e];
  }
  for (int e = tid; e < P * nb; e += 64) {
    sh.Wg[e] = red[off_Wg(P) + e];
    sh.Vg[e] = red[off_Vg(P, nb) + e];
  }
  if (tid < P) sh.araw[tid] = sqrt(red[off_a(P) + tid]);
  wave_sync();
  for (int e = tid; e < P * P; e += 64) {
    const int r = e / P, c = e % P;
    sh.Ak[r][c] = (r >= c) ? sh.G[r * P + c] : sh.G[c * P + r];
  }
  wave_sync();
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
  // in the same order as the row-oriented recurrence
#pragma unroll 1
  for (int l = 0; l < P; ++l) {
    if (tid == 0) {
      const double d = sh.T2[l][l];
      const double thr = st->tau_fb * sh.araw[l];
      const bool ok = (d > 0.0) && isfinite(d) && (sqrt(d) >= thr);
      sh.flag = ok;
      sh.piv = ok ? sqrt(d) : 0.0;
    }
    wave_sync();
    if (!sh.flag) return false;
    if (tid == l) sh.Bk[l][l] = sh.piv;
    if (tid > l && tid < P) sh.Bk[l][tid] = sh.T2[l][tid] / sh.piv;
    wave_sync();
    for (int e = tid; e < P * P; e += 64) {
      const int r = e / P, c = e % P;
      if (r > l && c > l) sh.T2[r][c] -= sh.Bk[l][r] * sh.Bk[l][c];
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

// Inputs of phase B that phase A does not touch: B_{k-1}, the rotations of
// blocks k-2 and k-1, the S-hat window and the column norms of B.  Issued
// first so that their latency overlaps phase A.
template <int P>
__device__ void load_band_inputs(const DevState* __restrict__ st, BandShared<P>& sh) {
  const int tid = threadIdx.x;
  const int64_t k = st->k;
  for (int e = tid; e < P * P; e += 64) {
    const int r = e / P, c = e % P;
    sh.Bp[r][c] = st->Bprev[r * MAXP + c];
  }
  for (int e = tid; e < 2 * P * P; e += 64) {
    const int b = e / (P * P), i = (e / P) % P, t = e % P;
    const int64_t kb = k - 2 + b;  // block whose rotations these are
    const bool have = kb >= 1;
    const int rb = have ? (int)(kb % 3) : 0;
    sh.rot[b][i][t][0] = have ? st->rot[rb][i][t][0] : 1.0;
    sh.rot[b][i][t][1] = have ? st->rot[rb][i][t][1] : 0.0;
  }
  for (int e = tid; e < 2 * P * P; e += 64) {  // S-hat window, column-major per lane
    const int q = e / (2 * P), r = e % (2 * P);
    sh.s2[q][r] = (r < P) ? st->Shat[r * MAXP + q] : 0.0;
  }
  if (tid < P) sh.beta[tid] = st->beta[tid];
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
  // C = R_c^{-1} (upper triangular) on the leading l* columns: lane q forms row q
  if (tid < P) {
    const int q = tid;
#pragma unroll 1
    for (int i = 0; i < P; ++i) {
      double c = 0.0;
      if (i < lstar && q <= i) {
        double a = (q == i) ? 1.0 : 0.0;
        for (int r = q; r < i; ++r) a -= sh.C[q][r] * sh.Rc[r][i];
        c = a / sh.Rc[i][i];
      }
      sh.C[q][i] = c;
    }
  }
  wave_sync();
  for (int e = tid; e < P * P; e += 64) {
    const int q = e / P, i = e % P;
    double d = 0.0, f = 0.0;
    if (i < lstar) {
      for (int r = 0; r <= i; ++r) {
        d -= sh.Rb[q][r] * sh.C[r][i];
        f -= sh.Ra[q][r] * sh.C[r][i];
      }
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

// Phase B: Givens QR of the p new columns of H-bar, S-hat window, residuals,
// stopping test, coefficients of the search directions and of the X update.
// Columns live in LDS and the outer loops stay rolled: the kernel runs as a
// single wavefront, so compact code matters more than register residency.
template <int P>
__device__ void phase_b(DevState* __restrict__ st, double* __restrict__ hist, BandShared<P>& sh) {
  const int tid = threadIdx.x;
  const int64_t k = st->k;
  const int64_t j0 = st->j;
  const int lcap = st->lcap, cap_status = st->cap_status;
  const double tol = st->tol;
  const int64_t max_iter = st->max_iter, hist_cap = st->hist_cap;
  // column l of H-bar over the rows of blocks k-2 .. k+1
  for (int e = tid; e < 4 * P * P; e += 64) {
    const int l = e / (4 * P), r = e % (4 * P);
    double v = 0.0;
    if (r >= P && r < 2 * P) v = (r - P >= l) ? sh.Bp[l][r - P] : 0.0;
    if (r >= 2 * P && r < 3 * P) v = sh.Ak[r - 2 * P][l];
    if (r >= 3 * P) v = (r - 3 * P <= l) ? sh.Bk[r - 3 * P][l] : 0.0;
    sh.col[l][r] = v;
  }
  wave_sync();
  // rotations of columns j-2p .. j-1 that lie in blocks k-2 (i >= l) and k-1
  if (tid < P) {
    const int l = tid;
#pragma unroll 1
    for (int b = 0; b < 2; ++b)
#pragma unroll 1
      for (int i = (b == 0 ? l : 0); i < P; ++i) {
        const int base = b * P + i;
        double x = sh.col[l][base], y[P];
#pragma unroll
        for (int t = 0; t < P; ++t) y[t] = sh.col[l][base + 1 + t];
#pragma unroll
        for (int t = 0; t < P; ++t) rotate(sh.rot[b][i][t][0], sh.rot[b][i][t][1], x, y[t]);
        sh.col[l][base] = x;
#pragma unroll
        for (int t = 0; t < P; ++t) sh.col[l][base + 1 + t] = y[t];
      }
  }
  wave_sync();

  // 1 / ||b_q|| of this lane's column (0 for a zero right-hand side)
  const double binv = (tid < P && sh.beta[tid] > 0.0) ? 1.0 / sh.beta[tid] : 0.0;
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
    {
      // New rotations zero the p subdiagonal entries y_1..y_p of column j
      // against its diagonal x_0.  Rotation t leaves
      //     x_t = sqrt(x_0^2 + y_1^2 + ... + y_t^2)
      // on the diagonal (x_0 itself while y_1..y_t are all zero, the identity
      // rotations of givens()), and is c_t = x_{t-1} / x_t, s_t = y_t / x_t.
      // Lane t-1 forms x_t from a prefix sum of squares over the lanes,
      // scaled by a power of two near the column's largest magnitude, so the
      // p rotations come out at once instead of through p dependent hypot
      // calls.
      const double x0 = sh.col[i][piv];
      const double y = (tid < P) ? sh.col[i][piv + 1 + tid] : 0.0;
      double m = fabs(y);
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) m = fmax(m, __shfl_xor(m, o, 16));
      m = fmax(m, fabs(x0));
      // power-of-two scale: exact, and keeps the squares in range
      int ex = 0;
      if (m > 0.0 && isfinite(m)) (void)frexp(m, &ex);
      const double inv = ldexp(1.0, -ex), scl = ldexp(1.0, ex);
      double ps = (y * inv) * (y * inv);
      int nz = (y != 0.0) ? 1 : 0;
#pragma unroll
      for (int o = 1; o < P; o <<= 1) {
        const double a = __shfl_up(ps, o, 64);
        const int b = __shfl_up(nz, o, 64);
        if (tid >= o) {
          ps += a;
          nz |= b;
        }
      }
      const double xs = x0 * inv;
      const double xt = nz ? scl * sqrt(xs * xs + ps) : x0;
      double xprev = __shfl_up(xt, 1, 64);
      if (tid == 0) xprev = x0;
      if (tid < P) {
        const bool ident = (y == 0.0);
        const double rinv = 1.0 / xt;
        sh.nrot[i][tid][0] = ident ? 1.0 : xprev * rinv;
        sh.nrot[i][tid][1] = ident ? 0.0 : y * rinv;
      }
      if (tid == P - 1) {
        sh.col[i][piv] = xt;
        sh.piv = xt;
      }
    }
    wave_sync();
    if (!(sh.piv != 0.0)) {
      if (tid == 0) {
        halt_with(st, isfinite(sh.piv) ? BMR_SINGULAR_R : BMR_NONFINITE, REASON_ERROR);
        st->j = j - 1;
      }
      return;
    }
    double ratio = 0.0;
    if (tid < P) {
      const int q = tid;
      // column j of R: rows of blocks k-2, k-1 and k (lane q writes row q of each)
      sh.Ra[q][i] = (q >= i) ? sh.col[i][q] : 0.0;
      sh.Rb[q][i] = sh.col[i][P + q];
      sh.Rc[q][i] = (q <= i) ? sh.col[i][2 * P + q] : 0.0;
      if (q > i) {  // later columns of the block receive the rotations of column i
        double x = sh.col[q][piv], y[P];
#pragma unroll
        for (int t = 0; t < P; ++t) y[t] = sh.col[q][piv + 1 + t];
#pragma unroll
        for (int t = 0; t < P; ++t) rotate(sh.nrot[i][t][0], sh.nrot[i][t][1], x, y[t]);
        sh.col[q][piv] = x;
#pragma unroll
        for (int t = 0; t < P; ++t) sh.col[q][piv + 1 + t] = y[t];
      }
      // S-hat rows i .. i+p of column q
      double x = sh.s2[q][i], y[P];
#pragma unroll
      for (int t = 0; t < P; ++t) y[t] = sh.s2[q][i + 1 + t];
#pragma unroll
      for (int t = 0; t < P; ++t)
        if (sh.nrot[i][t][1] != 0.0) rotate(sh.nrot[i][t][0], sh.nrot[i][t][1], x, y[t]);
      sh.s2[q][i] = x;
      // recurrence residual rho_j^{(q)} = ||S-hat(j+1:j+p, q)|| (eq. (3.5))
      double ss = 0.0;
#pragma unroll
      for (int t = 0; t < P; ++t) {
        sh.s2[q][i + 1 + t] = y[t];
        ss += y[t] * y[t];
      }
      ratio = binv > 0.0 ? sqrt(ss) * binv : 0.0;
      sh.Zk[i][q] = x;
      st->rho[q] = ratio;
      if (j <= hist_cap) hist[(j - 1) * P + q] = ratio;
    }
    // stopping test over the columns (lanes 0..p-1 of the first 16): the
    // largest ratio, with a non-finite ratio counted as +inf
    double worst = isfinite(ratio) ? ratio : INFINITY;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) worst = fmax(worst, __shfl_xor(worst, o, 16));
    worst = __shfl(worst, 0, 64);  // every lane takes lane 0's decision
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
// V_{k+1} as it is.
template <int P>
__global__ __launch_bounds__(64) void k_band(int mode, const double* __restrict__ red, double* __restrict__ hist,
                                            DevState* __restrict__ st) {
  __shared__ BandShared<P> sh;
  const int tid = threadIdx.x;
  if (tid == 0) sh.flag = st->halt;
  wave_sync();
  if (sh.flag) {
    if (tid == 0) st->k2 = 0;
    return;
  }
  wave_sync();
  load_band_inputs<P>(st, sh);
  if (mode == 0) {
    if (!phase_a<P>(red, st, sh)) {
      if (tid == 0) {
        for (int e = 0; e < P * P; ++e) st->Ak[(e / P) * MAXP + (e % P)] = sh.Ak[e / P][e % P];
        for (int c = 0; c < P; ++c) st->araw[c] = sh.araw[c];
        st->reason = REASON_EXPLICIT_QR;
        st->halt = 1;
        st->k2 = 0;
      }
      return;
    }
  } else {
    for (int e = tid; e < P * P; e += 64) {
      const int r = e / P, c = e % P;
      sh.Ak[r][c] = st->Ak[r * MAXP + c];
      sh.Bk[r][c] = st->Bk[r * MAXP + c];
      st->P2A[r * MAXP + c] = 0.0;
      st->P2B[r * MAXP + c] = (r == c) ? 1.0 : 0.0;
    }
    for (int e = tid; e < MAXB * MAXP; e += 64) st->bcoef[e] = 0.0;
    wave_sync();
  }
  phase_b<P>(st, hist, sh);
}

}  // namespace

hipError_t launch_reduce(const double* part, int n_wg, int n_ent, double* red, DevState* st, int check_halt,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(n_ent), dim3(256), 0, s, part, n_wg, red, st, check_halt);
  return hipGetLastError();
}

hipError_t launch_band(int p, int mode, const double* red, double* hist, DevState* st, hipStream_t s) {
#define LB(P) hipLaunchKernelGGL(k_band<P>, dim3(1), dim3(64), 0, s, mode, red, hist, st)
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
