// CSR block operator kernels for gfx950:
//   - pass 1 of a block iteration: W = A V_k - V_{k-1} B_{k-1}^T together with
//     the per-workgroup partial Gram products the band kernel needs,
//   - the plain block product W = A V,
//   - the explicit residual R = B - A X with column norms.
//
// Layout: every n x p block is row-interleaved (element (i, c) at i*p + c), so
// the p values one matrix entry multiplies are one contiguous 8p-byte segment.
// For p >= 3 a group of LPR lanes owns one row and lane c holds CPL adjacent
// columns (CPL = 2 for even p >= 6, so that one 16-byte load per lane and
// matrix entry covers the segment); the group loads up to LPR (column, value)
// pairs of the row at once, passes them round with cross-lane shuffles and
// issues all of the gathered loads before it consumes any.  Each row of A is
// read once for all p columns.  For p <= 2 one lane owns a whole row.  These
// shapes come from a sweep of lanes per row, columns per lane and grid size on
// the 128^3 Laplacian.
//
// The p x p Gram products of pass 1 (V^T V, V^T W, W^T W) are accumulated on
// the matrix cores: each wavefront stages its rows of [V_k  W] in LDS and feeds
// them, four rows at a time, to V_MFMA_F64_16X16X4F64 as both operands, so the
// 16 x 16 accumulator collects X^T X for X = [V_k W] (p <= 8) or one product
// per accumulator (p > 8).  The accumulators stay in registers for the whole
// row range of the workgroup.
//
// Every kernel is a template over the storage type T of the blocks and of the
// matrix values: double for the FP64 solver, float for the inner solve of the
// mixed-precision solver, where the block operator and the Gram products run
// in FP32 with FP32 accumulation (V_MFMA_F32_16X16X4F32); the per-workgroup
// partial sums are handed on in FP64 in both cases.
#include <algorithm>

#include "bmr_internal.hpp"

namespace bmr {
namespace {

constexpr int WG = 256;
constexpr int PASS1_MAX_WG = 2048;
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Per-type vector and matrix-core helpers.
template <typename T>
struct TypeOps;
template <>
struct TypeOps<double> {
  using v2 = double2;
  using acc4 = dbl4;
  __device__ static acc4 mfma(double a, double b, acc4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // accumulator layout (measured on gfx950): element i of lane l holds row
  // 4*i + l/16, column l%16 of the 16 x 16 product
  __device__ static int acc_row(int lane, int i) { return 4 * i + lane / 16; }
};
template <>
struct TypeOps<float> {
  using v2 = float2;
  using acc4 = flt4;
  __device__ static acc4 mfma(float a, float b, acc4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // measured on gfx950: element i of lane l holds row 4*(l/16) + i, column l%16
  __device__ static int acc_row(int lane, int i) { return 4 * (lane / 16) + i; }
};

// Row layout for block size p: one lane per row for p <= 2; otherwise a group
// of lpr lanes per row with cpl adjacent columns per lane.
__host__ __device__ constexpr int layout_cpl(int p) { return p <= 2 ? p : ((p % 2 == 0 && p >= 6) ? 2 : 1); }
__host__ __device__ constexpr int layout_lpr(int p) {
  return p <= 2 ? 1 : ((p + layout_cpl(p) - 1) / layout_cpl(p) <= 4 ? 4 : (p + layout_cpl(p) - 1) / layout_cpl(p) <= 8 ? 8 : 16);
}
__host__ __device__ constexpr int layout_rpg(int p) { return (WG / 64) * (64 / layout_lpr(p)); }

template <int P>
struct Lanes {
  static constexpr bool ROW = P <= 2;                // one lane per row
  static constexpr int CPL = layout_cpl(P);          // columns per lane
  static constexpr int LPR = layout_lpr(P);          // lanes per row
  static constexpr int RPW = 64 / LPR;               // rows per wavefront
  static constexpr int RPG = layout_rpg(P);          // rows per workgroup step
};

// x[0..CPL) = p[0 .. CPL) as one vector load (p is 2-element aligned when CPL = 2)
template <int CPL, typename T>
__device__ inline void vload(const T* __restrict__ p, T (&x)[CPL]) {
  if constexpr (CPL == 2) {
    const typename TypeOps<T>::v2 v = *reinterpret_cast<const typename TypeOps<T>::v2*>(p);
    x[0] = v.x;
    x[1] = v.y;
  } else {
#pragma unroll
    for (int k = 0; k < CPL; ++k) x[k] = p[k];
  }
}

template <int CPL, typename T>
__device__ inline void vstore(T* __restrict__ p, const T (&x)[CPL]) {
  if constexpr (CPL == 2) {
    typename TypeOps<T>::v2 v;
    v.x = x[0];
    v.y = x[1];
    *reinterpret_cast<typename TypeOps<T>::v2*>(p) = v;
  } else {
#pragma unroll
    for (int k = 0; k < CPL; ++k) p[k] = x[k];
  }
}

// In the group layout, loads and stores of data used once per launch (the
// CSR entries, V_{k-1}, W, the bench) carry the non-temporal hint, so that
// they do not push out of L2 the rows of V_k that neighbouring matrix rows
// gather again (pass 1 at 128^3, p = 8: 0.200 -> 0.177 ms).  The hint only
// pays where one instruction consumes whole cache lines (a group's lanes
// cover a row, or consecutive CSR entries): where consecutive instructions
// of a lane read the same lines (one lane per row), evict-first drops the
// line between them, so those accesses stay ordinary.
template <typename T>
__device__ inline T ldnt(const T* p) {
  return __builtin_nontemporal_load(p);
}

template <int CPL, typename T>
__device__ inline void vload_nt(const T* __restrict__ p, T (&x)[CPL]) {
  if constexpr (CPL == 2) {
    typedef T nv2 __attribute__((ext_vector_type(2)));
    const nv2 v = __builtin_nontemporal_load(reinterpret_cast<const nv2*>(p));
    x[0] = v.x;
    x[1] = v.y;
  } else {
#pragma unroll
    for (int k = 0; k < CPL; ++k) x[k] = __builtin_nontemporal_load(p + k);
  }
}

template <int CPL, typename T>
__device__ inline void vstore_nt(T* __restrict__ p, const T (&x)[CPL]) {
  if constexpr (CPL == 2) {
    typedef T nv2 __attribute__((ext_vector_type(2)));
    nv2 v;
    v.x = x[0];
    v.y = x[1];
    __builtin_nontemporal_store(v, reinterpret_cast<nv2*>(p));
  } else {
#pragma unroll
    for (int k = 0; k < CPL; ++k) __builtin_nontemporal_store(x[k], p + k);
  }
}

// x as held by lane u of the caller's group of W lanes (groups of W
// consecutive lanes, W = 1, 2, 4, 8 or 16), with u known once the caller's
// loop is unrolled.  The CSR entries a group loads are passed round this way:
// DPP moves on the vector ALU, without the round trip through the LDS unit
// that a bpermute-based shuffle takes (and that pass 1 shares with its Gram
// staging).  quad_perm covers W <= 4; row_newbcast (lane u of each row of 16
// lanes) covers W = 16, and W = 8 applies it to each half row in turn under
// a bank mask.  Every lane of a group must be active.
template <int W, int U, typename T>
__device__ inline T grp_bcast_c(T x) {
  static_assert(U >= 0 && U < W, "lane outside the group");
  if constexpr (W == 1) {
    return x;
  } else if constexpr (W == 2) {
    return __builtin_amdgcn_update_dpp(x, x, U | (U << 2) | ((2 + U) << 4) | ((2 + U) << 6), 0xF, 0xF, false);
  } else if constexpr (W == 4) {
    return __builtin_amdgcn_update_dpp(x, x, U * 0x55, 0xF, 0xF, false);
  } else if constexpr (W == 8) {
    const T t = __builtin_amdgcn_update_dpp(x, x, 0x150 + U, 0xF, 0x3, false);
    return __builtin_amdgcn_update_dpp(t, x, 0x158 + U, 0xF, 0xC, false);
  } else {
    static_assert(W == 16, "group width");
    return __builtin_amdgcn_update_dpp(x, x, 0x150 + U, 0xF, 0xF, false);
  }
}

template <int W, typename T>
__device__ inline T grp_bcast(T x, int u) {
  switch (u & (W - 1)) {
#define BMR_BC(k) \
  case k:         \
    if constexpr (k < W) return grp_bcast_c<W, k < W ? k : 0>(x);
    BMR_BC(0) BMR_BC(1) BMR_BC(2) BMR_BC(3) BMR_BC(4) BMR_BC(5) BMR_BC(6) BMR_BC(7)
    BMR_BC(8) BMR_BC(9) BMR_BC(10) BMR_BC(11) BMR_BC(12) BMR_BC(13) BMR_BC(14) BMR_BC(15)
#undef BMR_BC
    default:
      return x;
  }
}

// With fewer than 8 lanes per row (the group layout for p <= 8) a stencil
// row spans two chunks of CSR entries.  Their index and value loads are
// issued together ("lead" entries: s + c and s + LPR + c for lane c), and
// the gathered V rows of both chunks are loaded before any is consumed.
__host__ __device__ constexpr bool has_lead(int lpr) { return lpr > 1 && lpr < 8; }

template <typename T>
struct Lead {
  int colA, colB;
  T vA, vB;
};

template <int LPR, typename T>
__device__ inline void load_lead(const int32_t* __restrict__ ci, const T* __restrict__ va, int s, int e, int c,
                                 Lead<T>& q) {
  q.colA = q.colB = 0;
  q.vA = q.vB = T(0);
  if (s + c < e) {
    q.colA = ldnt(ci + s + c);
    q.vA = ldnt(va + s + c);
  }
  if (s + LPR + c < e) {
    q.colB = ldnt(ci + s + LPR + c);
    q.vB = ldnt(va + s + LPR + c);
  }
}

// acc[k] = sum over the entries of `row` of val * V[col*P + c0 + k], in CSR
// order (c0 = c * CPL).  In the group layout all lanes of a group call this
// with the same row; lanes whose columns lie beyond p return zeros.  With OWN,
// ov[0 .. CPL) also receives own[0 .. CPL) (zeros for own == nullptr), loaded
// together with the gathered rows.  With PIPE (lead layouts only), *lead
// holds this row's lead entries on entry and receives those of the entries
// [s_nx, e_nx) of the next row on return, loaded while the gathered rows are
// in flight.  mid() issues the caller's own loads: after the gathered loads
// with PIPE, before the gather otherwise, so that they share a round trip.
struct NoLoads {
  __device__ void operator()() const {}
};

template <int P, int LPR, int CPL, bool OWN = false, bool PIPE = false, typename T, typename Mid = NoLoads>
__device__ inline void gather_se(const int32_t* __restrict__ ci, const T* __restrict__ va, const T* __restrict__ V,
                                 int s, int e, int c, T (&acc)[CPL], const T* __restrict__ own = nullptr,
                                 T* ov = nullptr, Lead<T>* lead = nullptr, int s_nx = 0, int e_nx = 0,
                                 const Mid& mid = Mid());

template <int CPL, typename T>
__device__ inline void load_own(const T* __restrict__ own, T* ov) {
  if (own) {
    T x[CPL];
    vload<CPL>(own, x);
#pragma unroll
    for (int k = 0; k < CPL; ++k) ov[k] = x[k];
  } else {
#pragma unroll
    for (int k = 0; k < CPL; ++k) ov[k] = T(0);
  }
}

template <int P, int LPR, int CPL, typename T>
__device__ inline void gather_row(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const T* __restrict__ va, const T* __restrict__ V, int64_t row, bool valid, int c,
                                  T (&acc)[CPL]) {
  int s = 0, e = 0;
  if (valid) {
    s = rp[row];
    e = rp[row + 1];
  }
  gather_se<P, LPR, CPL>(ci, va, V, s, e, c, acc);
}

// the entries [s, e) of one row (s = e for an invalid row)
template <int P, int LPR, int CPL, bool OWN, bool PIPE, typename T, typename Mid>
__device__ inline void gather_se(const int32_t* __restrict__ ci, const T* __restrict__ va, const T* __restrict__ V,
                                 int s, int e, int c, T (&acc)[CPL], const T* __restrict__ own, T* ov,
                                 Lead<T>* lead, int s_nx, int e_nx, const Mid& mid) {
  constexpr bool PF = has_lead(LPR);
  if constexpr (!(PF && PIPE)) mid();
#pragma unroll
  for (int k = 0; k < CPL; ++k) acc[k] = T(0);
  if constexpr (LPR == 1) {
    if constexpr (OWN) load_own<CPL>(own, ov);
    constexpr int U = 8;
    for (int q = s; q < e; q += U) {
      int cq[U];
      T vq[U], x[U][CPL];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool in = q + u < e;
        cq[u] = in ? ci[q + u] : 0;
        vq[u] = in ? va[q + u] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (q + u < e) {
          vload<CPL>(V + (int64_t)cq[u] * P, x[u]);
        } else {
#pragma unroll
          for (int k = 0; k < CPL; ++k) x[u][k] = T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < CPL; ++k) acc[k] = fma(vq[u], x[u][k], acc[k]);
    }
  } else {
    constexpr int U = LPR < 8 ? LPR : 8;
    const bool mine = c * CPL < P;
    int base = s;
    if constexpr (PF) {
      Lead<T> cur;
      if constexpr (PIPE) {
        cur = *lead;
      } else {
        load_lead<LPR>(ci, va, s, e, c, cur);
      }
      // the two lead chunks form one batch: every gathered load of the
      // batch is issued before the first of them is consumed, so a row of up
      // to 2 * LPR entries costs one round trip to memory for its V rows
      // A wavefront about to issue its gather runs at raised priority until
      // the loads are out, so that the SIMD's arbiter lets the memory phase
      // of one wavefront start before the arithmetic of the others (pass 1
      // at 128^3: p = 8 0.1516 -> 0.1489 ms, p = 16 0.3908 -> 0.3873 ms;
      // with one lane per row it cost 2%, so that path keeps the default).
      __builtin_amdgcn_s_setprio(2);
      if constexpr (OWN) load_own<CPL>(own, ov);
      const int cnt = e - s;
      T x[2 * LPR][CPL];
#pragma unroll
      for (int u = 0; u < 2 * LPR; ++u) {
        const int cq = grp_bcast<LPR>(u < LPR ? cur.colA : cur.colB, u % LPR);
        if (u < cnt && mine) {
          vload<CPL>(V + (int64_t)cq * P + c * CPL, x[u]);
        } else {
#pragma unroll
          for (int k = 0; k < CPL; ++k) x[u][k] = T(0);
        }
      }
      if constexpr (PIPE) {
        load_lead<LPR>(ci, va, s_nx, e_nx, c, *lead);
        mid();
      }
      __builtin_amdgcn_s_setprio(0);
      // the values are passed round after the loads are in flight
#pragma unroll
      for (int u = 0; u < 2 * LPR; ++u) {
        const T vq = grp_bcast<LPR>(u < LPR ? cur.vA : cur.vB, u % LPR);
        const T co = u < cnt ? vq : T(0);
#pragma unroll
        for (int k = 0; k < CPL; ++k) acc[k] = fma(co, x[u][k], acc[k]);
      }
      base = s + 2 * LPR;
    } else if constexpr (OWN) {
      load_own<CPL>(own, ov);
    }
    for (; base < e; base += LPR) {
      const int idx = base + c;
      int col = 0;
      T v = T(0);
      if (idx < e) {
        col = ldnt(ci + idx);
        v = ldnt(va + idx);
      }
      // cnt > 0 here, so the first batch of U always runs: the compiler sees
      // that every loaded entry is consumed before the next row starts
      const int cnt = min(LPR, e - base);
#pragma unroll
      for (int h = 0; h < LPR / U; ++h) {
        if (h > 0 && h * U >= cnt) break;
        T x[U][CPL];
        __builtin_amdgcn_s_setprio(2);  // as for the lead entries above
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int cq = grp_bcast<LPR>(col, h * U + u);
          if (h * U + u < cnt && mine) {
            vload<CPL>(V + (int64_t)cq * P + c * CPL, x[u]);
          } else {
#pragma unroll
            for (int k = 0; k < CPL; ++k) x[u][k] = T(0);
          }
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const T vq = grp_bcast<LPR>(v, h * U + u);
          const T co = h * U + u < cnt ? vq : T(0);
#pragma unroll
          for (int k = 0; k < CPL; ++k) acc[k] = fma(co, x[u][k], acc[k]);
        }
      }
    }
  }
}

// Contiguous row range [r0, r1) of logical workgroup L out of n_wg, in whole
// workgroup steps of RPG rows.
template <int RPG>
__device__ inline void row_range(int64_t n, int n_wg, int L, int64_t& r0, int64_t& r1) {
  const int64_t steps = (n + RPG - 1) / RPG;
  const int64_t per = (steps + n_wg - 1) / n_wg;
  r0 = (int64_t)L * per * RPG;
  r1 = min(n, r0 + per * RPG);
}

// Row pointers and lead CSR entries of the row steps ahead of a lane's
// current row, for a workgroup that walks its row range in steps of RPG.
// Row pointers are loaded one step ahead; in the lead layouts the lead
// entries of the next step are loaded during the gather of the current one
// (gather_se with PIPE), which needs the row pointers two steps ahead.
template <int LPR, int RPG, typename T>
struct RowPipe {
  static constexpr bool PIPE = has_lead(LPR);
  int s_cur = 0, e_cur = 0, s_nx = 0, e_nx = 0, s_ahead = 0, e_ahead = 0;
  Lead<T> lead;

  __device__ void start(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, const T* __restrict__ va,
                        int64_t row, int64_t r1, int c) {
    if (row < r1) {
      s_cur = rp[row];
      e_cur = rp[row + 1];
    }
    if constexpr (PIPE) {
      if (row + RPG < r1) {
        s_nx = rp[row + RPG];
        e_nx = rp[row + RPG + 1];
      }
      load_lead<LPR>(ci, va, s_cur, e_cur, c, lead);
      // wait once here, so that the loop does not wait for the lead loads
      // (and with them for the previous step's stores) at every step
      __builtin_amdgcn_s_waitcnt(0);
    }
  }
  // row pointers of the step after the ones already held (row: current row)
  __device__ void load_ahead(const int32_t* __restrict__ rp, int64_t row, int64_t r1) {
    const int64_t ra = row + (PIPE ? 2 : 1) * RPG;
    s_ahead = e_ahead = 0;
    if (ra < r1) {
      s_ahead = rp[ra];
      e_ahead = rp[ra + 1];
    }
  }
  __device__ void advance() {
    if constexpr (PIPE) {
      s_cur = s_nx;
      e_cur = e_nx;
      s_nx = s_ahead;
      e_nx = e_ahead;
    } else {
      s_cur = s_ahead;
      e_cur = e_ahead;
    }
  }
};

// Sum x over the groups of a wavefront (lanes with equal c); the result is
// valid in every lane.
template <int LPR, typename T>
__device__ inline T group_sum(T x) {
#pragma unroll
  for (int o = LPR; o < 64; o <<= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// OPM selects the operator product the pass starts from:
//   OP_GATHER  A V_k, gathered through the CSR (rp, ci, va) from V_k;
//   OP_IDENT   formed beforehand (the preconditioned operator) and read row
//              by row from Z;
//   OP_TRI     the forward solve of a two-level IC(0) factor applied to Z on
//              the fly: (Z_i - sum_e va_e Z_(ci_e)) / diag_i, the CSR being the
//              factor's strictly lower part with its coefficients divided by
//              the pivots of the rows they multiply.
enum { OP_GATHER = 0, OP_IDENT = 1, OP_TRI = 2 };
template <int P, typename T, int OPM = OP_GATHER>
__global__ __launch_bounds__(WG) void k_pass1(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                              const T* __restrict__ va, int64_t n, T* __restrict__ Vbase,
                                              size_t slot, const T* __restrict__ bench,
                                              double* __restrict__ part, int n_wg, DevState* __restrict__ st,
                                              const T* __restrict__ Z = nullptr,
                                              const T* __restrict__ diag = nullptr) {
  constexpr bool IDENT = OPM == OP_IDENT;
  if (st->halt) return;
  using LN = Lanes<P>;
  using Ops = TypeOps<T>;
  using acc4 = typename Ops::acc4;
  constexpr int LPR = LN::LPR, CPL = LN::CPL, RPW = LN::RPW, RPG = LN::RPG;
  const int64_t k = st->k;
  constexpr int R = ring_len(P);
  const T* __restrict__ V = Vbase + (size_t)(k % R) * slot;
  const T* __restrict__ Vp = Vbase + (size_t)((k + R - 1) % R) * slot;  // V_{k-1}
  T* __restrict__ W = Vbase + (size_t)((k + 1) % R) * slot;             // becomes V_{k+1}
  const int nb = st->nb, taken = st->taken;
  const bool live_bench = taken < nb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = lane / LPR, c = lane % LPR;
  const int c0 = c * CPL;  // first column of this lane

  // LDS: B_{k-1} (padded against bank conflicts), then one region that holds
  // the per-wavefront staging of [V_k W], V_{k-1} and the bench rows (type T)
  // during the row loop and the per-wavefront partial sums (double) afterwards
  constexpr int SR = LN::ROW ? 1 : RPW;  // staged rows per wavefront
  constexpr int SC = P <= 8 ? 8 : 16;    // staged columns of V_k and W
  constexpr int STAGE = (SR * (2 * SC + P + MAXB) * (int)sizeof(T) + 7) / 8;
  constexpr int NEP = n_entries(P, MAXB);
  constexpr int PER_WAVE = STAGE > NEP ? STAGE : NEP;
  __shared__ T sBp[P][P + 1];
  __shared__ double smem[WG / 64][PER_WAVE];
  T* sv = reinterpret_cast<T*>(smem[wave]);  // [SR][SC]
  T* sw = sv + SR * SC;                      // [SR][SC]
  T* svp = sw + SR * SC;                     // [SR][P]
  T* sg = svp + SR * P;                      // [SR][MAXB]
  for (int e = tid; e < P * P; e += WG) sBp[e / P][e % P] = (T)st->Bprev[(e / P) * MAXP + (e % P)];
  __syncthreads();

  T aA[CPL];
  // one-lane-per-row (p <= 2) accumulators
  T lG[CPL][CPL], lQ[CPL][CPL], lP[CPL][CPL], lWg[CPL][MAXB], lVg[CPL][MAXB];
  // matrix-core accumulators: p <= 8: m0 = X^T X, m1 = X^T g with X = [V_k W];
  // p > 8: V^T V, V^T W, W^T W, V^T g, W^T g
  acc4 m0 = {0, 0, 0, 0}, m1 = {0, 0, 0, 0}, m2 = {0, 0, 0, 0}, m3 = {0, 0, 0, 0}, m4 = {0, 0, 0, 0};
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    aA[cc] = T(0);
#pragma unroll
    for (int r = 0; r < CPL; ++r) lG[cc][r] = lQ[cc][r] = lP[cc][r] = T(0);
#pragma unroll
    for (int b = 0; b < MAXB; ++b) lWg[cc][b] = lVg[cc][b] = T(0);
  }

  int64_t r0, r1;
  row_range<RPG>(n, n_wg, blockIdx.x, r0, r1);
  RowPipe<LPR, RPG, T> pipe;
  if constexpr (!IDENT) pipe.start(rp, ci, va, r0 + wave * RPW + grp, r1, c);

  for (int64_t base = r0; base < r1; base += RPG) {
    asm volatile("" ::: "memory");
    const int64_t row = base + wave * RPW + grp;
    const bool valid = row < r1;
    // The row pointers ahead, the row's V_{k-1} and bench entries travel
    // together with the gathered rows (or the CSR entries without the
    // pipeline); its own V_k row is loaded with the gathered rows.
    T v[CPL], w[CPL], vpo[CPL], vp[LN::ROW ? P : 1], g[LN::ROW ? MAXB : 1], gb = T(0);
    T zr[OPM == OP_TRI ? CPL : 1], dr = T(1);
    auto loads = [&]() {
      if constexpr (!IDENT) pipe.load_ahead(rp, row, r1);
      if constexpr (OPM == OP_TRI) {  // the row's own entries of Z and its pivot
        load_own<CPL>((valid && c0 < P) ? Z + row * P + c0 : nullptr, zr);
        if (valid) dr = diag[row];
      }
      if constexpr (LN::ROW) {
#pragma unroll
        for (int r = 0; r < P; ++r) vp[r] = valid ? Vp[row * P + r] : T(0);
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
          g[b] = (live_bench && b >= taken && b < nb && valid) ? bench[row * nb + b] : T(0);
      } else {
        if (valid && c0 < P) {
          vload_nt<CPL>(Vp + row * P + c0, vpo);
        } else {
#pragma unroll
          for (int cc = 0; cc < CPL; ++cc) vpo[cc] = T(0);
        }
        if (c < MAXB && live_bench && c >= taken && c < nb && valid) gb = ldnt(bench + row * nb + c);
      }
    };
    T a[CPL];
    const T* own = (valid && c0 < P) ? V + row * P + c0 : nullptr;
    if constexpr (IDENT) {
      loads();
      load_own<CPL>(own, v);
      load_own<CPL>((valid && c0 < P) ? Z + row * P + c0 : nullptr, a);
    } else {
      // OP_TRI gathers from Z through the factor's pattern, the others from V_k
      const T* src = OPM == OP_TRI ? Z : V;
      gather_se<P, LPR, CPL, true, RowPipe<LPR, RPG, T>::PIPE>(ci, va, src, pipe.s_cur, pipe.e_cur, c, a, own, v,
                                                               &pipe.lead, pipe.s_nx, pipe.e_nx, loads);
      pipe.advance();
      if constexpr (OPM == OP_TRI) {
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) a[cc] = (zr[cc] - a[cc]) / dr;
      }
    }
    if constexpr (LN::ROW) {
      // the lane owns the whole row: everything stays in registers
#pragma unroll
      for (int col = 0; col < P; ++col) {
        T t = a[col];
#pragma unroll
        for (int r = col; r < P; ++r) t = fma(-sBp[col][r], vp[r], t);
        w[col] = t;
        if (valid) W[row * P + col] = t;
        aA[col] = fma(a[col], a[col], aA[col]);
      }
#pragma unroll
      for (int r = 0; r < CPL; ++r)
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
          lG[r][cc] = fma(v[r], w[cc], lG[r][cc]);
          lQ[r][cc] = fma(w[r], w[cc], lQ[r][cc]);
          lP[r][cc] = fma(v[r], v[cc], lP[r][cc]);
        }
      if (live_bench) {
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc)
#pragma unroll
          for (int b = 0; b < MAXB; ++b) {
            lWg[cc][b] = fma(w[cc], g[b], lWg[cc][b]);
            lVg[cc][b] = fma(v[cc], g[b], lVg[cc][b]);
          }
      }
    } else {
      // stage this lane's columns of V_k and V_{k-1} and its bench entry
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc)
        if (c0 + cc < P) {
          sv[grp * SC + c0 + cc] = v[cc];
          svp[grp * P + c0 + cc] = vpo[cc];
        }
      if (c < MAXB) sg[grp * MAXB + c] = gb;
      __builtin_amdgcn_wave_barrier();
      // known coefficients by symmetry: column l loses sum_{r >= l} B_{k-1}(l, r) V_{k-1}(:, r)
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        const int col = c0 + cc;
        T t = a[cc];
#pragma unroll
        for (int r = 0; r < P; ++r)
          if (r >= col && col < P) t = fma(-sBp[col][r], svp[grp * P + r], t);
        w[cc] = t;
        if (col < P) sw[grp * SC + col] = t;
        aA[cc] = fma(a[cc], a[cc], aA[cc]);
      }
      if (valid && c0 < P) vstore_nt<CPL>(W + row * P + c0, w);
      __builtin_amdgcn_wave_barrier();
      // Gram products on the matrix cores, four staged rows per product
      const int m = lane % 16, rq = lane / 16;
#pragma unroll
      for (int h = 0; h < RPW / 4; ++h) {
        const int rl = 4 * h + rq;
        const T y = (m < MAXB) ? sg[rl * MAXB + m] : T(0);  // bench columns (zero when used up)
        if constexpr (P <= 8) {
          // X = [V_k | W] as 16 columns (zero padded)
          const T x = (m < 8) ? ((m < P) ? sv[rl * SC + m] : T(0)) : ((m - 8 < P) ? sw[rl * SC + m - 8] : T(0));
          m0 = Ops::mfma(x, x, m0);
          if (live_bench) m1 = Ops::mfma(x, y, m1);
        } else {
          const T xv = (m < P) ? sv[rl * SC + m] : T(0), xw = (m < P) ? sw[rl * SC + m] : T(0);
          m0 = Ops::mfma(xv, xv, m0);  // V^T V
          m1 = Ops::mfma(xv, xw, m1);  // V^T W
          m2 = Ops::mfma(xw, xw, m2);  // W^T W
          if (live_bench) {
            m3 = Ops::mfma(xv, y, m3);  // V^T g
            m4 = Ops::mfma(xw, y, m4);  // W^T g
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }

  // ---- workgroup reduction: deterministic order --------------------------
  __syncthreads();  // the partial sums reuse the staging region
  const int ne = n_entries(P, nb);
  double* s = smem[wave];
  for (int e = lane; e < ne; e += 64) s[e] = 0.0;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) aA[cc] = group_sum<LPR>(aA[cc]);
  if constexpr (LN::ROW) {
#pragma unroll
    for (int r = 0; r < CPL; ++r)
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        lG[r][cc] = group_sum<1>(lG[r][cc]);
        lQ[r][cc] = group_sum<1>(lQ[r][cc]);
        lP[r][cc] = group_sum<1>(lP[r][cc]);
      }
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc)
#pragma unroll
      for (int b = 0; b < MAXB; ++b) {
        lWg[cc][b] = group_sum<1>(lWg[cc][b]);
        lVg[cc][b] = group_sum<1>(lVg[cc][b]);
      }
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < CPL; ++r)
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
          s[off_G(P) + r * P + cc] = lG[r][cc];
          s[off_Q(P) + r * P + cc] = lQ[r][cc];
          s[off_P(P) + r * P + cc] = lP[r][cc];
        }
      for (int cc = 0; cc < CPL; ++cc)
        for (int b = 0; b < nb; ++b) {
          s[off_Wg(P) + cc * nb + b] = lWg[cc][b];
          s[off_Vg(P, nb) + cc * nb + b] = lVg[cc][b];
        }
    }
  } else {
    const int colD = lane % 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rowD = Ops::acc_row(lane, i);
      if constexpr (P <= 8) {
        const double d = m0[i];
        if (rowD < P && colD < P) s[off_P(P) + rowD * P + colD] = d;
        if (rowD < P && colD >= 8 && colD - 8 < P) s[off_G(P) + rowD * P + colD - 8] = d;
        if (rowD >= 8 && rowD - 8 < P && colD >= 8 && colD - 8 < P) s[off_Q(P) + (rowD - 8) * P + colD - 8] = d;
        if (colD < nb) {
          if (rowD < P) s[off_Vg(P, nb) + rowD * nb + colD] = m1[i];
          if (rowD >= 8 && rowD - 8 < P) s[off_Wg(P) + (rowD - 8) * nb + colD] = m1[i];
        }
      } else {
        if (rowD < P && colD < P) {
          s[off_P(P) + rowD * P + colD] = m0[i];
          s[off_G(P) + rowD * P + colD] = m1[i];
          s[off_Q(P) + rowD * P + colD] = m2[i];
        }
        if (rowD < P && colD < nb) {
          s[off_Vg(P, nb) + rowD * nb + colD] = m3[i];
          s[off_Wg(P) + rowD * nb + colD] = m4[i];
        }
      }
    }
  }
  if (grp == 0) {
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      const int col = c0 + cc;
      if (col < P) s[off_a(P) + col] = aA[cc];
    }
  }
  __syncthreads();
  for (int e = tid; e < ne; e += WG) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < WG / 64; ++q) t += smem[q][e];
    part[(size_t)e * n_wg + blockIdx.x] = t;
  }
}

// The gathers of two rows interleaved, for the layouts with several lanes per
// row: the CSR entries of both rows' first chunk (2 LPR entries with lead
// entries, LPR otherwise) are loaded together, then every gathered load of
// both chunks is issued before the first is consumed, so each lane group
// keeps two independent load chains in flight.  Entries beyond the first
// chunk follow row by row.  Each row accumulates in CSR order, as gather_se
// does, so the sums are bitwise those of two gather_se calls.
template <int P, int LPR, int CPL, typename T>
__device__ inline void gather_pair(const int32_t* __restrict__ ci, const T* __restrict__ va, const T* __restrict__ V,
                                   const int (&s)[2], const int (&e)[2], int c, T (&acc)[2][CPL]) {
  constexpr int NL = has_lead(LPR) ? 2 : 1;  // CSR entries per lane in the first chunk
  constexpr int CH = NL * LPR;               // entries of a row in the first chunk
  const bool mine = c * CPL < P;
  int col[2][NL];
  T v[2][NL];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int h = 0; h < NL; ++h) {
      const int idx = s[r] + h * LPR + c;
      col[r][h] = 0;
      v[r][h] = T(0);
      if (idx < e[r]) {
        col[r][h] = ldnt(ci + idx);
        v[r][h] = ldnt(va + idx);
      }
    }
  T x[2][CH][CPL];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int cq = grp_bcast<LPR>(col[r][u / LPR], u % LPR);
      if (u < e[r] - s[r] && mine) {
        vload<CPL>(V + (int64_t)cq * P + c * CPL, x[r][u]);
      } else {
#pragma unroll
        for (int k = 0; k < CPL; ++k) x[r][u][k] = T(0);
      }
    }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
#pragma unroll
    for (int k = 0; k < CPL; ++k) acc[r][k] = T(0);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const T vq = grp_bcast<LPR>(v[r][u / LPR], u % LPR);
      const T co = u < e[r] - s[r] ? vq : T(0);
#pragma unroll
      for (int k = 0; k < CPL; ++k) acc[r][k] = fma(co, x[r][u][k], acc[r][k]);
    }
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    for (int base = s[r] + CH; base < e[r]; base += LPR) {
      const int idx = base + c;
      int cl = 0;
      T vl = T(0);
      if (idx < e[r]) {
        cl = ldnt(ci + idx);
        vl = ldnt(va + idx);
      }
      const int cnt = min(LPR, e[r] - base);
      T y[LPR][CPL];
#pragma unroll
      for (int u = 0; u < LPR; ++u) {
        const int cq = grp_bcast<LPR>(cl, u);
        if (u < cnt && mine) {
          vload<CPL>(V + (int64_t)cq * P + c * CPL, y[u]);
        } else {
#pragma unroll
          for (int k = 0; k < CPL; ++k) y[u][k] = T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < LPR; ++u) {
        const T vq = grp_bcast<LPR>(vl, u);
        const T co = u < cnt ? vq : T(0);
#pragma unroll
        for (int k = 0; k < CPL; ++k) acc[r][k] = fma(co, y[u][k], acc[r][k]);
      }
    }
  }
}

// Shape of the standalone block operator, chosen per layout by measurement
// (128^3 7-point Laplacian, FP64, every shape on one box; the results are
// bitwise equal).  Two rows per lane group (gather_pair) pay where each lane
// holds two columns of a 4-lane row group (p = 6, 8: 105 -> 100-103 us at
// p = 8); with one column per lane, or 8-16 lanes per row, the second chain
// costs more in registers than it hides (p = 16: 161 -> 168-180 us).  With
// slabs, workgroup b (which runs on XCD b mod 8) takes logical range
// (b mod 8) * (n_wg / 8) + b / 8, so consecutive ranges share one XCD's L2:
// one lane per row gains (p = 1: 53.9 -> 50.5 us, p = 2: 60.0 -> 55.3 us),
// the 8- and 16-lane layouts lose (p = 12: 132 -> 137-140 us), and the paired
// layouts are level or gain.
__host__ __device__ constexpr int spmm_rows(int p) { return layout_lpr(p) == 4 && layout_cpl(p) == 2 ? 2 : 1; }
__host__ __device__ constexpr bool spmm_slab(int p) { return layout_lpr(p) == 1 || spmm_rows(p) == 2; }

template <int P, typename T>
__global__ __launch_bounds__(WG) void k_spmm(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                             const T* __restrict__ va, int64_t n, const T* __restrict__ V,
                                             T* __restrict__ W, int n_wg, const DevState* __restrict__ st) {
  if (st && st->halt) return;
  using LN = Lanes<P>;
  constexpr int LPR = LN::LPR, CPL = LN::CPL, RPW = LN::RPW, RPG = LN::RPG;
  constexpr int ROWS = spmm_rows(P);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / LPR, c = lane % LPR, c0 = c * CPL;
  const int L = spmm_slab(P) ? (int)(blockIdx.x % 8) * (n_wg / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  int64_t r0, r1;
  row_range<ROWS * RPG>(n, n_wg, L, r0, r1);
  for (int64_t base = r0; base < r1; base += ROWS * RPG) {
    if constexpr (ROWS == 2) {
      const int64_t row[2] = {base + wave * RPW + grp, base + RPG + wave * RPW + grp};
      int s[2] = {0, 0}, e[2] = {0, 0};
#pragma unroll
      for (int r = 0; r < 2; ++r)
        if (row[r] < r1) {
          s[r] = rp[row[r]];
          e[r] = rp[row[r] + 1];
        }
      T a[2][CPL];
      gather_pair<P, LPR, CPL>(ci, va, V, s, e, c, a);
#pragma unroll
      for (int r = 0; r < 2; ++r)
        if (row[r] < r1 && c0 < P) vstore_nt<CPL>(W + row[r] * P + c0, a[r]);
    } else {
      const int64_t row = base + wave * RPW + grp;
      const bool valid = row < r1;
      T a[CPL];
      gather_row<P, LPR, CPL>(rp, ci, va, V, row, valid, c, a);
      if (valid && c0 < P) vstore_nt<CPL>(W + row * P + c0, a);
    }
  }
}

// A triangular solve of a two-level IC(0) factor in one launch (out of
// place): y_i = (rhs_i - sum_e va_e rhs_(ci_e)) / diag_i for every row, where
// (rp, ci, va) is the factor's strictly lower or upper part with each
// coefficient divided by the pivot of the row it multiplies (every row with
// entries refers only to rows without any, whose solution is rhs / diag).
// The gather is the block operator's; the halt flag of st (when given) makes
// it a no-op.
template <int P>
__global__ __launch_bounds__(WG) void k_trisolve2(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                  const double* __restrict__ va, const double* __restrict__ diag,
                                                  int64_t n, const double* __restrict__ rhs,
                                                  double* __restrict__ y, int n_wg, const DevState* __restrict__ st) {
  if (st && st->halt) return;
  using LN = Lanes<P>;
  constexpr int LPR = LN::LPR, CPL = LN::CPL, RPW = LN::RPW, RPG = LN::RPG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / LPR, c = lane % LPR, c0 = c * CPL;
  int64_t r0, r1;
  row_range<RPG>(n, n_wg, blockIdx.x, r0, r1);
  for (int64_t base = r0; base < r1; base += RPG) {
    const int64_t row = base + wave * RPW + grp;
    const bool valid = row < r1;
    double a[CPL], own[CPL];
    load_own<CPL>((valid && c0 < P) ? rhs + row * P + c0 : nullptr, own);
    const double d = valid ? diag[row] : 1.0;
    gather_row<P, LPR, CPL>(rp, ci, va, rhs, row, valid, c, a);
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) a[cc] = (own[cc] - a[cc]) / d;
    if (valid && c0 < P) vstore<CPL>(y + row * P + c0, a);
  }
}

// R = B - A X and per-workgroup partial sums of the squared column norms, in
// FP64 (it is also the outer residual of the mixed-precision solver).
template <int P>
__global__ __launch_bounds__(WG) void k_residual(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const double* __restrict__ va, int64_t n,
                                                 const double* __restrict__ Bm, const double* __restrict__ X,
                                                 double* __restrict__ R, double* __restrict__ part, int n_wg) {
  using LN = Lanes<P>;
  constexpr int LPR = LN::LPR, CPL = LN::CPL, RPW = LN::RPW, RPG = LN::RPG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / LPR, c = lane % LPR, c0 = c * CPL;
  int64_t r0, r1;
  row_range<RPG>(n, n_wg, blockIdx.x, r0, r1);
  double acc[CPL];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) acc[cc] = 0.0;
  for (int64_t base = r0; base < r1; base += RPG) {
    const int64_t row = base + wave * RPW + grp;
    const bool valid = row < r1;
    double ax[CPL];
    gather_row<P, LPR, CPL>(rp, ci, va, X, row, valid, c, ax);
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) {
      if (valid && c0 + cc < P) {
        const double r = Bm[row * P + c0 + cc] - ax[cc];
        if (R) R[row * P + c0 + cc] = r;
        acc[cc] = fma(r, r, acc[cc]);
      }
    }
  }
  __shared__ double sh[WG / 64][16];
#pragma unroll
  for (int cc = 0; cc < CPL; ++cc) {
    acc[cc] = group_sum<LPR>(acc[cc]);
    if (grp == 0 && c0 + cc < P) sh[wave][c0 + cc] = acc[cc];
  }
  __syncthreads();
  if (threadIdx.x < P) {
    double t = 0.0;
    for (int q = 0; q < WG / 64; ++q) t += sh[q][threadIdx.x];
    part[(size_t)threadIdx.x * n_wg + blockIdx.x] = t;
  }
}

}  // namespace

int pass1_grid(int64_t n, int p) {
  // one workgroup step of the row layout each, at most PASS1_MAX_WG
  // workgroups so that the partial sums stay small
  int64_t g = (n + layout_rpg(p) - 1) / layout_rpg(p);
  if (g > PASS1_MAX_WG) g = PASS1_MAX_WG;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename T>
int pass1_resident_grid(int64_t n, int p) {
  // One round of workgroups: as many as the device holds at once
  // (occupancy x compute units), at most pass1_grid(n, p).  A second,
  // partial round left a tail (at 128^3 against 2048 workgroups: p = 8 FP32
  // 0.106 -> 0.100 ms, p = 16 FP64 0.441 -> 0.395 ms).  With one lane per
  // row (p <= 2) two rounds measured faster (p = 1: 0.074 against
  // 0.079 ms), so those keep pass1_grid.
  const int g = pass1_grid(n, p);
  if (layout_cpl(p) == p) return g;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return g;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return g;
  hipError_t e = hipErrorInvalidValue;
#define OC(P) \
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_pass1<P, T>), WG, 0)
  switch (p) {
    case 1: OC(1); break;
    case 2: OC(2); break;
    case 3: OC(3); break;
    case 4: OC(4); break;
    case 5: OC(5); break;
    case 6: OC(6); break;
    case 7: OC(7); break;
    case 8: OC(8); break;
    case 9: OC(9); break;
    case 10: OC(10); break;
    case 11: OC(11); break;
    case 12: OC(12); break;
    case 13: OC(13); break;
    case 14: OC(14); break;
    case 15: OC(15); break;
    case 16: OC(16); break;
    default: break;
  }
#undef OC
  if (e != hipSuccess || per < 1 || cus < 1) return g;
  const int64_t resident = (int64_t)per * cus;
  return (int)std::min<int64_t>(g, resident);
}
template int pass1_resident_grid<double>(int64_t, int);
template int pass1_resident_grid<float>(int64_t, int);

static int step_grid(int64_t n, int p) {
  // one workgroup step each: a grid that walks longer row ranges with the
  // pass-1 pipeline measured slower for the plain product
  return (int)std::max<int64_t>(1, (n + layout_rpg(p) - 1) / layout_rpg(p));
}

static int spmm_grid(int64_t n, int p) {
  // one step of spmm_rows(p) row groups each; a multiple of 8 with slabs
  const int64_t rows = (int64_t)spmm_rows(p) * layout_rpg(p);
  int64_t g = std::max<int64_t>(1, (n + rows - 1) / rows);
  if (spmm_slab(p)) g = (g + 7) / 8 * 8;
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
hipError_t launch_pass1(int p, const bmr_csr_t& A, const T* val, T* Vbase, size_t slot, const T* bench, double* part,
                        int n_wg, DevState* st, hipStream_t s) {
#define L1(P)                                                                                                 \
  hipLaunchKernelGGL((k_pass1<P, T>), dim3(n_wg), dim3(WG), 0, s, A.row_ptr, A.col_idx, val, A.n, Vbase, slot, \
                     bench, part, n_wg, st)
  BMR_DISPATCH_P(p, L1)
#undef L1
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spmm(int p, const bmr_csr_t& A, const T* val, const T* V, T* W, hipStream_t s,
                       const DevState* st) {
  const int n_wg = spmm_grid(A.n, p);
#define L2(P) \
  hipLaunchKernelGGL((k_spmm<P, T>), dim3(n_wg), dim3(WG), 0, s, A.row_ptr, A.col_idx, val, A.n, V, W, n_wg, st)
  BMR_DISPATCH_P(p, L2)
#undef L2
  return hipGetLastError();
}

template hipError_t launch_pass1<double>(int, const bmr_csr_t&, const double*, double*, size_t, const double*,
                                         double*, int, DevState*, hipStream_t);
template hipError_t launch_pass1<float>(int, const bmr_csr_t&, const float*, float*, size_t, const float*, double*,
                                        int, DevState*, hipStream_t);
template hipError_t launch_spmm<double>(int, const bmr_csr_t&, const double*, const double*, double*, hipStream_t,
                                        const DevState*);
template hipError_t launch_spmm<float>(int, const bmr_csr_t&, const float*, const float*, float*, hipStream_t,
                                       const DevState*);

hipError_t launch_pass1_ident(int p, const double* Z, double* Vbase, size_t slot, const double* bench, double* part,
                              int n_wg, int64_t n, DevState* st, hipStream_t s) {
#define L4(P)                                                                                                   \
  hipLaunchKernelGGL((k_pass1<P, double, OP_IDENT>), dim3(n_wg), dim3(WG), 0, s, (const int32_t*)nullptr,      \
                     (const int32_t*)nullptr, (const double*)nullptr, n, Vbase, slot, bench, part, n_wg, st, Z,  \
                     (const double*)nullptr)
  BMR_DISPATCH_P(p, L4)
#undef L4
  return hipGetLastError();
}

hipError_t launch_trisolve2(int p, const int32_t* rp, const int32_t* ci, const double* va, const double* diag,
                            int64_t n, const double* rhs, double* y, const DevState* st, hipStream_t s) {
  const int n_wg = step_grid(n, p);
#define L6(P) \
  hipLaunchKernelGGL(k_trisolve2<P>, dim3(n_wg), dim3(WG), 0, s, rp, ci, va, diag, n, rhs, y, n_wg, st)
  BMR_DISPATCH_P(p, L6)
#undef L6
  return hipGetLastError();
}

hipError_t launch_pass1_tri(int p, const int32_t* lrp, const int32_t* lci, const double* lval_s, const double* diag,
                            const double* Z, double* Vbase, size_t slot, const double* bench, double* part, int n_wg,
                            int64_t n, DevState* st, hipStream_t s) {
#define L5(P)                                                                                                    \
  hipLaunchKernelGGL((k_pass1<P, double, OP_TRI>), dim3(n_wg), dim3(WG), 0, s, lrp, lci, lval_s, n, Vbase, slot, \
                     bench, part, n_wg, st, Z, diag)
  BMR_DISPATCH_P(p, L5)
#undef L5
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
