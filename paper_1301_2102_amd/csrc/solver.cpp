// Host driver and C ABI of libbmr (see include/bmr.h).
//
// One solve = set-up (column norms of B, substitute bench, column-wise
// CGS2 QR of B: F_0 = U_p S, eq. (3.2)), then block iterations, each four
// launches on the caller's stream:
//     pass 1   W = A V_k - V_{k-1} B_{k-1}^T and partial Gram products
//     reduce   partials -> p x p Grams (fixed order)
//     band     A_k, B_k, Givens QR of p columns, S-hat, residuals, stop test
//     pass 2   V_{k+1}, bench update, M_k, X += M_k Z_k
// The kernels read the block index from the device state, so batches of
// block iterations are enqueued back to back and the host only polls a small
// status record (double-buffered, pinned) between batches.  When the band
// kernel rejects the Gram route for a near-dependent block, the device loop
// halts; at its next poll the host enqueues that block's QR column by column
// (kernels_colqr.hip: the dependence test and bench substitution of
// Section 5.1 are decided on the device) and the rest of the block
// iteration, and goes on enqueueing without waiting for any of it.
//
// The block-iteration driver is a template over the storage type of the
// n-length data: double for BMR_PREC_FP64, float for the inner solves of
// BMR_PREC_MIXED, whose FP64 iterative-refinement loop (explicit residual,
// inner solve of A D = R, X += D) sits at the end of this file.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "bmr_internal.hpp"

namespace bmr {
namespace {

// The Gram route to the new block's QR is rejected (and the block is
// orthogonalised column by column instead) when a Cholesky pivot falls below
// tau_fb * ||A u_j||.  With FP32 Gram products the pivot of a column that
// lost a fraction t of its norm carries a relative error of about
// 1e-6 / t^2, hence the larger threshold of the FP32 inner solve.
constexpr double TAU_FB = 1e-2;
constexpr double TAU_FB_F32 = 1e-1;
// Dependence tolerance floor of the FP32 inner solve.
constexpr double GAMMA_F32 = 1e-5;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
size_t slot_elems(int64_t n, int p) { return ((size_t)n * p + 31) / 32 * 32; }

static_assert(sizeof(bmr_opts_t) == 80 && sizeof(bmr_stats_t) == 488, "the Python binding mirrors these");

struct Ctl {  // leading fields of DevState polled by the host
  int halt, status, reason, taken;
  int64_t k, k2, j;
};
static_assert(offsetof(DevState, j) + sizeof(int64_t) == sizeof(Ctl), "Ctl must mirror DevState's head");

#define HIP_TRY(expr)                          \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return BMR_HIP_ERROR; \
  } while (0)

// Host side of a solve in storage type T: workspace pointers, stream,
// scratch for column sums.
template <typename T>
struct Run {
  const bmr_csr_t* A;
  const T* val;  // matrix values in T
  int p, nb;
  int64_t n;
  hipStream_t s;
  int n_wg;
  DevState* st;
  double *red, *part, *hist;
  T *V, *M, *bench;
  size_t slot;
  std::vector<double> hpart;
  // split preconditioning (FP64 only): the operator is C^{-1} A C^{-T},
  // formed block by block in Y (C^{-T} V_k) and Z (A Y, then C^{-1} in place)
  const Ic0View* pc = nullptr;
  double *Y = nullptr, *Z = nullptr;
  T* ret = nullptr;  // retained removed candidates (n x nb), or NULL
  // FP32 run after the switch of BMR_PREC_RELAXED: the search directions and
  // X stay FP64 (the flush reads the FP32 ring into FP64 sums)
  double *M64 = nullptr, *X64 = nullptr;

  T* Vslot(int64_t k) { return V + (size_t)(k % ring_len(p)) * slot; }

  // Column sums of k_coldots, summed on the host in workgroup order.
  template <typename U>
  int coldots(const U* Y, int ldy, int yc, const U* X, int ldx, int m, double* out) {
    const int g = coldots_grid(n);
    HIP_TRY(launch_coldots<U>(Y, ldy, yc, X, ldx, m, n, part, g, s));
    hpart.resize((size_t)g * (m + 1));
    HIP_TRY(hipMemcpyAsync(hpart.data(), part, sizeof(double) * hpart.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int r = 0; r <= m; ++r) {
      double t = 0.0;
      for (int w = 0; w < g; ++w) t += hpart[(size_t)w * (m + 1) + r];
      out[r] = t;
    }
    return 0;
  }
  // Column-wise QR of the block D on the device (launches only).
  int colqr(int mode, T* D, const T* Vk) {
    HIP_TRY(launch_colqr<T>(p, mode, D, Vk, bench, nb, n, part, colqr_grid(n), st, s, ret));
    return 0;
  }
};

#define TRY(expr)              \
  do {                         \
    int e_ = (expr);           \
    if (e_ != 0) return e_;    \
  } while (0)

}  // namespace

Layout layout_for(int64_t n, int64_t nnz, int p, int nb, int64_t hist_cap, int precision, int precond,
                  bool retain) {
  const bool mixed = precision == BMR_PREC_MIXED;
  const bool relaxed = precision == BMR_PREC_RELAXED;
  const size_t esz = mixed ? sizeof(float) : sizeof(double);
  Layout L{};
  L.n_wg = pass1_grid(n, p);
  size_t off = 0;
  L.off_state = off;
  off = align256(off + sizeof(DevState));
  L.off_red = off;
  off = align256(off + sizeof(double) * n_entries(MAXP, MAXB));
  size_t part = std::max<size_t>((size_t)n_entries(p, nb) * L.n_wg, (size_t)coldots_grid(n) * (MAXP + 1));
  part = std::max<size_t>(part, (size_t)colqr_grid(n) * std::max(MAXP, MAXB));
  part = std::max<size_t>(part, (size_t)p * L.n_wg);
  L.off_part = off;
  off = align256(off + sizeof(double) * part);
  L.off_hist = off;
  off = align256(off + (mixed ? 0 : sizeof(double) * (size_t)hist_cap * p));
  const size_t se = slot_elems(n, p);
  L.off_V = off;
  off = align256(off + esz * ring_len(p) * se);
  L.off_M = off;
  off = align256(off + esz * 2 * se);
  L.off_bench = off;
  off = align256(off + esz * (size_t)n * nb);
  if (mixed) {
    L.off_val32 = off;
    off = align256(off + sizeof(float) * (size_t)nnz);
    L.off_D = off;
    off = align256(off + sizeof(float) * (size_t)n * p);
    L.off_R = off;
    off = align256(off + sizeof(double) * (size_t)n * p);
  }
  if (relaxed) {
    L.off_V32 = off;
    off = align256(off + sizeof(float) * ring_len(p) * se);
    L.off_bench32 = off;
    off = align256(off + sizeof(float) * (size_t)n * nb);
    L.off_val32 = off;
    off = align256(off + sizeof(float) * (size_t)nnz);
  }
  if (retain) {
    L.off_ret = off;
    off = align256(off + esz * (size_t)n * nb);
  }
  if (precond == BMR_PRECOND_IC0) {
    L.off_Y = off;
    off = align256(off + sizeof(double) * (size_t)n * p);
    L.off_Z = off;
    off = align256(off + sizeof(double) * (size_t)n * p);
  }
  L.total = off;
  return L;
}

// R = B - A X (R may be NULL) and the column norms: per-workgroup partial
// sums (part: p * n_wg doubles of device scratch) added in a fixed order on
// the device into red (p doubles), then copied to the host.
int residual_norms(const bmr_csr_t* A, const double* B, const double* X, int p, double* R, double* part, int n_wg,
                   double* red, hipStream_t s, double* norms) {
  HIP_TRY(launch_residual(p, *A, B, X, R, part, n_wg, s));
  HIP_TRY(launch_reduce(part, n_wg, p, red, nullptr, 0, s));
  double h[MAXP];
  HIP_TRY(hipMemcpyAsync(h, red, sizeof(double) * p, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int c = 0; c < p; ++c) norms[c] = sqrt(h[c]);
  return 0;
}

}  // namespace bmr

using namespace bmr;

namespace {

bool opts_valid(const bmr_opts_t& o) {
  return o.tol > 0.0 && isfinite(o.tol) && o.max_iter >= 1 && o.gamma >= 0.0 && isfinite(o.gamma) &&
         o.n_bench >= 0 && o.n_bench <= BMR_MAX_BENCH && o.hist_cap >= 0 && o.poll_every >= 0 &&
         (o.precision == BMR_PREC_FP64 || o.precision == BMR_PREC_MIXED || o.precision == BMR_PREC_RELAXED) &&
         (o.precision != BMR_PREC_MIXED || (o.inner_tol > 0.0 && o.inner_tol < 1.0 && o.max_refine >= 1)) &&
         (o.precision != BMR_PREC_RELAXED ||
          ((o.relax_tol == 0.0 || (o.relax_tol > o.tol && o.relax_tol < 1.0)) && !(o.flags & BMR_FLAG_RETAIN))) &&
         (o.precond == BMR_PRECOND_NONE || (o.precond == BMR_PRECOND_IC0 && o.precision == BMR_PREC_FP64));
}

bool csr_valid(const bmr_csr_t* A) {
  return A && A->n >= 1 && A->n < (int64_t(1) << 31) && A->nnz >= 0 && A->nnz < (int64_t(1) << 31) &&
         A->row_ptr && (A->nnz == 0 || (A->col_idx && A->val));
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// The two pinned status records the host polls (the head of the state and,
// for the switch of BMR_PREC_RELAXED, the last residuals), allocated for one
// run of the block-iteration driver and freed at its end.
struct PinRec {
  Ctl ctl;
  double rho[MAXP];
};
struct PinnedCtl {
  PinRec* buf = nullptr;
  PinnedCtl() {
    void* p = nullptr;
    if (hipHostMalloc(&p, 2 * sizeof(PinRec), hipHostMallocDefault) == hipSuccess) buf = (PinRec*)p;
  }
  ~PinnedCtl() {
    if (buf) (void)hipHostFree(buf);
  }
  PinnedCtl(const PinnedCtl&) = delete;
  PinnedCtl& operator=(const PinnedCtl&) = delete;
};

// Parameters and results of one run of the block-iteration driver.
struct CoreParams {
  double tol, gamma, tau_fb;
  int64_t max_iter, hist_cap;
  uint64_t seed;
  int poll_every;
  bool prof;
  const double* beta_stop;  // per-column scale of the stopping test, or NULL for ||b_i||
  bool accumulate = false;  // apply the previous blocks' rotations as accumulated matrices
  // BMR_PREC_RELAXED.  switch_theta > 0: once every column's residual is
  // below it, run to the end of the current group of blocks and return
  // SWITCHED with the device state intact.  resume_k > 0: no set-up; the
  // device state (at the end of a group) goes on from block resume_k.
  double switch_theta = 0.0;
  int64_t resume_k = 0;
};
// Internal return of the driver: stopped for the switch to binary32.
constexpr int SWITCHED = 1000;
struct CoreOut {
  int64_t j = 0, k = 0;
  int n_replaced = 0, n_explicit = 0, n_kept = 0;
  double rho[MAXP] = {};
  double bnorm[MAXP] = {};  // ||b_i|| of the right-hand side solved
  double tk[4] = {0, 0, 0, 0};  // summed kernel times over n_prof block iterations
  int64_t n_prof = 0;
};

// Solve A X = B (X_0 = 0) with n-length data in T.  B is FP64 (the caller's
// right-hand side, or the residual of a refinement cycle).
template <typename T>
int solve_core(Run<T>& r, const double* B, T* X, const CoreParams& o, CoreOut& out, double* res_hist) {
  const int p = r.p, nb = r.nb;
  const int64_t n = r.n;
  DevState* hs = new DevState();
  struct Guard {
    DevState* p;
    ~Guard() { delete p; }
  } guard{hs};
  auto finish = [&](int64_t j, int64_t kblocks, const double* rho) {
    out.j = j;
    out.k = kblocks;
    out.n_replaced = hs->n_replaced;
    out.n_explicit = hs->n_explicit;
    out.n_kept = hs->n_kept;
    for (int i = 0; i < MAXP; ++i) out.rho[i] = (i < p && rho) ? rho[i] : 0.0;
  };
  if (o.resume_k > 0) {
    // the device state of a run stopped at SWITCHED: the ring, the search
    // directions, X and the bench go on as they are (nothing is cleared)
    HIP_TRY(hipMemcpyAsync(hs, r.st, sizeof(DevState), hipMemcpyDeviceToHost, r.s));
    HIP_TRY(hipStreamSynchronize(r.s));
    for (int i = 0; i < p; ++i) out.bnorm[i] = hs->beta[i];
  } else {
  // ---- set-up -------------------------------------------------------------
  HIP_TRY(launch_fill<T>(r.V, ring_len(p) * r.slot, T(0), r.s));
  HIP_TRY(launch_fill<T>(r.M, 2 * r.slot, T(0), r.s));
  HIP_TRY(launch_fill<T>(X, (size_t)n * p, T(0), r.s));
  HIP_TRY(launch_bench_init<T>(r.bench, n, nb, o.seed, r.s));
  memset(hs, 0, sizeof(DevState));
  hs->status = STATUS_RUNNING;
  hs->p = p;
  hs->nb = nb;
  hs->n = n;
  hs->max_iter = o.max_iter;
  hs->hist_cap = o.hist_cap;
  hs->tol = o.tol;
  hs->gamma = o.gamma;
  hs->tau_fb = o.tau_fb;
  hs->lcap = p;
  hs->k = 1;
  hs->retain = r.ret != nullptr;
  hs->accumulate = o.accumulate;

  double c[MAXP + 1];
  double bnorm[MAXP];
  for (int i = 0; i < p; ++i) {
    TRY(r.coldots(B, p, i, (const double*)nullptr, 0, 0, c));
    bnorm[i] = sqrt(c[0]);
    if (!isfinite(bnorm[i])) return BMR_NONFINITE;
    hs->beta[i] = o.beta_stop ? o.beta_stop[i] : bnorm[i];
    out.bnorm[i] = bnorm[i];
  }
  for (int b = 0; b < nb; ++b) {
    TRY(r.coldots(r.bench, nb, b, (const T*)nullptr, 0, 0, c));
    hs->bench_norm0[b] = sqrt(c[0]);
  }
  // initial QR of F_0 = B into V_1 (slot 1): copy (rounded to T), then
  // column-wise CGS2 on the device against the reference norms ||b_i||
  for (int i = 0; i < p; ++i) hs->qr_ref[i] = bnorm[i];
  HIP_TRY(hipMemcpyAsync(r.st, hs, sizeof(DevState), hipMemcpyHostToDevice, r.s));
  T* V1 = r.Vslot(1);
  if constexpr (sizeof(T) == sizeof(double)) {
    HIP_TRY(launch_copy(B, (double*)V1, (size_t)n * p, r.s));
  } else {
    HIP_TRY(launch_to_f32(B, V1, (size_t)n * p, r.s));
  }
  TRY(r.colqr(QR_SETUP, V1, nullptr));
  HIP_TRY(hipMemcpyAsync(hs, r.st, sizeof(DevState), hipMemcpyDeviceToHost, r.s));
  HIP_TRY(hipStreamSynchronize(r.s));
  if (hs->qr_error) return BMR_NONFINITE;
  if (hs->qr_lcap < p) {  // a dependent column found no substitute
    double one[MAXP];
    for (int i = 0; i < p; ++i) one[i] = hs->beta[i] > 0 ? 1.0 : 0.0;
    finish(0, 0, one);
    return BMR_BENCH_EXHAUSTED;
  }
  const double* S = hs->qr_R;
  // S-hat = E_1 S; stopping test at j = 0
  double worst = 0.0;
  for (int cidx = 0; cidx < p; ++cidx) {
    double ss = 0.0;
    for (int rr = 0; rr < p; ++rr) {
      hs->Shat[rr * MAXP + cidx] = S[rr * MAXP + cidx];
      ss += S[rr * MAXP + cidx] * S[rr * MAXP + cidx];
    }
    hs->rho[cidx] = hs->beta[cidx] > 0 ? sqrt(ss) / hs->beta[cidx] : 0.0;
    worst = std::max(worst, hs->rho[cidx]);
  }
  if (worst < o.tol) {
    finish(0, 0, hs->rho);
    return BMR_CONVERGED;
  }
  HIP_TRY(hipMemcpyAsync(r.st, hs, sizeof(DevState), hipMemcpyHostToDevice, r.s));
  }  // set-up

  // ---- block iterations -------------------------------------------------
  PinnedCtl pinned;
  PinRec* pin = pinned.buf;
  if (!pin) return BMR_HIP_ERROR;
  hipEvent_t ev[2];
  HIP_TRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
  } evg{ev};
  int batch = o.poll_every;
  if (batch <= 0) batch = r.pc ? 4 : ((double)n * p < 2e6) ? 32 : 16;
  const bool prof = o.prof;
  if (prof) batch = 1;
  hipEvent_t pev[2][5];
  if (prof)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 5; ++b) HIP_TRY(hipEventCreate(&pev[a][b]));
  struct PevGuard {
    hipEvent_t (*e)[5];
    bool on;
    ~PevGuard() {
      if (on)
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 5; ++b) (void)hipEventDestroy(e[a][b]);
    }
  } pevg{pev, prof};
  auto collect = [&](int slot) -> int {  // add the timings of the iteration in `slot`
    if (!prof) return 0;
    for (int q = 0; q < 4; ++q) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, pev[slot][q], pev[slot][q + 1]));
      out.tk[q] += ms;
    }
    ++out.n_prof;
    return 0;
  };

  // Enqueue `batch` block iterations, then a copy of the status record.
  // Every enqueued iteration is block kq of the device loop unless the loop
  // has halted (then its kernels return at once), so the host knows which
  // iterations end a group of search directions and enqueues the flush
  // after them; the flush checks the block number the band kernel recorded.
  const int grp = group_len(p);
  int64_t kq = o.resume_k > 0 ? o.resume_k : 1;
  auto flush = [&](int64_t kb) -> int {
    if constexpr (sizeof(T) == sizeof(float)) {
      if (r.M64) {
        HIP_TRY(launch_flush_vf(r.p, r.V, r.M64, r.slot, r.X64, r.n, kb, r.st, r.s));
        return 0;
      }
    }
    HIP_TRY(launch_flush<T>(r.p, r.V, r.M, r.slot, X, r.n, kb, r.st, r.s));
    return 0;
  };
  auto enq = [&](int slot) -> int {
    for (int q = 0; q < batch; ++q, ++kq) {
      if (prof) HIP_TRY(hipEventRecord(pev[slot][0], r.s));
      if constexpr (sizeof(T) == sizeof(double)) {
        if (r.pc) {  // W = C^{-1} A C^{-T} V_k, then pass 1 on the formed product
          const double* Vk = (const double*)r.Vslot(kq);
          HIP_TRY(launch_ic0_solve(*r.pc, p, true, Vk, r.Y, r.st, r.s));
          HIP_TRY(launch_spmm<double>(p, *r.A, r.A->val, r.Y, r.Z, r.s, r.st));
          if (r.pc->n_levels == 2) {  // the forward solve inside pass 1
            HIP_TRY(launch_pass1_tri(p, r.pc->lrp, r.pc->lci, r.pc->lval_s, r.pc->diag, r.Z, (double*)r.V,
                                     r.slot, (const double*)r.bench, r.part, r.n_wg, n, r.st, r.s));
          } else {  // level by level in place, then pass 1 on the formed product
            HIP_TRY(launch_ic0_solve(*r.pc, p, false, r.Z, r.Z, r.st, r.s));
            HIP_TRY(launch_pass1_ident(p, r.Z, (double*)r.V, r.slot, (const double*)r.bench, r.part, r.n_wg, n,
                                       r.st, r.s));
          }
        } else {
          HIP_TRY(launch_pass1<T>(r.p, *r.A, r.val, r.V, r.slot, r.bench, r.part, r.n_wg, r.st, r.s));
        }
      } else {
        HIP_TRY(launch_pass1<T>(r.p, *r.A, r.val, r.V, r.slot, r.bench, r.part, r.n_wg, r.st, r.s));
      }
      if (prof) HIP_TRY(hipEventRecord(pev[slot][1], r.s));
      HIP_TRY(launch_reduce(r.part, r.n_wg, n_entries(r.p, r.nb), r.red, r.st, 1, r.s));
      if (prof) HIP_TRY(hipEventRecord(pev[slot][2], r.s));
      HIP_TRY(launch_band(r.p, 0, r.nb, r.red, r.hist, r.st, r.s));
      if (prof) HIP_TRY(hipEventRecord(pev[slot][3], r.s));
      HIP_TRY(launch_pass2<T>(r.p, r.V, r.slot, r.bench, r.n, r.st, r.s));
      if (kq % grp == 0) TRY(flush(kq));
      if (prof) HIP_TRY(hipEventRecord(pev[slot][4], r.s));
    }
    HIP_TRY(hipMemcpyAsync(&pin[slot].ctl, r.st, sizeof(Ctl), hipMemcpyDeviceToHost, r.s));
    if (o.switch_theta > 0)
      HIP_TRY(hipMemcpyAsync(pin[slot].rho, (const char*)r.st + offsetof(DevState, rho), sizeof(double) * MAXP,
                             hipMemcpyDeviceToHost, r.s));
    HIP_TRY(hipEventRecord(ev[slot], r.s));
    return 0;
  };
  int64_t last_explicit = 0;  // block of the last column-wise QR (its flush is enqueued with it)
  for (;;) {
    TRY(enq(0));
    int cur = 0;
    Ctl ctl{};
    bool drain = false;
    for (;;) {
      if (!prof) TRY(enq(cur ^ 1));
      HIP_TRY(hipEventSynchronize(ev[cur]));
      ctl = pin[cur].ctl;
      // a halted iteration's kernels returned at once: time only live ones
      if (prof && (!ctl.halt || ctl.reason == REASON_FINISHED)) TRY(collect(cur));
      if (ctl.halt) break;
      if (o.switch_theta > 0) {
        double w = 0.0;
        for (int i = 0; i < p; ++i) w = std::max(w, pin[cur].rho[i]);
        if (w < o.switch_theta) {
          drain = true;
          break;
        }
      }
      if (prof) TRY(enq(cur ^ 1));
      cur ^= 1;
    }
    if (drain) {
      // enqueue up to the end of the group the last enqueued block is in,
      // let the device finish, and hand over unless it halted meanwhile
      const int64_t target = (kq - 1 + grp - 1) / grp * grp;
      if (kq <= target) {
        const int keep = batch;
        batch = (int)(target - kq + 1);
        TRY(enq(cur));  // slot cur: its record has been read
        batch = keep;
      }
      HIP_TRY(hipStreamSynchronize(r.s));
      HIP_TRY(hipMemcpy(hs, r.st, sizeof(DevState), hipMemcpyDeviceToHost));
      if (!hs->halt) {
        finish(hs->j, hs->k, hs->rho);
        return SWITCHED;
      }
      memcpy(&ctl, hs, sizeof(Ctl));
    }
    if (ctl.reason != REASON_EXPLICIT_QR) {
      HIP_TRY(hipStreamSynchronize(r.s));
      break;
    }
    // ---- column-wise QR of block k (near-dependent candidates) ----------
    // Enqueued behind the iterations still in flight, which return at once
    // while the loop is halted; the QR's last kernel resumes the loop, and
    // the band kernel (told that B_k and V_{k+1} are done), pass 2 and the
    // group's flush complete block k.  Nothing here waits for the device.
    const int64_t k = ctl.k;
    TRY(r.colqr(QR_LOOP, r.Vslot(k + 1), r.Vslot(k)));
    HIP_TRY(launch_band(r.p, 1, r.nb, r.red, r.hist, r.st, r.s));
    HIP_TRY(launch_pass2<T>(r.p, r.V, r.slot, r.bench, r.n, r.st, r.s));
    TRY(flush(k));
    last_explicit = k;
    kq = k + 1;
  }
  HIP_TRY(hipMemcpyAsync(hs, r.st, sizeof(DevState), hipMemcpyDeviceToHost, r.s));
  HIP_TRY(hipStreamSynchronize(r.s));
  // a stop inside a group: its search directions still go into X
  if (hs->reason == REASON_FINISHED && hs->flush_len > 0 && hs->flush_block % grp != 0 &&
      hs->flush_block != last_explicit) {
    TRY(flush(hs->flush_block));
    HIP_TRY(hipStreamSynchronize(r.s));
  }
  if (res_hist && o.hist_cap > 0) {
    const int64_t rows = std::min<int64_t>(hs->j, o.hist_cap);
    if (rows > 0)
      HIP_TRY(hipMemcpy(res_hist, r.hist, sizeof(double) * (size_t)rows * p, hipMemcpyDeviceToHost));
  }
  const int status = hs->status == STATUS_RUNNING ? BMR_HIP_ERROR : hs->status;
  finish(hs->j, hs->k, hs->rho);
  return status;
}

// Point the run's fields into the workspace.
template <typename T>
void bind(Run<T>& r, const bmr_csr_t* A, const T* val, int p, int nb, hipStream_t s, char* ws, const Layout& L) {
  r.A = A;
  r.val = val;
  r.p = p;
  r.nb = nb;
  r.n = A->n;
  r.s = s;
  r.n_wg = pass1_resident_grid<T>(A->n, p);  // <= L.n_wg, which sizes the partial sums
  r.st = (DevState*)(ws + L.off_state);
  r.red = (double*)(ws + L.off_red);
  r.part = (double*)(ws + L.off_part);
  r.hist = (double*)(ws + L.off_hist);
  r.V = (T*)(ws + L.off_V);
  r.M = (T*)(ws + L.off_M);
  r.bench = (T*)(ws + L.off_bench);
  r.slot = slot_elems(A->n, p);
  r.ret = L.off_ret ? (T*)(ws + L.off_ret) : nullptr;
}

void fill_stats(bmr_stats_t* stats, int status, int p, const CoreOut& o) {
  if (!stats) return;
  memset(stats, 0, sizeof(*stats));
  stats->status = status;
  stats->n_replaced = o.n_replaced;
  stats->band_iters = o.j;
  stats->block_iters = o.k;
  stats->n_explicit_qr = o.n_explicit;
  stats->n_retained = o.n_kept;
  stats->p = p;
  for (int i = 0; i < BMR_MAX_P; ++i) stats->res_rec[i] = i < p ? o.rho[i] : 0.0;
  for (int q = 0; q < 4; ++q) stats->t_kernel_ms[q] = o.n_prof ? o.tk[q] / o.n_prof : 0.0;
  stats->n_profiled = o.n_prof;
}

// pc: with an IC(0) factor C, block MINRES runs on C^{-1} A C^{-T} with
// right-hand sides C^{-1} B (formed in Y before the iteration takes Y over),
// and X = C^{-T} X-hat at the end; the stopping test and res_rec refer to
// the preconditioned residual, res_explicit to B - A X.
int solve_fp64(const bmr_csr_t* A, const double* B, double* X, int p, const bmr_opts_t& o, char* ws,
               const Layout& L, hipStream_t s, bmr_stats_t* stats, double* res_hist, const Ic0View* pc = nullptr) {
  Run<double> r{};
  bind(r, A, A->val, p, o.n_bench, s, ws, L);
  const double* rhs = B;
  if (pc) {
    r.pc = pc;
    r.Y = (double*)(ws + L.off_Y);
    r.Z = (double*)(ws + L.off_Z);
    HIP_TRY(launch_ic0_solve(*pc, p, false, B, r.Y, nullptr, s));
    rhs = r.Y;
  }
  CoreParams cp{o.tol, o.gamma, TAU_FB, o.max_iter, o.hist_cap, o.seed, o.poll_every,
                (o.flags & BMR_FLAG_PROFILE) != 0, nullptr, (o.flags & BMR_FLAG_ACCUMULATE) != 0};
  CoreOut out;
  const int status = solve_core<double>(r, rhs, X, cp, out, res_hist);
  if (status < 0) return status;
  double bnorm[MAXP];
  for (int i = 0; i < p; ++i) bnorm[i] = out.bnorm[i];
  if (pc) {  // X = C^{-T} X-hat in place; the explicit residual is relative to ||b_i||
    HIP_TRY(launch_ic0_solve(*pc, p, true, X, X, nullptr, s));
    double c[MAXP + 1];
    for (int i = 0; i < p; ++i) {
      TRY(r.coldots(B, p, i, (const double*)nullptr, 0, 0, c));
      bnorm[i] = sqrt(c[0]);
    }
  }
  // the explicit residual of the result, reported beside the recurrence
  // values (Algorithm 7.1's output)
  double rn[MAXP];
  TRY(residual_norms(A, B, X, p, nullptr, r.part, L.n_wg, r.red, s, rn));
  fill_stats(stats, status, p, out);
  if (stats)
    for (int i = 0; i < p; ++i) stats->res_explicit[i] = bnorm[i] > 0 ? rn[i] / bnorm[i] : 0.0;
  return status;
}

// FP64 iterative refinement around the FP32 driver:
//   R = B - A X (FP64); stop when every ||r_i|| / ||b_i|| < tol;
//   solve A D = R in FP32 until each column's recurrence residual is below
//   max(inner_tol * ||r_i||, tol * ||b_i|| / 2);  X += D (FP64).
int solve_mixed(const bmr_csr_t* A, const double* B, double* X, int p, const bmr_opts_t& o, char* ws,
                const Layout& L, hipStream_t s, bmr_stats_t* stats, double* res_hist) {
  const int64_t n = A->n;
  float* val32 = (float*)(ws + L.off_val32);
  float* D = (float*)(ws + L.off_D);
  double* R = (double*)(ws + L.off_R);
  double* part = (double*)(ws + L.off_part);
  double* red = (double*)(ws + L.off_red);
  Run<float> r{};
  bind(r, A, (const float*)val32, p, o.n_bench, s, ws, L);
  HIP_TRY(launch_to_f32(A->val, val32, (size_t)A->nnz, s));
  HIP_TRY(launch_fill<double>(X, (size_t)n * p, 0.0, s));

  double beta[MAXP], rn[MAXP], stop[MAXP], rel[MAXP];
  TRY(residual_norms(A, B, X, p, R, part, L.n_wg, red, s, beta));  // X = 0: R = B
  for (int i = 0; i < p; ++i) {
    if (!isfinite(beta[i])) return BMR_NONFINITE;
    rn[i] = beta[i];
  }
  CoreOut tot;
  int status = BMR_MAX_ITER, cycles = 0;
  double prev_worst = HUGE_VAL;
  for (;;) {
    double worst = 0.0;
    for (int i = 0; i < p; ++i) {
      rel[i] = beta[i] > 0 ? rn[i] / beta[i] : 0.0;
      if (!isfinite(rel[i])) return BMR_NONFINITE;
      worst = std::max(worst, rel[i]);
    }
    if (cycles > 0 && res_hist && cycles <= o.hist_cap)
      for (int i = 0; i < p; ++i) res_hist[(size_t)(cycles - 1) * p + i] = rel[i];
    if (worst < o.tol) {
      status = BMR_CONVERGED;
      break;
    }
    if (cycles > 0 && worst > 0.5 * prev_worst) {
      status = BMR_STAGNATED;
      break;
    }
    if (cycles >= o.max_refine || tot.j >= o.max_iter) {
      status = BMR_MAX_ITER;
      break;
    }
    if (status == BMR_BENCH_EXHAUSTED) break;
    prev_worst = worst;
    for (int i = 0; i < p; ++i) stop[i] = std::max(rn[i], 0.5 * o.tol * beta[i] / o.inner_tol);
    CoreParams cp{o.inner_tol, std::max(o.gamma, GAMMA_F32), TAU_FB_F32, o.max_iter - tot.j, 0, o.seed,
                  o.poll_every, (o.flags & BMR_FLAG_PROFILE) != 0, stop, (o.flags & BMR_FLAG_ACCUMULATE) != 0};
    CoreOut out;
    const int st = solve_core<float>(r, R, D, cp, out, nullptr);
    if (st < 0) return st;
    ++cycles;
    tot.j += out.j;
    tot.k += out.k;
    tot.n_replaced += out.n_replaced;
    tot.n_explicit += out.n_explicit;
    for (int q = 0; q < 4; ++q) tot.tk[q] += out.tk[q];
    tot.n_prof += out.n_prof;
    HIP_TRY(launch_add_f32(X, D, (size_t)n * p, s));
    TRY(residual_norms(A, B, X, p, R, part, L.n_wg, red, s, rn));
    status = st == BMR_BENCH_EXHAUSTED ? BMR_BENCH_EXHAUSTED : BMR_MAX_ITER;
  }
  for (int i = 0; i < p; ++i) tot.rho[i] = rel[i];
  fill_stats(stats, status, p, tot);
  if (stats) {
    stats->precision = BMR_PREC_MIXED;
    stats->n_refine = cycles;
    for (int i = 0; i < p; ++i) stats->res_true[i] = stats->res_explicit[i] = rel[i];
  }
  return status;
}

// BMR_PREC_RELAXED: the FP64 driver until every column's recurrence
// residual is below relax_tol and the current group of blocks has ended,
// then the FP32 driver on the same device state: V_k and V_{k-1} of the next
// block and the bench are rounded to FP32, tau_fb and gamma take the FP32
// values, and the flush reads the FP32 ring into the FP64 search directions
// and X.  Keeping those two FP64 matters: the search directions follow a
// three-term recurrence, M_k = (V_k - M_{k-1} D_k - M_{k-2} E_k) C_k, whose
// rounding errors MINRES's residual gap grows with, and they are of the size
// of the whole solution, not of the error left at the switch.
int solve_relaxed(const bmr_csr_t* A, const double* B, double* X, int p, const bmr_opts_t& o, char* ws,
                  const Layout& L, hipStream_t s, bmr_stats_t* stats, double* res_hist) {
  const int64_t n = A->n;
  Run<double> r{};
  bind(r, A, A->val, p, o.n_bench, s, ws, L);
  const bool prof = (o.flags & BMR_FLAG_PROFILE) != 0, acc = (o.flags & BMR_FLAG_ACCUMULATE) != 0;
  CoreParams cp{o.tol, o.gamma, TAU_FB, o.max_iter, o.hist_cap, o.seed, o.poll_every, prof, nullptr, acc};
  cp.switch_theta = o.relax_tol > 0 ? o.relax_tol : std::min(1e-2, 1e3 * o.tol);
  CoreOut out;
  int status = solve_core<double>(r, B, X, cp, out, res_hist);
  if (status < 0) return status;
  int64_t switch_j = 0;
  CoreOut tot = out;
  if (status == SWITCHED) {
    switch_j = out.j;
    const int64_t k = out.k;  // the next block; blocks up to k - 1 are flushed into X
    float* val32 = (float*)(ws + L.off_val32);
    Run<float> q{};
    q.A = A;
    q.val = val32;
    q.p = p;
    q.nb = o.n_bench;
    q.n = n;
    q.s = s;
    q.n_wg = pass1_resident_grid<float>(n, p);  // <= L.n_wg, which sizes the partial sums
    q.st = r.st;
    q.red = r.red;
    q.part = r.part;
    q.hist = r.hist;
    q.V = (float*)(ws + L.off_V32);
    q.M = nullptr;
    q.M64 = r.M;
    q.X64 = X;
    q.bench = (float*)(ws + L.off_bench32);
    q.slot = r.slot;
    HIP_TRY(launch_to_f32(A->val, val32, (size_t)A->nnz, s));
    HIP_TRY(launch_to_f32(r.Vslot(k), q.Vslot(k), (size_t)n * p, s));
    HIP_TRY(launch_to_f32(r.Vslot(k - 1), q.Vslot(k - 1), (size_t)n * p, s));
    if (o.n_bench > 0) HIP_TRY(launch_to_f32(r.bench, q.bench, (size_t)n * o.n_bench, s));
    const double gt[2] = {std::max(o.gamma, GAMMA_F32), TAU_FB_F32};  // DevState: gamma, tau_fb
    static_assert(offsetof(DevState, tau_fb) == offsetof(DevState, gamma) + sizeof(double), "gamma, tau_fb");
    HIP_TRY(hipMemcpyAsync((char*)r.st + offsetof(DevState, gamma), gt, sizeof(gt), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    CoreParams cq{o.tol, gt[0], TAU_FB_F32, o.max_iter, o.hist_cap, o.seed, o.poll_every, prof, nullptr, acc};
    cq.resume_k = k;
    CoreOut o32;
    status = solve_core<float>(q, nullptr, nullptr, cq, o32, res_hist);
    if (status < 0) return status;
    tot.j = o32.j;  // the device counters run on across the switch
    tot.k = o32.k;
    tot.n_replaced = o32.n_replaced;
    tot.n_explicit = o32.n_explicit;
    tot.n_kept = o32.n_kept;
    for (int i = 0; i < MAXP; ++i) tot.rho[i] = o32.rho[i];
    for (int c = 0; c < 4; ++c) tot.tk[c] += o32.tk[c];
    tot.n_prof += o32.n_prof;
  }
  double rn[MAXP];
  TRY(residual_norms(A, B, X, p, nullptr, r.part, L.n_wg, r.red, s, rn));
  fill_stats(stats, status, p, tot);
  if (stats) {
    for (int i = 0; i < p; ++i) stats->res_explicit[i] = out.bnorm[i] > 0 ? rn[i] / out.bnorm[i] : 0.0;
    stats->switch_iter = switch_j;
  }
  return status;
}

}  // namespace

extern "C" {

int bmr_version(void) { return BMR_VERSION; }

const char* bmr_status_string(int status) {
  switch (status) {
    case BMR_CONVERGED: return "converged";
    case BMR_MAX_ITER: return "maximum iterations reached";
    case BMR_BENCH_EXHAUSTED: return "substitute bench exhausted";
    case BMR_STAGNATED: return "refinement stagnated";
    case BMR_INVALID_ARG: return "invalid argument";
    case BMR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case BMR_HIP_ERROR: return "HIP runtime error";
    case BMR_NONFINITE: return "non-finite value";
    case BMR_SINGULAR_R: return "singular band QR factor";
    case BMR_IC0_BREAKDOWN: return "incomplete Cholesky factorisation broke down";
    default: return "unknown status";
  }
}

void bmr_default_opts(bmr_opts_t* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->max_iter = 10000;
  o->gamma = 1e-10;
  o->n_bench = 2;
  o->poll_every = 0;
  o->seed = 0;
  o->hist_cap = 0;
  o->flags = 0;
  o->precision = BMR_PREC_FP64;
  o->inner_tol = 1e-6;
  o->max_refine = 30;
  o->relax_tol = 0.0;
}

int bmr_workspace_bytes(int64_t n, int64_t nnz, int p, const bmr_opts_t* opts, size_t* bytes) {
  bmr_opts_t o;
  bmr_default_opts(&o);
  if (opts) o = *opts;
  if (!bytes || n < 1 || nnz < 0 || p < 1 || p > BMR_MAX_P || !opts_valid(o)) return BMR_INVALID_ARG;
  *bytes = layout_for(n, nnz, p, o.n_bench, o.hist_cap, o.precision, o.precond, (o.flags & BMR_FLAG_RETAIN) != 0)
               .total;
  return BMR_CONVERGED;
}

int bmr_solve(const bmr_csr_t* A, const double* B, double* X, int p, const bmr_opts_t* opts, void* workspace,
              size_t workspace_bytes, hipStream_t stream, bmr_stats_t* stats, double* res_hist) {
  bmr_opts_t o;
  bmr_default_opts(&o);
  if (opts) o = *opts;
  if (!csr_valid(A) || !B || !X || !workspace || p < 1 || p > BMR_MAX_P || !opts_valid(o)) return BMR_INVALID_ARG;
  if (o.precond != BMR_PRECOND_NONE) return BMR_INVALID_ARG;  // the factor comes with bmr_solve_ic0
  if (((uintptr_t)workspace) % 256 != 0 || !aligned16(B) || !aligned16(X)) return BMR_INVALID_ARG;
  const Layout L = layout_for(A->n, A->nnz, p, o.n_bench, o.hist_cap, o.precision, BMR_PRECOND_NONE,
                              (o.flags & BMR_FLAG_RETAIN) != 0);
  if (workspace_bytes < L.total) return BMR_WORKSPACE_TOO_SMALL;
  hipEvent_t t0, t1;
  if (hipEventCreate(&t0) != hipSuccess) return BMR_HIP_ERROR;
  if (hipEventCreate(&t1) != hipSuccess) return BMR_HIP_ERROR;
  (void)hipEventRecord(t0, stream);
  const int status = o.precision == BMR_PREC_MIXED
                         ? solve_mixed(A, B, X, p, o, (char*)workspace, L, stream, stats, res_hist)
                     : o.precision == BMR_PREC_RELAXED
                         ? solve_relaxed(A, B, X, p, o, (char*)workspace, L, stream, stats, res_hist)
                         : solve_fp64(A, B, X, p, o, (char*)workspace, L, stream, stats, res_hist);
  (void)hipEventRecord(t1, stream);
  (void)hipEventSynchronize(t1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, t0, t1);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (stats) {
    if (status < 0) {
      memset(stats, 0, sizeof(*stats));
      stats->status = status;
      stats->p = p;
    }
    stats->precision = o.precision;
    stats->time_ms = ms;
  }
  return status;
}

int bmr_solve_ic0(const bmr_csr_t* A, const void* ic0, const double* B, double* X, int p, const bmr_opts_t* opts,
                  void* workspace, size_t workspace_bytes, hipStream_t stream, bmr_stats_t* stats,
                  double* res_hist) {
  bmr_opts_t o;
  bmr_default_opts(&o);
  if (opts) o = *opts;
  o.precond = BMR_PRECOND_IC0;
  if (!csr_valid(A) || !ic0 || !B || !X || !workspace || p < 1 || p > BMR_MAX_P || !opts_valid(o))
    return BMR_INVALID_ARG;
  if (((uintptr_t)workspace) % 256 != 0 || !aligned16(B) || !aligned16(X) || B == X) return BMR_INVALID_ARG;
  const Layout L = layout_for(A->n, A->nnz, p, o.n_bench, o.hist_cap, o.precision, o.precond,
                              (o.flags & BMR_FLAG_RETAIN) != 0);
  if (workspace_bytes < L.total) return BMR_WORKSPACE_TOO_SMALL;
  Ic0View v;
  const int e = ic0_view(ic0, &v);
  if (e) return e;
  if (v.n != A->n) return BMR_INVALID_ARG;
  hipEvent_t t0, t1;
  if (hipEventCreate(&t0) != hipSuccess) return BMR_HIP_ERROR;
  if (hipEventCreate(&t1) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return BMR_HIP_ERROR;
  }
  (void)hipEventRecord(t0, stream);
  const int status = solve_fp64(A, B, X, p, o, (char*)workspace, L, stream, stats, res_hist, &v);
  (void)hipEventRecord(t1, stream);
  (void)hipEventSynchronize(t1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, t0, t1);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (stats) {
    if (status < 0) {
      memset(stats, 0, sizeof(*stats));
      stats->status = status;
      stats->p = p;
    }
    stats->precision = BMR_PREC_FP64;
    stats->time_ms = ms;
  }
  return status;
}

int bmr_spmm(const bmr_csr_t* A, const double* V, double* W, int p, hipStream_t stream) {
  if (!csr_valid(A) || !V || !W || V == W || p < 1 || p > BMR_MAX_P || !aligned16(V) || !aligned16(W))
    return BMR_INVALID_ARG;
  return launch_spmm<double>(p, *A, A->val, V, W, stream) == hipSuccess ? BMR_CONVERGED : BMR_HIP_ERROR;
}

int bmr_spmm_f32(const bmr_csr_t* A, const float* val32, const float* V, float* W, int p, hipStream_t stream) {
  if (!csr_valid(A) || (A->nnz > 0 && !val32) || !V || !W || V == W || p < 1 || p > BMR_MAX_P || !aligned16(V) ||
      !aligned16(W))
    return BMR_INVALID_ARG;
  return launch_spmm<float>(p, *A, val32, V, W, stream) == hipSuccess ? BMR_CONVERGED : BMR_HIP_ERROR;
}

int bmr_pattern_grad(const bmr_csr_t* A, const double* Lam, const double* X, int p, double* grad,
                     hipStream_t stream) {
  if (!csr_valid(A) || !Lam || !X || !grad || p < 1 || p > BMR_MAX_P) return BMR_INVALID_ARG;
  if (A->nnz == 0) return BMR_CONVERGED;
  return launch_pattern_grad(p, *A, Lam, X, grad, stream) == hipSuccess ? BMR_CONVERGED : BMR_HIP_ERROR;
}

int bmr_residual(const bmr_csr_t* A, const double* B, const double* X, int p, double* R, double* norms,
                 void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!csr_valid(A) || !B || !X || !norms || !workspace || p < 1 || p > BMR_MAX_P) return BMR_INVALID_ARG;
  if (!aligned16(X)) return BMR_INVALID_ARG;
  bmr_opts_t o;
  bmr_default_opts(&o);
  const Layout L = layout_for(A->n, 0, p, o.n_bench, 0, BMR_PREC_FP64);
  const size_t need = L.off_part + sizeof(double) * (size_t)p * L.n_wg;
  if (workspace_bytes < need) return BMR_WORKSPACE_TOO_SMALL;
  double* part = (double*)((char*)workspace + L.off_part);
  double* red = (double*)((char*)workspace + L.off_red);
  return residual_norms(A, B, X, p, R, part, L.n_wg, red, stream, norms) == 0 ? BMR_CONVERGED : BMR_HIP_ERROR;
}

}  // extern "C"
