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
// halts and the host runs that block's QR column by column (with the
// dependence test and bench substitution of Section 5.1), then resumes.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "bmr_internal.hpp"

namespace bmr {
namespace {

constexpr double TAU_FB = 1e-2;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
size_t slot_elems(int64_t n, int p) { return ((size_t)n * p + 31) / 32 * 32; }

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

// Host side of a solve: workspace pointers, stream, scratch for column sums.
struct Run {
  const bmr_csr_t* A;
  int p, nb;
  int64_t n;
  hipStream_t s;
  Layout L;
  char* ws;
  DevState* st;
  double *red, *part, *hist, *V, *M, *bench;
  size_t slot;
  std::vector<double> hpart;

  double* Vslot(int64_t k) { return V + (size_t)(k % 3) * slot; }

  // Column sums of k_coldots, summed on the host in workgroup order.
  int coldots(const double* Y, int ldy, int yc, const double* X, int ldx, int m, double* out) {
    const int g = coldots_grid(n);
    HIP_TRY(launch_coldots(Y, ldy, yc, X, ldx, m, n, part, g, s));
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
  int colop(double* D, int ldd, int dc, const double* S, int lds, int sc, const double* X, int ldx, int m,
            const double* coef, double div) {
    ColCoef cc;
    for (int r = 0; r < MAXP; ++r) cc.c[r] = (r < m) ? coef[r] : 0.0;
    HIP_TRY(launch_colop(D, ldd, dc, S, lds, sc, X, ldx, m, cc, div, n, s));
    return 0;
  }
};

// Column-wise QR of the p columns of D (in place, row-interleaved, stride p):
// classical Gram-Schmidt applied twice against the columns already done,
// dependence when the remainder norm is <= gamma * ref[l], substitution by
// the next bench vector, and one Gram-Schmidt step of the unused bench
// vectors against every new column.  Coefficients go to R (stride MAXP).
// Returns 0, or BMR_BENCH_EXHAUSTED with *lcap = the dependent column, or an
// error.
int column_qr(Run& r, double* D, const double* ref, double gamma, const double* bench_norm0, int* taken,
              int* n_replaced, double* R, int* lcap) {
  const int p = r.p, nb = r.nb;
  double c[MAXP + 1];
  *lcap = p;
  for (int l = 0; l < p; ++l) {
    for (int q = 0; q < MAXP; ++q) R[q * MAXP + l] = 0.0;
    if (l > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        int e = r.coldots(D, p, l, D, p, l, c);
        if (e) return e;
        for (int q = 0; q < l; ++q) R[q * MAXP + l] += c[q];
        e = r.colop(D, p, l, D, p, l, D, p, l, c, 1.0);
        if (e) return e;
      }
    }
    int e = r.coldots(D, p, l, nullptr, 0, 0, c);
    if (e) return e;
    const double eta = sqrt(c[0]);
    if (!isfinite(eta)) return BMR_NONFINITE;
    if (eta <= gamma * ref[l]) {
      R[l * MAXP + l] = 0.0;
      bool ok = *taken < nb;
      double gn = 0.0;
      if (ok) {
        e = r.coldots(r.bench, nb, *taken, nullptr, 0, 0, c);
        if (e) return e;
        gn = sqrt(c[0]);
        ok = gn > gamma * bench_norm0[*taken];
      }
      if (!ok) {
        *lcap = l;
        return BMR_BENCH_EXHAUSTED;
      }
      e = r.colop(D, p, l, r.bench, nb, *taken, nullptr, 0, 0, nullptr, gn);
      if (e) return e;
      ++*taken;
      ++*n_replaced;
    } else {
      R[l * MAXP + l] = eta;
      e = r.colop(D, p, l, D, p, l, nullptr, 0, 0, nullptr, eta);
      if (e) return e;
    }
    for (int b = *taken; b < nb; ++b) {
      e = r.coldots(r.bench, nb, b, D + l, p, 1, c);
      if (e) return e;
      e = r.colop(r.bench, nb, b, r.bench, nb, b, D + l, p, 1, c, 1.0);
      if (e) return e;
    }
  }
  return 0;
}

#define TRY(expr)              \
  do {                         \
    int e_ = (expr);           \
    if (e_ != 0) return e_;    \
  } while (0)

}  // namespace

Layout layout_for(int64_t n, int p, int nb, int64_t hist_cap) {
  Layout L{};
  L.n_wg = pass1_grid(n, p);
  size_t off = 0;
  L.off_state = off;
  off = align256(off + sizeof(DevState));
  L.off_red = off;
  off = align256(off + sizeof(double) * n_entries(MAXP, MAXB));
  size_t part = std::max<size_t>((size_t)n_entries(p, nb) * L.n_wg, (size_t)coldots_grid(n) * (MAXP + 1));
  part = std::max<size_t>(part, (size_t)p * L.n_wg);
  L.off_part = off;
  off = align256(off + sizeof(double) * part);
  L.off_hist = off;
  off = align256(off + sizeof(double) * (size_t)hist_cap * p);
  const size_t se = slot_elems(n, p);
  L.off_V = off;
  off = align256(off + sizeof(double) * 3 * se);
  L.off_M = off;
  off = align256(off + sizeof(double) * 3 * se);
  L.off_bench = off;
  off = align256(off + sizeof(double) * (size_t)n * nb);
  L.total = off;
  return L;
}

}  // namespace bmr

using namespace bmr;

namespace {

bool opts_valid(const bmr_opts_t& o) {
  return o.tol > 0.0 && isfinite(o.tol) && o.max_iter >= 1 && o.gamma >= 0.0 && isfinite(o.gamma) &&
         o.n_bench >= 0 && o.n_bench <= BMR_MAX_BENCH && o.hist_cap >= 0 && o.poll_every >= 0;
}

bool csr_valid(const bmr_csr_t* A) {
  return A && A->n >= 1 && A->n < (int64_t(1) << 31) && A->nnz >= 0 && A->nnz < (int64_t(1) << 31) &&
         A->row_ptr && (A->nnz == 0 || (A->col_idx && A->val));
}

// Two pinned status records per host thread, reused by every solve of that
// thread (allocated once, never freed).
Ctl* pinned_ctl() {
  static thread_local Ctl* buf = nullptr;
  if (!buf) {
    void* p = nullptr;
    if (hipHostMalloc(&p, 2 * sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return nullptr;
    buf = (Ctl*)p;
  }
  return buf;
}

int solve_impl(Run& r, const double* B, double* X, const bmr_opts_t& o, bmr_stats_t* stats, double* res_hist) {
  const int p = r.p, nb = r.nb;
  const int64_t n = r.n;
  // ---- set-up -------------------------------------------------------------
  HIP_TRY(launch_fill(r.V, 3 * r.slot, 0.0, r.s));
  HIP_TRY(launch_fill(r.M, 3 * r.slot, 0.0, r.s));
  HIP_TRY(launch_fill(X, (size_t)n * p, 0.0, r.s));
  HIP_TRY(launch_bench_init(r.bench, n, nb, o.seed, r.s));

  DevState* hs = new DevState();
  struct Guard {
    DevState* p;
    ~Guard() { delete p; }
  } guard{hs};
  memset(hs, 0, sizeof(DevState));
  hs->status = STATUS_RUNNING;
  hs->p = p;
  hs->nb = nb;
  hs->n = n;
  hs->max_iter = o.max_iter;
  hs->hist_cap = o.hist_cap;
  hs->tol = o.tol;
  hs->gamma = o.gamma;
  hs->tau_fb = TAU_FB;
  hs->lcap = p;
  hs->k = 1;

  double c[MAXP + 1];
  for (int i = 0; i < p; ++i) {
    TRY(r.coldots(B, p, i, nullptr, 0, 0, c));
    hs->beta[i] = sqrt(c[0]);
    if (!isfinite(hs->beta[i])) return BMR_NONFINITE;
  }
  for (int b = 0; b < nb; ++b) {
    TRY(r.coldots(r.bench, nb, b, nullptr, 0, 0, c));
    hs->bench_norm0[b] = sqrt(c[0]);
  }
  // initial QR of F_0 = B into V_1 (slot 1): copy, then column-wise CGS2
  double* V1 = r.Vslot(1);
  for (int i = 0; i < p; ++i) TRY(r.colop(V1, p, i, B, p, i, nullptr, 0, 0, nullptr, 1.0));
  double S[MAXP * MAXP];
  int lcap = p;
  int qr = column_qr(r, V1, hs->beta, o.gamma, hs->bench_norm0, &hs->taken, &hs->n_replaced, S, &lcap);
  auto finish_stats = [&](int status, int64_t j, int64_t kblocks, const double* rho) {
    if (stats) {
      stats->status = status;
      stats->n_replaced = hs->n_replaced;
      stats->band_iters = j;
      stats->block_iters = kblocks;
      stats->n_explicit_qr = hs->n_explicit;
      stats->p = p;
      for (int i = 0; i < BMR_MAX_P; ++i) stats->res_rec[i] = (i < p && rho) ? rho[i] : 0.0;
    }
  };
  if (qr == BMR_BENCH_EXHAUSTED) {
    double one[MAXP];
    for (int i = 0; i < p; ++i) one[i] = hs->beta[i] > 0 ? 1.0 : 0.0;
    finish_stats(BMR_BENCH_EXHAUSTED, 0, 0, one);
    return BMR_BENCH_EXHAUSTED;
  }
  if (qr) return qr;
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
    finish_stats(BMR_CONVERGED, 0, 0, hs->rho);
    return BMR_CONVERGED;
  }
  HIP_TRY(hipMemcpyAsync(r.st, hs, sizeof(DevState), hipMemcpyHostToDevice, r.s));

  // ---- block iterations -------------------------------------------------
  Ctl* pin = pinned_ctl();
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
  if (batch <= 0) batch = ((double)n * p < 2e6) ? 32 : 8;
  const bool prof = (o.flags & BMR_FLAG_PROFILE) != 0;
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
  double tk[4] = {0, 0, 0, 0};
  int64_t nprof = 0;
  auto collect = [&](int slot) -> int {  // add the timings of the iteration in `slot`
    if (!prof) return 0;
    for (int q = 0; q < 4; ++q) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, pev[slot][q], pev[slot][q + 1]));
      tk[q] += ms;
    }
    ++nprof;
    return 0;
  };

  // enqueue `batch` block iterations, then a copy of the status record
  auto enq = [&](int slot) -> int {
    for (int q = 0; q < batch; ++q) {
      if (prof) HIP_TRY(hipEventRecord(pev[slot][0], r.s));
      HIP_TRY(launch_pass1(r.p, *r.A, r.V, r.slot, r.bench, r.part, r.L.n_wg, r.st, r.s));
      if (prof) HIP_TRY(hipEventRecord(pev[slot][1], r.s));
      HIP_TRY(launch_reduce(r.part, r.L.n_wg, n_entries(r.p, r.nb), r.red, r.st, 1, r.s));
      if (prof) HIP_TRY(hipEventRecord(pev[slot][2], r.s));
      HIP_TRY(launch_band(r.p, 0, r.red, r.hist, r.st, r.s));
      if (prof) HIP_TRY(hipEventRecord(pev[slot][3], r.s));
      HIP_TRY(launch_pass2(r.p, r.V, r.M, r.slot, X, r.bench, r.n, r.st, r.s));
      if (prof) HIP_TRY(hipEventRecord(pev[slot][4], r.s));
    }
    HIP_TRY(hipMemcpyAsync(&pin[slot], r.st, sizeof(Ctl), hipMemcpyDeviceToHost, r.s));
    HIP_TRY(hipEventRecord(ev[slot], r.s));
    return 0;
  };
  for (;;) {
    TRY(enq(0));
    int cur = 0;
    Ctl ctl{};
    for (;;) {
      if (!prof) TRY(enq(cur ^ 1));
      HIP_TRY(hipEventSynchronize(ev[cur]));
      ctl = pin[cur];
      // a halted iteration's kernels returned at once: time only live ones
      if (prof && (!ctl.halt || ctl.reason == REASON_FINISHED)) TRY(collect(cur));
      if (ctl.halt) break;
      if (prof) TRY(enq(cur ^ 1));
      cur ^= 1;
    }
    HIP_TRY(hipStreamSynchronize(r.s));
    if (ctl.reason != REASON_EXPLICIT_QR) break;

    // ---- column-wise QR of block k (near-dependent candidates) ----------
    const int64_t k = ctl.k;
    HIP_TRY(hipMemcpyAsync(hs, r.st, sizeof(DevState), hipMemcpyDeviceToHost, r.s));
    HIP_TRY(hipStreamSynchronize(r.s));
    double* Wn = r.Vslot(k + 1);
    const double* Vk = r.Vslot(k);
    for (int l = 0; l < p; ++l) {
      double a[MAXP];
      for (int q = 0; q < p; ++q) a[q] = hs->Ak[q * MAXP + l];
      TRY(r.colop(Wn, p, l, Wn, p, l, Vk, p, p, a, 1.0));
    }
    double Bk[MAXP * MAXP];
    int taken = hs->taken, nrep = hs->n_replaced, cap = p;
    int e = column_qr(r, Wn, hs->araw, o.gamma, hs->bench_norm0, &taken, &nrep, Bk, &cap);
    if (e && e != BMR_BENCH_EXHAUSTED) return e;
    for (int q = 0; q < MAXP * MAXP; ++q) hs->Bk[q] = Bk[q];
    hs->taken = taken;
    hs->n_replaced = nrep;
    hs->n_explicit += 1;
    hs->lcap = cap;
    hs->cap_status = BMR_BENCH_EXHAUSTED;
    hs->halt = 0;
    hs->reason = REASON_NONE;
    HIP_TRY(hipMemcpyAsync(r.st, hs, sizeof(DevState), hipMemcpyHostToDevice, r.s));
    HIP_TRY(launch_band(r.p, 1, r.red, r.hist, r.st, r.s));
    HIP_TRY(launch_pass2(r.p, r.V, r.M, r.slot, X, r.bench, r.n, r.st, r.s));
    HIP_TRY(hipStreamSynchronize(r.s));
  }
  HIP_TRY(hipMemcpyAsync(hs, r.st, sizeof(DevState), hipMemcpyDeviceToHost, r.s));
  HIP_TRY(hipStreamSynchronize(r.s));
  if (res_hist && o.hist_cap > 0) {
    const int64_t rows = std::min<int64_t>(hs->j, o.hist_cap);
    if (rows > 0)
      HIP_TRY(hipMemcpy(res_hist, r.hist, sizeof(double) * (size_t)rows * p, hipMemcpyDeviceToHost));
  }
  const int status = hs->status == STATUS_RUNNING ? BMR_HIP_ERROR : hs->status;
  finish_stats(status, hs->j, hs->k, hs->rho);
  if (stats) {
    for (int q = 0; q < 4; ++q) stats->t_kernel_ms[q] = nprof ? tk[q] / nprof : 0.0;
    stats->n_profiled = nprof;
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
    case BMR_INVALID_ARG: return "invalid argument";
    case BMR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case BMR_HIP_ERROR: return "HIP runtime error";
    case BMR_NONFINITE: return "non-finite value";
    case BMR_SINGULAR_R: return "singular band QR factor";
    default: return "unknown status";
  }
}

void bmr_default_opts(bmr_opts_t* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->max_iter = 10000;
  o->gamma = 1e-10;
  o->n_bench = 2;
  o->poll_every = 0;
  o->seed = 0;
  o->hist_cap = 0;
  o->flags = 0;
  o->_reserved = 0;
}

int bmr_workspace_bytes(int64_t n, int p, const bmr_opts_t* opts, size_t* bytes) {
  bmr_opts_t o;
  bmr_default_opts(&o);
  if (opts) o = *opts;
  if (!bytes || n < 1 || p < 1 || p > BMR_MAX_P || !opts_valid(o)) return BMR_INVALID_ARG;
  *bytes = layout_for(n, p, o.n_bench, o.hist_cap).total;
  return BMR_CONVERGED;
}

int bmr_solve(const bmr_csr_t* A, const double* B, double* X, int p, const bmr_opts_t* opts, void* workspace,
              size_t workspace_bytes, hipStream_t stream, bmr_stats_t* stats, double* res_hist) {
  bmr_opts_t o;
  bmr_default_opts(&o);
  if (opts) o = *opts;
  if (!csr_valid(A) || !B || !X || !workspace || p < 1 || p > BMR_MAX_P || !opts_valid(o)) return BMR_INVALID_ARG;
  if (((uintptr_t)workspace) % 256 != 0) return BMR_INVALID_ARG;
  Run r{};
  r.A = A;
  r.p = p;
  r.nb = o.n_bench;
  r.n = A->n;
  r.s = stream;
  r.L = layout_for(A->n, p, o.n_bench, o.hist_cap);
  if (workspace_bytes < r.L.total) return BMR_WORKSPACE_TOO_SMALL;
  r.ws = (char*)workspace;
  r.st = (DevState*)(r.ws + r.L.off_state);
  r.red = (double*)(r.ws + r.L.off_red);
  r.part = (double*)(r.ws + r.L.off_part);
  r.hist = (double*)(r.ws + r.L.off_hist);
  r.V = (double*)(r.ws + r.L.off_V);
  r.M = (double*)(r.ws + r.L.off_M);
  r.bench = (double*)(r.ws + r.L.off_bench);
  r.slot = slot_elems(A->n, p);
  hipEvent_t t0, t1;
  if (hipEventCreate(&t0) != hipSuccess) return BMR_HIP_ERROR;
  if (hipEventCreate(&t1) != hipSuccess) return BMR_HIP_ERROR;
  (void)hipEventRecord(t0, stream);
  int status = solve_impl(r, B, X, o, stats, res_hist);
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
    stats->time_ms = ms;
  }
  return status;
}

int bmr_spmm(const bmr_csr_t* A, const double* V, double* W, int p, hipStream_t stream) {
  if (!csr_valid(A) || !V || !W || V == W || p < 1 || p > BMR_MAX_P) return BMR_INVALID_ARG;
  return launch_spmm(p, *A, V, W, stream) == hipSuccess ? BMR_CONVERGED : BMR_HIP_ERROR;
}

int bmr_residual(const bmr_csr_t* A, const double* B, const double* X, int p, double* R, double* norms,
                 void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!csr_valid(A) || !B || !X || !norms || !workspace || p < 1 || p > BMR_MAX_P) return BMR_INVALID_ARG;
  bmr_opts_t o;
  bmr_default_opts(&o);
  const Layout L = layout_for(A->n, p, o.n_bench, 0);
  const size_t need = L.off_part + sizeof(double) * (size_t)p * L.n_wg;
  if (workspace_bytes < need) return BMR_WORKSPACE_TOO_SMALL;
  double* part = (double*)((char*)workspace + L.off_part);
  if (launch_residual(p, *A, B, X, R, part, L.n_wg, stream) != hipSuccess) return BMR_HIP_ERROR;
  std::vector<double> h((size_t)p * L.n_wg);
  if (hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return BMR_HIP_ERROR;
  if (hipStreamSynchronize(stream) != hipSuccess) return BMR_HIP_ERROR;
  for (int c = 0; c < p; ++c) {
    double t = 0.0;
    for (int w = 0; w < L.n_wg; ++w) t += h[(size_t)c * L.n_wg + w];
    norms[c] = sqrt(t);
  }
  return BMR_CONVERGED;
}

}  // extern "C"
