// Internal definitions shared by the HIP kernels and the host driver of
// libbmr: the device-resident solver state, workspace layout and the launch
// wrappers.  Not part of the public ABI (see include/bmr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "bmr.h"

namespace bmr {

constexpr int MAXP = BMR_MAX_P;
constexpr int MAXB = BMR_MAX_BENCH;
constexpr int STATUS_RUNNING = 100;

// The search directions and the iterate (eqs. (4.1)-(4.2)) are applied in
// groups of s = group_len(p) blocks: pass 2 of the group's last block adds
// the group's contributions to X from the group's Lanczos blocks and the two
// search-direction blocks before the group.  The flush moves s + 6 blocks
// per s block iterations, so longer groups move fewer bytes; s is capped so
// that the 3 (s + 2) p x p coefficient blocks of a group fit in the LDS of
// the flush and of the band kernel: 2048 / p^2 up to 32 blocks for p <= 8
// (where the flush runs one wavefront per SIMD), 1024 / p^2 above.  V_k
// lives in slot k mod ring_len(p) of the V ring.
constexpr int MAXS = 32;
__host__ __device__ constexpr int group_len(int p) {
  return p <= 8 ? (2048 / (p * p) > MAXS ? MAXS : 2048 / (p * p)) : (1024 / (p * p) < 2 ? 2 : 1024 / (p * p));
}
__host__ __device__ constexpr int ring_len(int p) { return group_len(p) + 2; }

// Why the device loop stopped (DevState::reason).
enum : int {
  REASON_NONE = 0,
  REASON_FINISHED = 1,     // converged, max_iter or bench exhausted
  REASON_EXPLICIT_QR = 2,  // the Gram QR of the new block was rejected: it runs column by column
  REASON_ERROR = 3,
};

// Number of reduced entries pass 1 produces for block size p and bench nb:
// G = V_k^T W (p x p), Q = W^T W (p x p), P = V_k^T V_k (p x p),
// a = column norms^2 of A V_k (p), W^T g (p x nb), V_k^T g (p x nb).
__host__ __device__ constexpr int n_entries(int p, int nb) { return 3 * p * p + p + 2 * p * nb; }
__host__ __device__ constexpr int off_G(int) { return 0; }
__host__ __device__ constexpr int off_Q(int p) { return p * p; }
__host__ __device__ constexpr int off_P(int p) { return 2 * p * p; }
__host__ __device__ constexpr int off_a(int p) { return 3 * p * p; }
__host__ __device__ constexpr int off_Wg(int p) { return 3 * p * p + p; }
__host__ __device__ constexpr int off_Vg(int p, int nb) { return 3 * p * p + p + p * nb; }

// Device-resident state of one solve.  Written by the host at set-up, then
// only by the single-workgroup band kernel and the single-workgroup decision
// kernels of the column-wise QR.  Small matrices use a fixed stride MAXP:
// M[r * MAXP + c] is row r, column c (0-based).
struct DevState {
  // ---- control --------------------------------------------------------
  int halt;          // != 0: pass 1, the reduction and the band kernel return at once
  int status;        // bmr_status once finished, STATUS_RUNNING before
  int reason;        // REASON_*
  int taken;         // bench vectors consumed
  int64_t k;         // block iteration the next pass 1 works on (1-based)
  int64_t k2;        // block iteration pass 2 applies (0: pass 2 does nothing)
  int64_t j;         // band iterations completed
  int lstar;         // columns of block k2 whose search direction enters X
  int n_replaced;
  int n_explicit;
  int lcap;          // the band kernel processes columns l < lcap of the block (p normally)
  int cap_status;    // status to finish with when it reaches lcap < p
  int _pad0;
  // ---- parameters -------------------------------------------------------
  int p, nb;
  int64_t n;
  int64_t max_iter;
  int64_t hist_cap;
  double tol, gamma, tau_fb;
  double beta[MAXP];          // ||b_i||
  double bench_norm0[MAXB];   // initial norms of the bench vectors
  // ---- band state ------------------------------------------------------
  double Bprev[MAXP * MAXP];  // B_{k-1}: h_{(k-1)p+r+1, (k-2)p+c+1}, upper triangular
  double Ak[MAXP * MAXP];     // A_k: diagonal block of H-bar, symmetric
  double Bk[MAXP * MAXP];     // B_k: upper triangular, diagonal = h_{j+p,j}
  double rot[3][MAXP][MAXP][2];  // Givens (c, s) of the columns of block b, ring b mod 3
  double Shat[MAXP * MAXP];   // live rows of S-hat at the start of block k
  // ---- coefficients for pass 2 of block k2 ------------------------------
  double P2A[MAXP * MAXP];    // W' = W - V_k * P2A
  double P2B[MAXP * MAXP];    // V_{k+1} = W' * P2B^{-1} (upper triangular)
  double bcoef[MAXB * MAXP];  // bench update: g_b -= V_{k+1} bcoef[b]
  double araw[MAXP];          // ||A u_j|| of the block's columns
  double rho[MAXP];           // last rho_j / beta
  // ---- search directions in groups of s = group_len(p) blocks -----------
  // Block k = g + 1 + t of the group that starts after block g sits at
  // position t.  Its search directions satisfy (eq. (4.1))
  //     M_k = V_k C_k + M_{k-1} D_k + M_{k-2} E_k,
  // C_k = R_c^{-1}, D_k = -R_b R_c^{-1}, E_k = -R_a R_c^{-1} (R_a, R_b, R_c: the
  // rows of blocks k-2, k-1, k of R in the columns of block k), and it adds
  // M_k Z_k to X (eq. (4.2); row l of Z_k is z_j^T for j = (k-1)p + l + 1).
  // Columns l >= l* of a finishing block are zero in C, D, E and Z.
  double gC[MAXS][MAXP * MAXP], gD[MAXS][MAXP * MAXP], gE[MAXS][MAXP * MAXP], gZ[MAXS][MAXP * MAXP];
  // The flush after the group's last block g + m (m = flush_len) forms
  //     out_o = [X if o = 0] + sum_{t<m} V_{g+1+t} Y[o][t] + M_g Y[o][MAXS] + M_{g-1} Y[o][MAXS+1],
  // o = 0: X, o = 1: M_{g+m-1}, o = 2: M_{g+m} (the two blocks the next group
  // starts from; not needed when the iteration stops at g + m).
  double Y[3][MAXS + 2][MAXP * MAXP];
  int64_t flush_block;  // g + m of the last group whose coefficients are in Y
  int flush_len;        // m
  int flush_keep;       // != 0: the flush also writes M_{g+m-1} and M_{g+m}
  // ---- column-wise QR on the device (initial QR, rejected Gram route) ----
  // The QR kernels read and write these between launches; the host only
  // enqueues them.  qr_R collects the triangular factor (S at set-up, B_k in
  // the loop), qr_ref the norms the dependence test compares against.
  double qr_R[MAXP * MAXP];
  double qr_ref[MAXP];
  double qr_coef[MAXP + MAXB];  // coefficients of the next column update
  double qr_div;                // divisor of the next normalisation
  int qr_active;                // 0 once the bench ran out: later QR steps do nothing
  int qr_need_bench;            // the current column is dependent: a substitute is needed
  int qr_src;                   // 0: normalise the column itself, 1: take bench vector qr_b
  int qr_b;
  int qr_lcap;                  // first column without a basis vector (p when none)
  int qr_error;                 // a non-finite norm was met
  // ---- retained removed candidates (BMR_FLAG_RETAIN) ----------------------
  // A removed candidate that would have been basis vector u_m is kept,
  // normalised, in slot s of the retained array (n x nb, like the bench),
  // and the new basis vectors u_{m+1} .. u_{m+2p} take one Gram-Schmidt
  // step against it.  Each removal takes a bench vector, so at most nb are
  // ever kept.  While one is in its window the band kernel sends every block
  // to the column-wise QR, which applies those steps.
  // ---- accumulated rotations (BMR_FLAG_ACCUMULATE) -------------------------
  // Qacc[b & 1] holds the p^2 rotations of block b multiplied into one 2p x 2p
  // matrix (rows of blocks b and b+1), formed by the band kernel of block b+1.
  int accumulate;
  double Qacc[2][2 * MAXP][2 * MAXP];
  int retain;
  int n_kept;
  int qr_keep;                  // the current column's candidate is kept in slot qr_keep_slot
  int qr_keep_slot;
  int qr_hit;                   // the current column's substitute was projected out of a kept candidate
  int64_t kept_m[MAXB];
  // With retained candidates the basis is no longer exactly orthonormal, and
  // a new block is orthogonalised in the oracle's order (modified
  // Gram-Schmidt, symmetric coefficients from storage): qr_M[r * MAXP + l]
  // (r >= l) is the coefficient of u_{(k-1)p+r+1} in the candidate of column l.
  double qr_M[MAXP * MAXP];
};
// Retained candidates need a norm above this fraction of the dependence
// test's reference norm (2^-26): below it most of their direction is rounding.
constexpr double RETAIN_FLOOR = 1.0 / 67108864.0;

// Workspace carve-up (offsets into the caller's workspace).  The blocks V, M
// and the bench hold the storage type of the solve (8 bytes for FP64, 4 for
// the FP32 inner solve of BMR_PREC_MIXED); the mixed-precision solver also
// keeps the FP32 matrix values, the FP32 correction D and the FP64 residual R.
// BMR_PREC_RELAXED holds the FP64 blocks and, beside them, the FP32 ring,
// bench and matrix values it switches to.
struct Layout {
  size_t off_state, off_red, off_part, off_hist, off_V, off_M, off_bench;
  size_t off_val32, off_D, off_R;  // BMR_PREC_MIXED; BMR_PREC_RELAXED uses off_val32
  size_t off_V32, off_bench32;  // BMR_PREC_RELAXED only: the FP32 ring and bench after the switch
  size_t off_Y, off_Z;             // BMR_PRECOND_IC0 only: two n x p blocks for the operator
  size_t off_ret;                  // BMR_FLAG_RETAIN only: retained candidates, n x nb
  size_t total;
  int n_wg;  // workgroups of pass 1 (partials)
};

Layout layout_for(int64_t n, int64_t nnz, int p, int nb, int64_t hist_cap, int precision, int precond = 0,
                  bool retain = false);

// An IC(0) factor in its device buffer (see kernels_ic0.hip): device
// pointers into the buffer, and the level boundaries on the host (the
// launches of a level-scheduled solve need them).
struct Ic0View {
  int64_t n = 0, nnz_l = 0;
  int n_levels = 0;
  std::vector<int> level_ptr;  // host, n_levels + 1: rows level_rows[level_ptr[l] .. level_ptr[l+1]) form level l
  const int32_t* level_rows = nullptr;
  const int32_t *lrp = nullptr, *lci = nullptr, *lmap = nullptr, *dmap = nullptr;  // strictly lower part of C
  const int32_t *urp = nullptr, *uci = nullptr, *upos = nullptr;                   // its transpose
  double *lval = nullptr, *uval = nullptr, *diag = nullptr;
  // two-level factors (every row's entries point at rows without entries,
  // as in a red-black ordering): the coefficients divided by the pivot of
  // the row they multiply, so that a solve is one gather
  double *lval_s = nullptr, *uval_s = nullptr;
  int* fail = nullptr;
};
// Reads the header of an IC(0) buffer (synchronously).  0 or a bmr_status error.
int ic0_view(const void* buf, Ic0View* v);
hipError_t launch_ic0_factor(const Ic0View& v, const double* mval, int* fail, hipStream_t s);
// y = C^{-1} rhs (trans = false) or C^{-T} rhs (trans = true), p right-hand
// sides; rhs may be y.  st: a solver state whose halt flag turns the solve
// into a no-op, or NULL.
hipError_t launch_ic0_solve(const Ic0View& v, int p, bool trans, const double* rhs, double* y, const DevState* st,
                            hipStream_t s);
// Pass 1 for a preconditioned operator whose product with V_k is already in
// Z: W = Z - V_{k-1} B_{k-1}^T and the Gram partials, as launch_pass1.
hipError_t launch_pass1_ident(int p, const double* Z, double* Vbase, size_t slot_elems, const double* bench,
                              double* part, int n_wg, int64_t n, DevState* st, hipStream_t s);
// y = (rhs - T rhs) / diag for the scaled strictly triangular part T of a
// two-level IC(0) factor: one whole triangular solve (rhs must not be y).
hipError_t launch_trisolve2(int p, const int32_t* rp, const int32_t* ci, const double* va, const double* diag,
                            int64_t n, const double* rhs, double* y, const DevState* st, hipStream_t s);
// Pass 1 on C^{-1} Z for a two-level IC(0) factor, the forward solve done on
// the fly from the factor's scaled strictly lower part (lrp, lci, lval_s).
hipError_t launch_pass1_tri(int p, const int32_t* lrp, const int32_t* lci, const double* lval_s, const double* diag,
                            const double* Z, double* Vbase, size_t slot_elems, const double* bench, double* part,
                            int n_wg, int64_t n, DevState* st, hipStream_t s);
// R = B - A X (R may be NULL) and the column norms ||b_i - A x_i|| (host
// output), with p * n_wg doubles of partial sums in part and p reduced sums in
// red (device scratch); synchronises the stream.  0 or a bmr_status error.
int residual_norms(const bmr_csr_t* A, const double* B, const double* X, int p, double* R, double* part, int n_wg,
                   double* red, hipStream_t s, double* norms);
int pass1_grid(int64_t n, int p);  // the most pass-1 workgroups (sizes the partial sums)
// The pass-1 workgroups of a solve in storage type T: one resident round on
// the current device, at most pass1_grid(n, p).
template <typename T>
int pass1_resident_grid(int64_t n, int p);

// ---- launch wrappers (kernels_*.hip) ------------------------------------
// T = double (FP64 solve) or float (inner solve of the mixed-precision solver);
// val holds the matrix values in T (A.val itself for double).
template <typename T>
hipError_t launch_pass1(int p, const bmr_csr_t& A, const T* val, T* Vbase, size_t slot_elems, const T* bench,
                        double* part, int n_wg, DevState* st, hipStream_t s);
template <typename T>
hipError_t launch_spmm(int p, const bmr_csr_t& A, const T* val, const T* V, T* W, hipStream_t s,
                       const DevState* st = nullptr);  // st: halt flag makes it a no-op
hipError_t launch_residual(int p, const bmr_csr_t& A, const double* B, const double* X, double* R,
                           double* part, int n_wg, hipStream_t s);
hipError_t launch_reduce(const double* part, int n_wg, int n_ent, double* red, DevState* st, int check_halt,
                         hipStream_t s);
hipError_t launch_band(int p, int mode, int nb, const double* red, double* hist, DevState* st, hipStream_t s);
template <typename T>
hipError_t launch_pass2(int p, T* Vbase, size_t slot_elems, T* bench, int64_t n, DevState* st, hipStream_t s);
// The group's search directions into X (and the next group's two M blocks);
// does nothing unless the band kernel recorded a group ending at block k.
template <typename T>
hipError_t launch_flush(int p, const T* Vbase, T* Mbase, size_t slot_elems, T* X, int64_t n, int64_t k,
                        const DevState* st, hipStream_t s);
// The flush with the ring's Lanczos blocks in FP32 and the search directions
// and X in FP64 (BMR_PREC_RELAXED after its switch).
hipError_t launch_flush_vf(int p, const float* Vbase, double* Mbase, size_t slot_elems, double* X, int64_t n,
                           int64_t k, const DevState* st, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* x, size_t count, T v, hipStream_t s);
template <typename T>
hipError_t launch_bench_init(T* bench, int64_t n, int nb, uint64_t seed, hipStream_t s);
// Column-wise QR on the device (kernels_colqr.hip): the QR of the p columns
// of D in place, written as a fixed launch sequence whose decisions (the
// dependence test, the substitute taken, exhaustion) are taken by
// single-workgroup kernels from device-resident sums, so the host never
// waits inside it.  SETUP: the initial QR of B (reference norms qr_ref set
// by the host), the factor left in qr_R.  LOOP: the new block of block
// iteration k after a rejected Gram route: W -= V_k A_k first (A_k and the
// reference norms ||A u_j|| from the state), and at the end B_k := qr_R, the
// column cap and the counters go to the state and the device loop resumes.
enum { QR_SETUP = 0, QR_LOOP = 1 };
// ret: the retained candidates (n x nb, storage type T), or NULL when none are kept.
template <typename T>
hipError_t launch_colqr(int p, int mode, T* D, const T* Vk, T* bench, int nb, int64_t n, double* part, int n_wg,
                        DevState* st, hipStream_t s, T* ret = nullptr);
int colqr_grid(int64_t n);
// Column kernels of the set-up norms, FP64 arithmetic.
//   coldots: part[wg * (m+1) + r] = sum_i X[i*ldx + r] * Y[i*ldy + yc] (r < m), last = sum Y^2
template <typename T>
hipError_t launch_coldots(const T* Y, int ldy, int yc, const T* X, int ldx, int m, int64_t n, double* part,
                          int n_wg, hipStream_t s);
int coldots_grid(int64_t n);
// Conversions of the mixed-precision solver: dst = (float)src; x += (double)d; dst = src.
hipError_t launch_to_f32(const double* src, float* dst, size_t count, hipStream_t s);
hipError_t launch_add_f32(double* x, const float* d, size_t count, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, size_t count, hipStream_t s);
// g_e = -(Lam_i . X_j + Lam_j . X_i) / 2 for every stored entry e = (i, j) of A.
hipError_t launch_pattern_grad(int p, const bmr_csr_t& A, const double* Lam, const double* X, double* g,
                               hipStream_t s);

}  // namespace bmr
