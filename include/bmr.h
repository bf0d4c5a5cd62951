/*
 * bmr.h -- band-Lanczos block MINRES on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libbmr.so.  The library solves
 *
 *     A X = B,   A in R^{n x n} sparse, symmetric (indefinite),  B in R^{n x p},
 *
 * (the problem statement, eq. (1.1) of K. M. Soodhalter, "A block MINRES
 * algorithm based on the band Lanczos method") by block MINRES over the band
 * Lanczos basis: one basis vector per band iteration j, the operator applied
 * to a block of p vectors every p iterations, dependent candidates replaced by
 * pre-generated random vectors kept orthogonal to the basis, the band Hessenberg
 * matrix reduced by Givens rotations and X updated progressively
 * (Sections 3-5 and Algorithm 7.1 of the paper).
 *
 * Conventions shared by every entry point
 *   - Precision: the interface is IEEE binary64 throughout.  bmr_solve runs
 *     either in binary64 (BMR_PREC_FP64) or as a binary32 inner solver inside
 *     binary64 iterative refinement (BMR_PREC_MIXED, see bmr_opts_t).
 *   - Blocks (B, X, V, W, R) are n x p, row-interleaved: element (i, c) is at
 *     offset i*p + c.  This is a C-contiguous (n, p) array.
 *   - A is CSR with int32 row pointers and column indices, column indices
 *     sorted and unique within each row.  A must be symmetric; this is not
 *     checked.
 *   - Pointers documented as "device" must point to memory of the current
 *     HIP device; "host" pointers to ordinary host memory.  The caller owns
 *     all memory.  The library never allocates device memory: scratch comes
 *     from the caller's workspace.
 *   - All device work is enqueued on the given stream (NULL = legacy default
 *     stream).  Entry points that return host results synchronise that
 *     stream before returning.
 *   - Return value: a bmr_status code.  Negative values are errors; on error
 *     the contents of output arrays are unspecified.
 */
#ifndef BMR_H
#define BMR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BMR_VERSION 10300 /* 1.3.0 */
#define BMR_MAX_P 16      /* largest block size p */
#define BMR_MAX_BENCH 4   /* largest substitutes bench */

enum bmr_status {
  BMR_CONVERGED = 0,          /* max_i ||b_i - A x_i|| / ||b_i|| < tol (recurrence residual) */
  BMR_MAX_ITER = 1,           /* max_iter band iterations done; X is the last iterate */
  BMR_BENCH_EXHAUSTED = 2,    /* a dependent vector found no substitute; X is the last iterate */
  BMR_STAGNATED = 3,          /* BMR_PREC_MIXED: a refinement cycle reduced the largest explicit
                                 relative residual by less than half; X is the last iterate */
  BMR_INVALID_ARG = -1,       /* p outside [1, BMR_MAX_P], n < 1, NULL pointer, tol <= 0, ... */
  BMR_WORKSPACE_TOO_SMALL = -2,
  BMR_HIP_ERROR = -3,         /* a HIP runtime call failed */
  BMR_NONFINITE = -4,         /* NaN or Inf in B or in a computed coefficient */
  BMR_SINGULAR_R = -5,        /* a diagonal entry of the band QR factor R is zero */
  BMR_IC0_BREAKDOWN = -6      /* bmr_ic0_factor: a pivot of the incomplete factorisation was not positive */
};

/* Sparse symmetric matrix, CSR.  All pointers are device pointers. */
typedef struct bmr_csr {
  int64_t n;                /* rows = columns, 1 <= n < 2^31 */
  int64_t nnz;              /* stored entries, < 2^31 */
  const int32_t* row_ptr;   /* n + 1 entries, row_ptr[0] = 0, row_ptr[n] = nnz */
  const int32_t* col_idx;   /* nnz entries */
  const double* val;        /* nnz entries */
} bmr_csr_t;

/* Solver options (Algorithm 7.1's eps and M, the dependence tolerance of
 * Section 5 and the bench size of Section 5.1).  bmr_default_opts fills it. */
typedef struct bmr_opts {
  double tol;          /* eps > 0: stop when every column has recurrence residual
                          ||b_i - A x_i|| / ||b_i|| < tol (columns with b_i = 0 count
                          as converged with x_i = 0).  Default 1e-8. */
  int64_t max_iter;    /* M >= 1: band iterations j (p per block iteration). Default 10000. */
  double gamma;        /* dependence tolerance, relative: the candidate of iteration j
                          is dependent when its norm after orthogonalisation is
                          <= gamma * ||A u_j|| (initial QR: <= gamma * ||b_i||).
                          Default 1e-10. */
  int32_t n_bench;     /* substitute vectors, 0 .. BMR_MAX_BENCH.  Default 2. */
  int32_t poll_every;  /* block iterations enqueued between host status polls; 0 = auto */
  uint64_t seed;       /* seed of the substitute generator (SplitMix64).  Default 0. */
  int64_t hist_cap;    /* rows of the residual history kept on the device (>= 0).
                          Default 0. */
  uint32_t flags;      /* BMR_FLAG_* bits.  Default 0. */
  int32_t precision;   /* BMR_PREC_FP64 (default), BMR_PREC_MIXED or BMR_PREC_RELAXED. */
  double inner_tol;    /* BMR_PREC_MIXED: each refinement cycle runs the FP32 inner solve
                          until its recurrence residual has dropped by this factor
                          (or below what the outer tolerance still needs).
                          0 < inner_tol < 1.  Default 1e-6. */
  int32_t max_refine;  /* BMR_PREC_MIXED: refinement cycles at most (>= 1).  Default 30. */
  int32_t precond;     /* BMR_PRECOND_NONE (default) or BMR_PRECOND_IC0: sizes the workspace of
                          bmr_workspace_bytes for bmr_solve_ic0 (bmr_solve accepts NONE only). */
  double relax_tol;    /* BMR_PREC_RELAXED: the iteration continues in binary32 once every
                          column's recurrence residual is below relax_tol (relative to
                          ||b_i||).  0 (default) = min(1e-2, 1e3 * tol); else tol < relax_tol < 1. */
} bmr_opts_t;

/* bmr_opts_t.precision.
 *
 * BMR_PREC_FP64: the solver of Algorithm 7.1 in binary64.
 *
 * BMR_PREC_MIXED: iterative refinement in binary64 around the same solver
 * run with binary32 data (not part of the paper).  Each cycle computes the
 * explicit residual R = B - A X in binary64, stops when every column has
 * ||r_i|| / ||b_i|| < tol, and otherwise solves A D = R with the block
 * operator, the Gram products, the update pass and all n-length vectors in
 * binary32 (binary32 accumulation), while the band kernel (Givens QR,
 * Cholesky of the new block, dependence test, residual recurrence) stays in
 * binary64; then X += D in binary64.  The inner dependence tolerance is
 * max(gamma, 1e-5), the level at which binary32 data cannot tell a dependent
 * candidate from rounding noise.  The stopping test is on the explicit
 * binary64 residual, not on the recurrence. */
#define BMR_PREC_FP64 0
#define BMR_PREC_MIXED 1
/* BMR_PREC_RELAXED: one run of the solver of Algorithm 7.1 (not part of the
 * paper), in binary64 until every column's recurrence residual is below
 * relax_tol, then with the block operator, the Gram products, the update
 * pass, the Lanczos blocks and the bench in binary32 as in BMR_PREC_MIXED's
 * inner solve (the band kernel stays binary64), without a restart: at the
 * end of a group of blocks the two Lanczos blocks the iteration needs next
 * and the bench are rounded to binary32, while the search directions and X
 * stay binary64 (the flush reads the binary32 blocks into binary64 sums;
 * the search directions' three-term recurrence would otherwise carry
 * binary32 rounding at the scale of the whole solution into the residual
 * gap).  This is a relaxed-accuracy inexact Krylov method: a product's error
 * may grow as the residual falls (Simoncini and Szyld, SIAM J. Sci. Comput.
 * 25, 2003; van den Eshof and Sleijpen, SIAM J. Matrix Anal. Appl. 26,
 * 2004): the error a product may carry grows like tol * sigma_min(A) /
 * ||r_j||, so binary32 rounding (u = 2^-24 of ||A||) may enter once the
 * residual is below about tol * sigma_min(A) / (u ||A||).  The default
 * switch level 1e3 * tol keeps the explicit residual at tol on a 7-point
 * Laplacian with condition number 4e4; better conditioned systems allow a
 * larger relax_tol, worse ones need a smaller.  The stopping test is on
 * the recurrence, as for BMR_PREC_FP64; res_explicit reports the explicit
 * residual.  Not with BMR_FLAG_RETAIN. */
#define BMR_PREC_RELAXED 2

/* bmr_opts_t.precond. */
#define BMR_PRECOND_NONE 0
#define BMR_PRECOND_IC0 1

/* bmr_opts_t.flags: time every kernel of every block iteration with HIP
 * events on the solve stream (one block iteration in flight at a time; the
 * averages go to bmr_stats_t.t_kernel_ms). */
#define BMR_FLAG_PROFILE 1u

/* bmr_opts_t.flags: keep removed candidates (Section 5.1, last paragraph).
 * A candidate removed as dependent in place of basis vector u_m is kept,
 * normalised, when its norm exceeds 2^-26 times the reference norm of the
 * dependence test (below that most of its direction is rounding error, so
 * with the default gamma nothing is kept), and the new basis vectors
 * u_{m+1} .. u_{m+2p} (those whose band window would have held u_m) take one
 * Gram-Schmidt step against it after their orthogonalisation against the
 * band, with the coefficient not recorded in H-bar.  Blocks in such a window
 * are orthogonalised column by column.  Sizes the workspace (n x n_bench
 * more entries). */
#define BMR_FLAG_RETAIN 2u

/* bmr_opts_t.flags: apply the rotations of the two previous blocks to a new
 * block's columns as accumulated matrices (Section 4's remark on keeping the
 * action of a block of reflectors as one matrix, applied by matrix
 * products): the p^2 Givens rotations of each block become one orthogonal
 * 2p x 2p matrix.  The same iterate in exact arithmetic; only the rounding
 * of the band factor changes. */
#define BMR_FLAG_ACCUMULATE 4u

/* Host-side result summary. */
typedef struct bmr_stats {
  int32_t status;          /* enum bmr_status */
  int32_t n_replaced;      /* basis vectors taken from the bench */
  int64_t band_iters;      /* band iterations j performed */
  int64_t block_iters;     /* operator applications (block iterations) */
  int32_t n_explicit_qr;   /* block iterations whose new-block QR ran column by column */
  int32_t p;
  double res_rec[BMR_MAX_P];  /* final recurrence residual ||b_i - A x_i|| / ||b_i|| */
  double time_ms;          /* wall time of the solve on the stream (HIP events) */
  /* with BMR_FLAG_PROFILE: mean duration per block iteration of the four
   * kernels (block operator pass, partial-sum reduction, band kernel, update
   * pass) and the number of block iterations timed */
  double t_kernel_ms[4];
  int64_t n_profiled;
  int32_t precision;       /* the bmr_opts_t.precision the solve ran with */
  int32_t n_refine;        /* BMR_PREC_MIXED: refinement cycles run (inner solves) */
  double res_true[BMR_MAX_P]; /* BMR_PREC_MIXED: final explicit ||b_i - A x_i|| / ||b_i||
                                 in binary64 (also copied to res_rec); 0 for BMR_PREC_FP64 */
  double res_explicit[BMR_MAX_P]; /* explicit ||b_i - A x_i|| / ||b_i|| of the returned X,
                                     computed in binary64 after the iteration (one extra
                                     operator application; Algorithm 7.1's output);
                                     0 where b_i = 0 */
  int32_t n_retained;      /* BMR_FLAG_RETAIN: removed candidates kept */
  int32_t _pad;
  int64_t switch_iter;     /* BMR_PREC_RELAXED: band iterations run in binary64 before the
                              switch to binary32 (0: the solve ended before it) */
} bmr_stats_t;

/* Library version, BMR_VERSION of the build. */
int bmr_version(void);

/* Static, human-readable name of a status code. */
const char* bmr_status_string(int status);

/* Fill *opts with the defaults listed in bmr_opts_t.  opts: host. */
void bmr_default_opts(bmr_opts_t* opts);

/* Bytes of device workspace bmr_solve and bmr_residual need for a system of
 * n rows, nnz stored matrix entries, block size p and the given options (opts
 * may be NULL for defaults; nnz only matters for BMR_PREC_MIXED, which keeps a
 * binary32 copy of the matrix values).  bytes: host output.  Returns
 * BMR_INVALID_ARG for p outside [1, BMR_MAX_P], n < 1, nnz < 0 or invalid
 * options. */
int bmr_workspace_bytes(int64_t n, int64_t nnz, int p, const bmr_opts_t* opts, size_t* bytes);

/* Solve A X = B with X_0 = 0 (eq. (1.1); Algorithm 7.1 inputs and outputs).
 *
 *   A          host pointer to a bmr_csr_t whose arrays are on the device.
 *   B          device, n x p row-interleaved, read only.
 *   X          device, n x p row-interleaved, output (overwritten).  Must not
 *              alias B or the workspace.
 *   p          block size, 1 <= p <= BMR_MAX_P.
 *   opts       host, may be NULL (defaults).
 *   workspace  device, at least bmr_workspace_bytes(n, A->nnz, p, opts) bytes,
 *              256-byte aligned; contents on entry are ignored.
 *   stream     HIP stream all work is enqueued on.
 *   stats      host, may be NULL.
 *   res_hist   host, may be NULL; else at least opts->hist_cap * p doubles.
 *              BMR_PREC_FP64: row j-1 receives rho_j^{(i)} / ||b_i|| (eq. (3.5))
 *              for band iterations j = 1 .. min(band_iters, hist_cap).
 *              BMR_PREC_MIXED: row c-1 receives the explicit relative residual
 *              ||b_i - A x_i|| / ||b_i|| after refinement cycle c.
 *              0 where b_i = 0.
 *
 * B and X must be 16-byte aligned.  The stream is synchronised before return.
 * Status: BMR_CONVERGED, BMR_MAX_ITER, BMR_BENCH_EXHAUSTED, BMR_STAGNATED or
 * an error code.  With BMR_PREC_MIXED, band_iters and block_iters count all
 * inner solves, and max_iter bounds their sum. */
int bmr_solve(const bmr_csr_t* A, const double* B, double* X, int p, const bmr_opts_t* opts,
              void* workspace, size_t workspace_bytes, hipStream_t stream, bmr_stats_t* stats,
              double* res_hist);

/* W = A V, the block operator application of Algorithm 7.1 (A applied to p
 * vectors at once; each row of A is read once for all p columns).
 * V, W: device, n x p row-interleaved, 16-byte aligned, must not alias.
 * Asynchronous: returns after enqueueing on stream. */
int bmr_spmm(const bmr_csr_t* A, const double* V, double* W, int p, hipStream_t stream);

/* W = A V in binary32 (the block operator of the mixed-precision inner
 * solve): the structure of A with the binary32 values val32 (device, nnz
 * entries), V and W device n x p binary32 row-interleaved, 16-byte aligned,
 * not aliasing.  Products and sums in binary32.  Asynchronous. */
int bmr_spmm_f32(const bmr_csr_t* A, const float* val32, const float* V, float* W, int p, hipStream_t stream);

/* Gradient of a scalar loss L(X) of the solution X = A^{-1} B with respect to
 * the stored entries of A, given the adjoint solution Lam = A^{-1} dL/dX
 * (computed with bmr_solve on the same A, which is symmetric).  Since
 * dL = <Lam, dB> - <Lam X^T, dA>, the gradient restricted to A's pattern and
 * symmetrised (the gradient with respect to symmetric perturbations supported
 * on the pattern) is, for the stored entry e = (i, j),
 *     grad[e] = -(Lam_i . X_j + Lam_j . X_i) / 2,
 * where Lam_i . X_j is the dot product of row i of Lam and row j of X.  Not
 * part of the paper: the backward pass of a differentiable solve.
 *   Lam, X     device, n x p row-interleaved binary64.
 *   grad       device, A->nnz doubles, in the order of A's entries.
 * Asynchronous. */
int bmr_pattern_grad(const bmr_csr_t* A, const double* Lam, const double* X, int p, double* grad,
                     hipStream_t stream);

/* Explicit residual R = B - A X and its column norms (the quantity the
 * stopping test of Algorithm 7.1 bounds).
 *   B, X       device, n x p row-interleaved; X 16-byte aligned.
 *   R          device n x p output, or NULL to compute the norms only.
 *   norms      host, p doubles: ||b_i - A x_i||.
 *   workspace  device, >= bmr_workspace_bytes(n, 0, p, NULL) bytes.
 * Synchronises the stream. */
int bmr_residual(const bmr_csr_t* A, const double* B, const double* X, int p, double* R,
                 double* norms, void* workspace, size_t workspace_bytes, hipStream_t stream);

/* The explicit residual of bmr_residual without a workspace, for callers that
 * cannot allocate or pass device memory (code under graph capture, serving
 * loops, harnesses that forbid allocation).  Same arguments and results as
 * bmr_residual (the same kernels and summation order, so the same bits),
 * with the partial sums in a static device array of the library: 2048 x 16
 * partial sums + 16 reduced sums (262 KB per device, held until the process
 * ends), enough for every valid n and p.  Calls no allocator.  Every call on
 * a device shares that device's array: calls that overlap on one device (two
 * streams, two host threads) race.  Synchronises the stream. */
int bmr_residual_noalloc(const bmr_csr_t* A, const double* B, const double* X, int p, double* R, double* norms,
                         hipStream_t stream);

/* ---- IC(0) preconditioning --------------------------------------------
 *
 * The paper's experiments precondition with the incomplete Cholesky factor
 * of the Laplacian part of the matrix (Section 8), without saying how the
 * preconditioner enters Algorithm 7.1.  Here: M = C C^T with C the IC(0)
 * factor of a symmetric matrix M (C lower triangular with the pattern of the
 * lower triangle of M, (C C^T)_{ij} = M_{ij} on that pattern), and split
 * preconditioning: block MINRES on C^{-1} A C^{-T} with right-hand sides
 * C^{-1} B, then X = C^{-T} X-hat.  Column i of the iterate minimises
 * ||C^{-1} (b_i - A x)|| over the preconditioned block Krylov space (for
 * p = 1 the iterates of MINRES preconditioned with M^{-1}).
 *
 * The factor lives in a caller-owned device buffer (the "IC(0) object").
 * Its set-up reads the pattern of M on the host once (integer work: the
 * strictly lower pattern, the level of every row for the level-scheduled
 * factorisation and solves, the transposed pattern); the factorisation and
 * every triangular solve run on the device. */

/* Device bytes of an IC(0) object for a matrix with n rows and nnz stored
 * entries.  bytes: host output. */
int bmr_ic0_bytes(int64_t n, int64_t nnz, size_t* bytes);

/* Set up the IC(0) object of M in buf and factorise M on the device.
 *   M      host pointer to a bmr_csr_t on the device; symmetric, every
 *          diagonal entry stored, column indices sorted and unique.
 *   buf    device, >= bmr_ic0_bytes(M->n, M->nnz) bytes, 256-byte aligned,
 *          owned by the caller; it must outlive every use of the object.
 * Synchronises the stream.  Returns BMR_IC0_BREAKDOWN when a pivot is not
 * positive (IC(0) does not exist for every symmetric positive definite M;
 * it does for M-matrices such as Laplacians), BMR_INVALID_ARG for a
 * malformed pattern or a missing diagonal entry. */
int bmr_ic0_factor(const bmr_csr_t* M, void* buf, size_t bytes, hipStream_t stream);

/* W = C^{-1} V (trans = 0, forward substitution) or W = C^{-T} V (trans != 0,
 * backward substitution) for the factor in the IC(0) object ic0; V, W device
 * n x p row-interleaved (W may be V).  Asynchronous after reading the
 * object's header. */
int bmr_ic0_apply(const void* ic0, const double* V, double* W, int p, int trans, hipStream_t stream);

/* Solve A X = B (X_0 = 0) by block MINRES with the split IC(0)
 * preconditioner of the object ic0 (n must match A).  Arguments as in
 * bmr_solve, binary64 only; the workspace must hold
 * bmr_workspace_bytes(n, nnz, p, opts with precond = BMR_PRECOND_IC0) bytes;
 * X must not alias B.  The stopping test, res_rec and the history refer to
 * the preconditioned residual ||C^{-1}(b_i - A x_i)|| / ||C^{-1} b_i||;
 * res_explicit is ||b_i - A x_i|| / ||b_i||. */
int bmr_solve_ic0(const bmr_csr_t* A, const void* ic0, const double* B, double* X, int p, const bmr_opts_t* opts,
                  void* workspace, size_t workspace_bytes, hipStream_t stream, bmr_stats_t* stats,
                  double* res_hist);

#ifdef __cplusplus
}
#endif

#endif /* BMR_H */
