"""Band-Lanczos block MINRES in binary64, one Lanczos vector per iteration.

TEST INFRASTRUCTURE (see ``oracle/__init__.py``): only tests, the smoke check
and the benchmark's CPU-baseline leg may use this module.

What is computed.  For A symmetric (indefinite) and B in R^{n x p}, after
band iteration j the iterate X_j has, column by column, the minimal residual
||b_i - A x|| over x in span{u_1, ..., u_j}, where u_1..u_p is the QR basis of
B and every later u_{j+p} is A u_j orthogonalised against the band
(Section 3, eqs. (3.2)-(3.3)).  The iteration reaches it through the short
recurrences of Section 4 (search directions, eq. (4.1); progressive update,
eq. (4.2)) driven by the loop of Algorithm 7.1 ("Block MINRES (band Lanczos
version)"), with dependent candidates replaced from the dynamic substitutes
bench of Section 5.1.

Readings taken where the printed text is garbled or silent (each one is cited
again where the code depends on it):

  R1  Band window (eq. (2.6), Algorithm 2.1): A u_j is orthogonalised against
      u_i for i = max(1, j-p) ... j+p-1.
  R2  Operator application (Algorithm 7.1): W = A [u_j ... u_{j+p-1}] whenever
      (j-1) mod p = 0, for every p >= 1; column l = ((j-1) mod p) + 1 of W is
      A u_j.
  R3  The two update statements of the orthogonalisation read
      w <- w - h_{i,j} u_i.  For i < j the coefficient is the stored h_{j,i}
      (symmetry, Section 7's C_{pxp} queue); for i >= j it is the modified
      Gram-Schmidt inner product u_i^T w.
  R4  The new vector is u_{j+p} = w / h_{j+p,j}.
  R5  Initial QR (eq. (3.2), F_0 = B since X_0 = 0): classical Gram-Schmidt
      applied twice per column, S upper triangular with S(i,i) >= 0.  Column i
      counts as dependent when S(i,i) <= gamma ||b_i||; then S(i,i) := 0 and a
      bench vector takes the place of u_i.
  R6  S-hat starts as E_1 S = [S; 0]; at iteration j only rows j..j+p change.
  R7  The band QR of H-bar (Section 4) uses Givens rotations instead of
      Householder reflectors: column j is reduced by p rotations of the row
      pairs (j, j+t), t = 1..p, each with r = hypot(a, b), c = a/r, s = b/r,
      and the identity when b = 0.  The same rotations act on rows j..j+p of
      S-hat (Section 4 text; the printed algorithm names only the H column).
      R, the m_j and the z_j then differ from the Householder form only in
      row signs; X_j, rho_j, U and H-bar do not change.
  R8  Search directions (eq. (4.1)): the sum starts at max(1, j-2p); for j = 1
      it is empty and m_1 = u_1 / r_{1,1}.
  R9  Stopping (Algorithm 7.1's loop test and output statement): after
      iteration j, rho_j^{(i)} = ||S-hat(j+1:j+p, i)|| (eq. (3.5)); stop when
      max over columns with ||b_i|| > 0 of rho_j^{(i)} / ||b_i|| < eps.  The
      test is made at j = 0 too; at most M iterations are run.
  R10 Dependence (Section 5, Section 5.1): the candidate is dependent when
      h_{j+p,j} <= gamma ||A u_j|| (the paper's absolute test h <= gamma made
      relative, identical when ||A u_j|| = 1).  Then h_{j+p,j} := 0 and
      u_{j+p} is the next bench vector.
  R11 Bench (Section 5.1): n_b random vectors are made before the iteration
      and each is orthogonalised (one Gram-Schmidt step) against every new
      basis vector as soon as it exists, u_1..u_p included.  A bench vector
      taken into the basis is normalised.  With no vector left, or one whose
      norm has fallen to <= gamma times its initial norm, the solve stops with
      BENCH_EXHAUSTED and returns the last iterate.
  R12 A removed candidate is discarded by default.  With ``retain=True``
      (Section 5.1's last paragraph: a removed vector is kept, and new
      Lanczos vectors are still orthogonalised against it until it would
      have left the band) see R13.
  R13 Retained removed vectors.  The removed candidate would have been basis
      vector u_m; the new basis vectors whose window would have held it are
      u_{m+1} .. u_{m+2p}.  Each of them, after the band orthogonalisation
      (and after the CGS2 of the initial QR), takes one Gram-Schmidt step
      against the retained vector, normalised, before its norm and the
      dependence test; the coefficient is not recorded in H-bar (as the
      paper says, this leaves the mathematical derivation).  The substitute
      that takes u_m's place (and any substitute taken while a retained
      candidate's window is open, u_m included) also takes one Gram-Schmidt
      step against it and is normalised again: the retained direction is
      orthogonal to u_1 .. u_{m-1} (it is their remainder), so with the
      substitute and the later vectors kept out of it the basis stays
      orthonormal, and only the unrecorded coefficients are lost.  A
      candidate is retained only when its norm exceeds 2^-26 times the
      reference norm of the dependence test: below that most of its
      direction is rounding error (an exactly dependent candidate leaves
      only rounding noise), so with the default gamma nothing is ever
      retained.
  R14 Accumulated rotations (the remark of Section 4 on keeping the action
      of a block of reflectors as one matrix applied by matrix products,
      which the paper's own code does not do): with ``accumulate=True`` the
      p^2 rotations of each complete block b of p columns are multiplied
      into one orthogonal 2p x 2p matrix Q_b acting on the rows of blocks b
      and b+1, and column j of block k applies Q_{k-2} and Q_{k-1} as
      matrix-vector products before the rotations of the earlier columns of
      its own block.  The rotations Q_{k-2} holds beyond those of columns
      j-2p .. j-1 act on rows of column j that are still zero, so the
      result is the sequential one in exact arithmetic; the rows above the
      window stay exact zeros.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .rng import bench_vector

CONVERGED = 0
MAX_ITER = 1
BENCH_EXHAUSTED = 2
SINGULAR_R = -5


@dataclass
class Result:
    X: np.ndarray                 # (n, p) final iterate
    status: int                   # CONVERGED / MAX_ITER / BENCH_EXHAUSTED / SINGULAR_R
    iters: int                    # band iterations j performed
    beta: np.ndarray              # (p,) ||b_i||
    hist: np.ndarray              # (iters, p) rho_j^{(i)} / ||b_i|| (0 where b_i = 0)
    S: np.ndarray                 # (p, p) initial QR factor
    replaced: list                # basis indices (1-based) filled from the bench
    # filled only with record=True
    U: Optional[np.ndarray] = None       # (n, iters+p) basis u_1..u_{j+p}
    H: Optional[np.ndarray] = None       # (iters+p, iters) H-bar_j
    R: Optional[np.ndarray] = None       # (iters, iters) R_j (Givens form)
    Z: Optional[np.ndarray] = None       # (iters, p) rows z_j^T
    Xs: list = field(default_factory=list)  # X_1 .. X_j
    retained: list = field(default_factory=list)  # R13: basis indices m of retained removed candidates


def _givens(a: float, b: float):
    """Rotation (c, s) with [c s; -s c] [a; b] = [r; 0], r = hypot(a, b) >= 0;
    the identity when b = 0 (reading R7)."""
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


RETAIN_FLOOR = 2.0 ** -26   # R13: smallest retained norm, relative to the reference norm


def solve(A, B, tol: float = 1e-8, max_iter: int = 1000, gamma: float = 1e-10,
          n_bench: int = 2, seed: int = 0, record: bool = False, retain: bool = False,
          accumulate: bool = False) -> Result:
    """Solve A X = B (A symmetric, scipy CSR or anything with ``@``) by band-
    Lanczos block MINRES with X_0 = 0.

    ``tol`` is eps of Algorithm 7.1 relative to ||b_i||, ``max_iter`` is M (band
    iterations), ``gamma`` the relative dependence tolerance, ``n_bench`` and
    ``seed`` the size and generator seed of the substitutes bench; ``retain``
    keeps removed candidates (R13); ``accumulate`` applies the rotations of
    whole blocks as accumulated matrices (R14).
    """
    B = np.asarray(B, dtype=np.float64)
    if B.ndim != 2:
        raise ValueError("B must be (n, p)")
    n, p = B.shape
    beta = np.array([np.linalg.norm(B[:, i]) for i in range(p)])
    live = beta > 0

    # ---- dynamic substitutes bench (Section 5.1; R11) -----------------------
    bench = [bench_vector(n, b, seed) for b in range(n_bench)]
    bench_norm0 = [np.linalg.norm(g) for g in bench]
    taken = 0

    def orthogonalise_bench(v):
        # one Gram-Schmidt step of every unused bench vector against new u
        for g in bench[taken:]:
            g -= (v @ g) * v

    def take_bench():
        nonlocal taken
        if taken >= len(bench):
            return None
        g = bench[taken]
        nrm = np.linalg.norm(g)
        if nrm <= gamma * bench_norm0[taken]:
            return None
        taken += 1
        return g / nrm

    u = {}          # 1-based basis vectors u_i (a sliding window unless record)
    replaced = []
    kept = []       # R13: (m, unit vector) of retained removed candidates

    def project_kept(w, m_new):
        # one Gram-Schmidt step of the new basis vector u_{m_new} against every
        # retained vector whose band window would still hold it
        for m, r in kept:
            if m + 1 <= m_new <= m + 2 * p:
                w -= (r @ w) * r

    kept_at = []

    def substitute_out_of_kept(g, m):
        # R13: a substitute taken as u_m while retained candidates apply to
        # it (their window m_k .. m_k + 2p, m_k included) is kept out of them
        hit = False
        for mk, r in kept:
            if mk <= m <= mk + 2 * p:
                g = g - (r @ g) * r
                hit = True
        return g / np.linalg.norm(g) if hit else g

    def keep(m, w, nrm, ref):
        # kept only when a substitute remains to take its place (otherwise the
        # solve ends at this candidate anyway)
        if retain and nrm > RETAIN_FLOOR * ref and taken < len(bench):
            kept.append((m, w / nrm))
            kept_at.append(m)

    # ---- initial QR, F_0 = U_p S (eq. (3.2); R5) --------------------------
    S = np.zeros((p, p))
    for i in range(p):
        w = B[:, i].copy()
        if i:
            Up = np.column_stack([u[r] for r in range(1, i + 1)])
            for _ in range(2):                       # CGS applied twice
                c = Up.T @ w
                S[:i, i] += c
                w -= Up @ c
        project_kept(w, i + 1)
        sigma = np.linalg.norm(w)
        if sigma <= gamma * beta[i]:
            keep(i + 1, w, sigma, beta[i])
            S[i, i] = 0.0
            g = take_bench()
            if g is None:
                return Result(np.zeros((n, p)), BENCH_EXHAUSTED, 0, beta,
                              np.zeros((0, p)), S, replaced)
            u[i + 1] = substitute_out_of_kept(g, i + 1)
            replaced.append(i + 1)
        else:
            S[i, i] = sigma
            u[i + 1] = w / sigma
        orthogonalise_bench(u[i + 1])

    def ratios(rho):
        out = np.zeros(p)
        out[live] = rho[live] / beta[live]
        return out

    # S-hat = E_1 S (R6); rows are 1-based through an offset of one
    Shat = np.zeros((max_iter + p + 2, p))
    Shat[1:p + 1] = S
    X = np.zeros((n, p))
    hist = []
    Xs = []
    if not live.any() or ratios(np.linalg.norm(Shat[1:p + 1], axis=0)).max() < tol:
        return Result(X, CONVERGED, 0, beta, np.zeros((0, p)), S, replaced,
                      U=np.column_stack([u[i] for i in range(1, p + 1)]) if record else None)

    h = {}          # band entries h[(row, col)] of H-bar (1-based)
    rcol = {}       # R columns, rcol[j] = {row: value}
    rot = {}        # rot[j] = [(c, s) for t = 1..p] acting on rows (j, j+t)
    Qacc = {}       # R14: Qacc[b] = accumulated rotations of block b (2p x 2p)
    m = {}          # search directions m_i (window of 2p)
    zrows = []
    W = None
    status = MAX_ITER
    j = 0
    while j < max_iter:
        j += 1
        ell = (j - 1) % p + 1
        # -- operator on a block every p iterations (R2) --
        if ell == 1:
            W = A @ np.column_stack([u[i] for i in range(j, j + p)])
            W = np.asarray(W)
        w = W[:, ell - 1].copy()
        aw = np.linalg.norm(W[:, ell - 1])
        # -- band orthogonalisation (Algorithm 7.1 / eq. (2.6); R1, R3) --
        for i in range(max(1, j - p), j):           # known by symmetry
            h[(i, j)] = h[(j, i)]
            w -= h[(i, j)] * u[i]
        for i in range(j, j + p):                   # modified Gram-Schmidt
            h[(i, j)] = u[i] @ w
            w -= h[(i, j)] * u[i]
        project_kept(w, j + p)                      # R13
        eta = np.linalg.norm(w)
        # -- dependence test and replacement (Section 5.1; R10) --
        if eta <= gamma * aw:
            keep(j + p, w, eta, aw)
            h[(j + p, j)] = 0.0
            g = take_bench()
            if g is None:
                status = BENCH_EXHAUSTED
                j -= 1
                break
            u[j + p] = substitute_out_of_kept(g, j + p)
            replaced.append(j + p)
        else:
            h[(j + p, j)] = eta
            u[j + p] = w / eta                     # R4
        orthogonalise_bench(u[j + p])

        # -- QR of column j of H-bar by Givens rotations (Section 4; R7) --
        lo = max(1, j - 2 * p)
        r = {i: 0.0 for i in range(lo, j + p + 1)}
        for i in range(max(1, j - p), j + p + 1):
            r[i] = h[(i, j)]
        kb = (j - 1) // p + 1                       # block of column j
        own = range(lo, j)                          # columns whose rotations apply one by one
        if accumulate:                              # R14
            for i in range(max(1, (kb - 3) * p + 1), lo):
                r[i] = 0.0
            for b in (kb - 2, kb - 1):
                if b >= 1:
                    rows = range((b - 1) * p + 1, (b + 1) * p + 1)
                    seg = Qacc[b] @ np.array([r[i] for i in rows])
                    for i, v in zip(rows, seg):
                        r[i] = v
            own = range((kb - 1) * p + 1, j)
        for i in own:                               # rotations of columns lo..j-1
            for t, (c, s) in enumerate(rot[i], start=1):
                a, b = r[i], r[i + t]
                r[i], r[i + t] = c * a + s * b, -s * a + c * b
        if accumulate:
            for i in range(max(1, (kb - 3) * p + 1), lo):
                assert r[i] == 0.0, "rows above the band window must stay zero"
                del r[i]
        rot[j] = []
        for t in range(1, p + 1):                   # new rotations zero rows j+1..j+p
            c, s = _givens(r[j], r[j + t])
            rot[j].append((c, s))
            if s != 0.0:
                r[j] = np.hypot(r[j], r[j + t])
                r[j + t] = 0.0
                a, b = Shat[j].copy(), Shat[j + t].copy()
                Shat[j], Shat[j + t] = c * a + s * b, -s * a + c * b
        rcol[j] = {i: r[i] for i in range(lo, j + 1)}
        if accumulate and j % p == 0:               # block j/p complete: its rotations as one matrix
            b, base = j // p, j - p + 1
            Qb = np.eye(2 * p)
            for i in range(base, j + 1):
                for t, (c, s) in enumerate(rot[i], start=1):
                    a, bb = Qb[i - base].copy(), Qb[i - base + t].copy()
                    Qb[i - base], Qb[i - base + t] = c * a + s * bb, -s * a + c * bb
            Qacc[b] = Qb
            Qacc.pop(b - 2, None)
        if r[j] == 0.0:
            status = SINGULAR_R
            break
        # -- search direction (eq. (4.1); R8) and progressive X (eq. (4.2)) --
        mj = u[j].copy()
        for i in range(lo, j):
            mj -= r[i] * m[i]
        mj /= r[j]
        m[j] = mj
        z = Shat[j].copy()
        X += np.outer(mj, z)
        zrows.append(z)
        # -- recurrence residual (eq. (3.5)) and stopping test (R9) --
        rho = np.linalg.norm(Shat[j + 1:j + p + 1], axis=0)
        hist.append(ratios(rho))
        if record:
            Xs.append(X.copy())
        # -- drop what has left the band (Section 7 FIFO queues) --
        if not record:
            u.pop(j - p, None)
            rot.pop(j - 2 * p, None)
            rcol.pop(j - 2 * p, None)
        m.pop(j - 2 * p, None)
        kept[:] = [(mk, r) for mk, r in kept if mk + 2 * p > j + p]
        if hist[-1][live].max() < tol:
            status = CONVERGED
            break

    res = Result(X, status, j, beta, np.array(hist).reshape(-1, p), S, replaced)
    res.retained = list(kept_at)
    if record:
        J = j
        res.U = np.column_stack([u[i] for i in sorted(u)])
        H = np.zeros((J + p, J))
        for (a, b), v in h.items():
            if b <= J and a <= J + p:
                H[a - 1, b - 1] = v
        res.H = H
        R = np.zeros((J, J))
        for col, entries in rcol.items():
            if col <= J:
                for row, v in entries.items():
                    R[row - 1, col - 1] = v
        res.R = R
        res.Z = np.array(zrows).reshape(-1, p)
        res.Xs = Xs
    return res
