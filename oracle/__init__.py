"""Plain FP64 CPU oracle for band-Lanczos block MINRES (Soodhalter,
"A block MINRES algorithm based on the band Lanczos method").

TEST INFRASTRUCTURE.  Only the test suite, the package's smoke check and the
CPU-baseline leg of the benchmark may import, call or execute anything in
this directory.  The GPU library never routes through it and shares no code
with it; the two meet only in the seeded generators of ``workloads``.

Every function takes the paper's steps in the paper's order, one Lanczos
vector per iteration, in binary64, with numpy/scipy routines (a norm, a dot
product, a CSR times dense product, a Givens pair via hypot) as the only
library steps.  Readings of passages that are garbled or silent are listed in
``block_minres.py`` next to the code that depends on them.

Pins (tests that tie this code to something other than itself) live in
``tests/test_oracle_*.py``: a dense direct solve, the least-squares definition
over a brute-force band basis, classical MINRES at p = 1, the band Arnoldi
relation, the worked replacement example of Section 5.1, the C_{pxp} layout
of Section 7 and the dependence demonstration of Section 8.  The adjoint
gradients of ``adjoint.py`` (an extension, not in the paper) are pinned by
central finite differences of dense direct solves.  The preconditioned solve
of ``precond.py`` (IC(0) and split preconditioning; the paper's experiments
precondition but do not say how) is pinned by dense Cholesky factors, the
defining property of IC(0), a dense direct solve and scipy's preconditioned
MINRES at p = 1 (``tests/test_oracle_precond.py``).
"""
from .block_minres import (  # noqa: F401
    CONVERGED,
    MAX_ITER,
    BENCH_EXHAUSTED,
    SINGULAR_R,
    Result,
    solve,
)
from .rng import bench_vector, splitmix64  # noqa: F401
from .adjoint import Grad, loss_grad, pattern_grad  # noqa: F401
