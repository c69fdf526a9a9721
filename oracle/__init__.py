"""Plain, slow, FP64 CPU oracle for Chebyshev-filtered subspace iteration with
the condition-number-driven choice of the QR variant (Di Napoli & Wu,
"Estimating the condition number of Chebyshev filtered vectors with
application to the ChASE library", arXiv 2603.10514).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (``paper_2603_10514_amd`` and its HIP library) never imports,
links or calls it, and this package imports nothing from the product path:
the two share no kernels, helpers, constants or pre/post-processing.  Inputs
(matrices, start blocks) come from the separate ``synth`` package, which holds
none of the method's arithmetic.

Every function follows a passage of the paper, cited in its docstring by
section / algorithm / equation label.  numpy / scipy (LAPACK) primitives are
used only as single steps (a matrix product, a Cholesky factorisation, a
triangular solve, a dense Hermitian eigensolver, an SVD); nothing is blocked,
fused or reordered beyond what the paper's algorithms state.

Parity status per module (the pins live in ``tests/test_oracle_*.py``):
  chebyshev  pinned (closed forms of the Chebyshev polynomials, Sec. 2.1)
  filter     pinned (spectral closed form of p(A)V on planted spectra, Sec. 2.3)
  estimate   pinned (hand-evaluated cases; reduction of estimate (1.2) to
             estimate (1.1) at k = 0; empirical upper-bound property, Sec. 4.3;
             Lemma 3.1's closed form on filtered eigenvectors; Theorem 3.4
             by brute force)
  qr         pinned (orthogonality and backward error on planted singular
             values; Table 1 validity ranges; LAPACK Householder QR)
  rr         pinned (full diagonalisation of planted spectra)
  solver     pinned (planted eigenvalues, full diagonalisation, residual bound)
  degrees    pinned by a property (the predicted degree reaches tol on a
             planted diagonal case, one degree fewer does not); the formula
             and its margin are a reading (the paper gives none)
  lanczos    pinned by properties (Gauss-quadrature weights on a matrix
             with three distinct eigenvalues; top Ritz pair and its residual
             against a Rayleigh-Ritz on an independently built Krylov basis;
             the upper-bound property; the run-averaged density count
             against the eigenvalue count); the estimator itself is a
             reading (the paper gives no details of it)
"""

from .chebyshev import cheb_closed, rho_abs, sigma_sequence, scaled_poly_recurrence
from .filter import chebyshev_filter
from .estimate import cond_estimate, log_cond_estimate, select_variant, VARIANTS
from .qr import cholqr, shifted_cholqr_pass, householder_qr, dynamic_caqr, shift_value
from .rr import rayleigh_ritz, residual_norms
from .degrees import optimised_degrees
from .lanczos import lanczos_bounds
from .solver import chase_solve, ChaseResult

__all__ = [
    "cheb_closed", "rho_abs", "sigma_sequence", "scaled_poly_recurrence",
    "chebyshev_filter", "cond_estimate", "log_cond_estimate", "select_variant",
    "VARIANTS", "cholqr", "shifted_cholqr_pass", "householder_qr",
    "dynamic_caqr", "shift_value", "rayleigh_ritz", "residual_norms",
    "optimised_degrees", "lanczos_bounds", "chase_solve", "ChaseResult",
]
