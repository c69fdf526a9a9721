"""CholeskyQR (Alg. 2), shifted CholeskyQR2, Householder QR and the dynamic
selection of Alg. 3 (paper Sec. 1.3, Table 1).

Oracle module (test infrastructure only).
"""
import numpy as np
import scipy.linalg as sla

UNIT_ROUNDOFF = 2.0 ** -53


class CholeskyFailure(Exception):
    """The Cholesky factorisation of the Gram matrix did not succeed
    (info != 0 in Alg. 2)."""


def _gram(X):
    G = X.conj().T @ X
    return 0.5 * (G + G.conj().T)


def _chol_upper(G):
    """R upper triangular with G = R^H R; raises CholeskyFailure when G is not
    numerically positive definite."""
    if not np.all(np.isfinite(G)):
        raise CholeskyFailure("non-finite Gram matrix")
    try:
        R = sla.cholesky(G, lower=False, check_finite=False)
    except np.linalg.LinAlgError as exc:
        raise CholeskyFailure(str(exc)) from exc
    if not np.all(np.isfinite(R)):
        raise CholeskyFailure("non-finite factor")
    return R


def _right_solve(X, R):
    """X R^{-1}: solve Q R = X, i.e. R^H Q^H = X^H (triangular solve)."""
    Y = sla.solve_triangular(R, X.conj().T, trans="C", lower=False, check_finite=False)
    return Y.conj().T


def cholqr(X, chol_deg):
    """Alg. 2: chol_deg passes of R <- X^H X, R <- Cholesky(R), X <- X R^{-1}.
    Raises CholeskyFailure on the pass that fails (its input is returned in
    the exception's ``x`` attribute, so the caller can continue from it)."""
    for _ in range(chol_deg):
        try:
            R = _chol_upper(_gram(X))
        except CholeskyFailure as exc:
            exc.x = X
            raise
        X = _right_solve(X, R)
    return X


def shift_value(X):
    """Shift of shifted CholeskyQR (Alg. 3): s = 11 (N l + l (l+1)) u ||X||_F^2
    with u the unit round-off of double precision.  The paper prints the norm
    unsquared; the squared Frobenius norm matches the scale of X^H X and the
    shifted-CholeskyQR analysis the paper builds on (reading documented in the
    design notes)."""
    n_rows, n_cols = X.shape
    fro2 = float(np.sum(np.abs(X) ** 2))
    return 11.0 * (n_rows * n_cols + n_cols * (n_cols + 1)) * UNIT_ROUNDOFF * fro2


def shifted_cholqr_pass(X):
    """One shifted pass of Alg. 3: R <- Cholesky(X^H X + s I); X <- X R^{-1}."""
    s = shift_value(X)
    G = _gram(X)
    G = G + s * np.eye(G.shape[0])
    try:
        R = _chol_upper(G)
    except CholeskyFailure as exc:
        exc.x = X
        raise
    return _right_solve(X, R)


def householder_qr(X):
    """Householder QR (LAPACK geqrf/orgqr through numpy), reduced Q."""
    Q, _ = np.linalg.qr(X, mode="reduced")
    return Q


def dynamic_caqr(X, variant):
    """Alg. 3 for a given variant ("chol1", "chol2", "shifted" or
    "householder").  Returns (Q, chol_failed).  When any Cholesky fails the
    Householder QR is applied to the block as it stood before the failing
    pass (the paper's fallback, extended to the non-shifted branches)."""
    if variant == "householder":
        return householder_qr(X), False
    try:
        if variant == "shifted":
            Xs = shifted_cholqr_pass(X)
            return cholqr(Xs, 2), False
        if variant == "chol1":
            return cholqr(X, 1), False
        if variant == "chol2":
            return cholqr(X, 2), False
    except CholeskyFailure as exc:
        return householder_qr(exc.x), True
    raise ValueError("unknown variant %r" % (variant,))
