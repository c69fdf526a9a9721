"""Spectral bounds by a few Lanczos steps (paper Alg. 1 and the discussion of
the bounds lambda_1, lambda_l, lambda_n in Sec. 1.2).

Oracle module (test infrastructure only).

PARITY UNPINNED beyond one property: the paper only requires that the upper
end be a true upper bound of the spectrum and lets the other two be rough.
Reading used here: k Lanczos steps with full reorthogonalisation from a given
unit start vector; T_k = tridiag(beta, alpha, beta); upper bound = largest Ritz
value of T_k + |beta_k|; lambda_1 estimate = smallest Ritz value; lambda_l
estimate = the Ritz value at which the Lanczos spectral-density count
sum_j N |s_1j|^2 (over Ritz values <= x) first reaches l, clamped into
(lambda_1, upper).
"""
import numpy as np
import scipy.linalg as sla


def lanczos_tridiag(H, v0, steps):
    """Return (alpha, beta) of T_k: alpha has k entries, beta has k entries
    (beta[k-1] is the norm of the final residual)."""
    N = H.shape[0]
    k = min(steps, N)
    V = np.zeros((N, k), dtype=H.dtype)
    alpha = np.zeros(k)
    beta = np.zeros(k)
    v = v0 / np.linalg.norm(v0)
    for j in range(k):
        V[:, j] = v
        w = H @ v
        alpha[j] = float(np.real(np.vdot(v, w)))
        Vj = V[:, : j + 1]
        for _ in range(2):  # classical Gram-Schmidt, twice
            w = w - Vj @ (Vj.conj().T @ w)
        beta[j] = float(np.linalg.norm(w))
        if beta[j] == 0.0:
            return alpha[: j + 1], beta[: j + 1]
        v = w / beta[j]
    return alpha, beta


def lanczos_bounds(H, n_search, v0, steps=40):
    """(lambda_1 estimate, lambda_l estimate, upper bound) for l = n_search."""
    N = H.shape[0]
    alpha, beta = lanczos_tridiag(H, v0, steps)
    k = alpha.size
    if k == 1:
        theta = alpha.copy()
        S = np.ones((1, 1))
    else:
        theta, S = sla.eigh_tridiagonal(alpha, beta[: k - 1])
    upper = float(theta[-1] + abs(beta[k - 1]))
    low = float(theta[0])
    weights = N * np.abs(S[0, :]) ** 2
    cum = np.cumsum(weights)
    idx = int(np.searchsorted(cum, n_search, side="left"))
    idx = min(idx, k - 1)
    mid = float(theta[idx])
    # clamp into (low, upper): keep the damped interval non-degenerate
    span = upper - low
    mid = min(max(mid, low + 1e-3 * span), upper - 1e-3 * span)
    return low, mid, upper
