"""Spectral bounds by a few Lanczos runs (paper Alg. 1 and the discussion of
the bounds lambda_1, lambda_l, lambda_n in Sec. 1.2).

Oracle module (test infrastructure only).

The paper fixes one property only: the estimate of lambda_n must bound the
spectrum from above, while the estimates of lambda_1 and lambda_l may be
rough.  Reading used here (pinned by properties in the tests: Gauss weights,
the top Ritz pair's residual, the upper-bound property, and the density
count against the eigenvalue count):

* nvec independent runs, one per start vector, each k steps with full
  reorthogonalisation; run r gives T_k = tridiag(beta, alpha, beta) with
  eigenpairs (theta_rj, s_rj);
* upper bound = max over runs of theta_max + 2 |beta_k| |e_k^T s_max|, the
  largest Ritz value plus twice the residual norm of its Ritz pair.  By
  interlacing theta_max <= lambda_n, and an eigenvalue lies within one
  residual of theta_max; it is lambda_n itself once the top of the spectrum
  has converged, which 40 steps reach on all but the smallest matrices.  The
  factor 2 and the maximum over independent runs cover the rest.  The usual
  safe choice theta_max + |beta_k| overshoots lambda_n by about a quarter of
  the spectrum's width on spread spectra, which widens the filter interval;
* lambda_1 estimate = smallest Ritz value over the runs;
* lambda_l estimate = the Ritz value at which the spectral-density count
  (1/nvec) sum_r sum_j N |e_1^T s_rj|^2 over Ritz values <= x first reaches
  l, clamped into (lambda_1, upper).
"""
import numpy as np
import scipy.linalg as sla


def lanczos_tridiag(H, v0, steps):
    """Return (alpha, beta) of T_k: alpha has k entries, beta has k entries
    (beta[k-1] is the norm of the final residual).  The run stops early when
    the Krylov space becomes invariant (a zero beta)."""
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


def lanczos_dos(alpha, beta, N):
    """Ritz values theta (ascending), spectral-density weights N |e_1^T s_j|^2
    and the residual norm |beta_k| |e_k^T s_max| of the top Ritz pair, for one
    run's T_k."""
    k = alpha.size
    if k == 1:
        theta = alpha.copy()
        S = np.ones((1, 1))
    else:
        theta, S = sla.eigh_tridiagonal(alpha, beta[: k - 1])
    weights = N * np.abs(S[0, :]) ** 2
    top_resid = abs(beta[k - 1]) * abs(S[k - 1, k - 1])
    return theta, weights, float(top_resid)


def start_columns(v0):
    """The start vectors as the columns of an N x nvec array."""
    v0 = np.asarray(v0)
    return v0[:, None] if v0.ndim == 1 else v0


UPPER_RESID_FACTOR = 2.0


def bounds_from_runs(runs, N, n_search):
    """(lambda_1 estimate, lambda_l estimate, upper bound) from the
    (alpha, beta) of each run."""
    thetas, weights = [], []
    low, upper = np.inf, -np.inf
    for alpha, beta in runs:
        theta, w, r = lanczos_dos(alpha, beta, N)
        thetas.append(theta)
        weights.append(w)
        low = min(low, float(theta[0]))
        upper = max(upper, float(theta[-1]) + UPPER_RESID_FACTOR * r)
    theta = np.concatenate(thetas)
    w = np.concatenate(weights) / len(runs)
    order = np.argsort(theta, kind="stable")
    theta, w = theta[order], w[order]
    cum = np.cumsum(w)
    idx = min(int(np.searchsorted(cum, n_search, side="left")), theta.size - 1)
    mid = float(theta[idx])
    # clamp into (low, upper): keep the damped interval non-degenerate
    span = upper - low
    mid = min(max(mid, low + 1e-3 * span), upper - 1e-3 * span)
    return low, mid, upper


def lanczos_bounds(H, n_search, v0, steps=40):
    """(lambda_1 estimate, lambda_l estimate, upper bound) for l = n_search;
    v0 is one start vector or an N x nvec block (one run per column)."""
    V0 = start_columns(v0)
    runs = [lanczos_tridiag(H, V0[:, r], steps) for r in range(V0.shape[1])]
    return bounds_from_runs(runs, H.shape[0], n_search)
