"""ChASE driver loop (paper Alg. 1) with the dynamic QR choice (Alg. 3)
driven by the condition-number estimate (estimate (1.2)).

Oracle module (test infrastructure only).

Readings of points the paper leaves open (each is listed in the design notes):
  * filter interval: damp [alpha, beta] = [lambda_l estimate, upper bound],
    normalise at gamma = lambda_1 estimate (Sec. 2.1-2.2, Fig. 1; the centre
    and half-width printed in Alg. 4 give sigma_1 = -1 and are not used);
  * first iteration: no Ritz values yet, so theta_{k+1} = gamma;
  * step 0: the start block is orthonormalised with CholeskyQR2 before the
    first filter (Sec. 4.3 calls the QR of the random block "step 0");
  * QR always on [Y V] (Sec. 1.2), then the locked columns are restored
    exactly; Rayleigh-Ritz acts on the unlocked part only;
  * locking: the contiguous prefix (ascending Ritz order, index < nev) whose
    residuals are below tol;
  * bounds update: alpha <- the largest Ritz value of the search space,
    beta fixed; the filter is normalised (p(gamma) = 1) at the lowest
    unconverged Ritz value gamma = theta_{k+1}, while |rho_1| of the estimate
    is taken at the lowest Ritz value overall (locked or not).  Normalising at
    theta_{k+1} is what makes estimate (1.2) (|rho_{k+1}|^m without degree
    optimisation, Sec. 4.3) an upper bound of kappa_2([Y, filtered]): with the
    normalisation at the lowest locked value the filtered columns shrink by
    (|rho_{k+1}|/|rho_1|)^m against the unit-norm locked ones and kappa_2
    grows to about |rho_1|^m;
  * degrees: see ``degrees.py`` (a reading pinned by a property);
  * upper bound: Sec. 1.2 requires beta >= lambda_n.  Ritz values never
    exceed lambda_n, so a Ritz value above beta proves the bound wrong; beta
    is then moved past it (``upper_bound_check``).  With a valid bound this
    never happens.
"""
from dataclasses import dataclass, field

import numpy as np

from .degrees import optimised_degrees
from .estimate import cond_estimate, select_variant
from .filter import chebyshev_filter
from .lanczos import lanczos_bounds
from .qr import CholeskyFailure, cholqr, dynamic_caqr, householder_qr, shift_value
from .rr import rayleigh_ritz, residual_norms


@dataclass
class ChaseResult:
    evals: np.ndarray
    evecs: np.ndarray
    resid: np.ndarray
    iters: int
    matvecs: int
    converged: int
    bounds: tuple
    log: list = field(default_factory=list)


def step0(V0):
    """Orthonormalise the start block with CholeskyQR2 (Householder if the
    Cholesky fails)."""
    try:
        return cholqr(V0, 2)
    except CholeskyFailure as exc:
        return householder_qr(exc.x)


def upper_bound_check(theta, r, beta):
    """beta, or, when the largest Ritz value theta[-1] exceeds it (then beta
    is not an upper bound of the spectrum: a Ritz value is at most lambda_n),
    theta[-1] + 2 r[-1] + 1e-3 (theta[-1] - theta[0]): an eigenvalue lies
    within r[-1] of theta[-1], taken twice over, plus a margin that keeps the
    damped interval from collapsing when r[-1] = 0."""
    top = float(theta[-1])
    if top > beta:
        return top + 2.0 * float(r[-1]) + 1e-3 * (top - float(theta[0]))
    return beta


def chase_solve(H, nev, nex, deg=20, tol=1e-10, *, V0, bounds=None,
                lanczos_v0=None, lanczos_steps=40, deg_opt=True, min_deg=1,
                max_deg=36, max_iter=25, qr_policy="auto", exact_cond=False,
                est_hi=1e8, est_lo=20.0):
    """Lowest nev eigenpairs of the Hermitian H by Alg. 1.

    V0 (N x (nev+nex)) is the start block (random or a warm start); bounds is
    (lambda_1, lambda_l, upper) or None for the Lanczos estimate from
    lanczos_v0 (one start vector, or an N x nvec block: one run per
    column).  qr_policy "auto" is Alg. 3; "chol1", "chol2", "shifted" or
    "householder" force one variant every iteration."""
    H = np.asarray(H)
    N = H.shape[0]
    L = nev + nex
    if not (1 <= nev and 1 <= nex and L <= N):
        # Alg. 1 sets a search space l > nev
        raise ValueError("need 1 <= nev, 1 <= nex and nev + nex <= N")
    if bounds is None:
        if lanczos_v0 is None:
            raise ValueError("bounds or lanczos_v0 required")
        bounds = lanczos_bounds(H, L, lanczos_v0, lanczos_steps)
    gamma, alpha, beta = (float(b) for b in bounds)

    lam1 = gamma
    Vbuf = step0(np.array(V0, dtype=H.dtype, copy=True))
    k = 0
    m = np.full(L, deg, dtype=np.int64)
    theta_act = None
    lam = []
    res_locked = []
    matvecs = 0
    log = []
    it = 0
    for it in range(1, max_iter + 1):
        c = 0.5 * (alpha + beta)
        e = 0.5 * (beta - alpha)
        # filter the active columns in ascending-degree order (stable)
        order = np.argsort(m, kind="stable")
        Xin = Vbuf[:, k:][:, order]
        filt = chebyshev_filter(H, Xin, m[order], c, e, gamma)
        matvecs += int(m.sum())
        # estimate (estimate (1.2)); theta_{k+1} is the lowest unconverged Ritz
        # value and m[0] its degree (columns are in Ritz order before sorting)
        th_next = gamma if theta_act is None else float(theta_act[0])
        est = cond_estimate(th_next, int(m[0]), int(m.max()), lam1, c, e)
        variant = select_variant(est, est_hi, est_lo) if qr_policy == "auto" else qr_policy
        X = np.concatenate([Vbuf[:, :k], filt], axis=1)
        kappa = None
        if exact_cond:
            sv = np.linalg.svd(X, compute_uv=False)
            kappa = float(sv[0] / sv[-1])
        Q, failed = dynamic_caqr(X, variant)
        Q[:, :k] = Vbuf[:, :k]
        theta, Vr, HV = rayleigh_ritz(H, Q[:, k:])
        r = residual_norms(HV, Vr, theta)
        Vbuf[:, k:] = Vr
        j = k
        while j < nev and r[j - k] < tol:
            j += 1
        newly = j - k
        lam.extend(theta[:newly].tolist())
        res_locked.extend(r[:newly].tolist())
        log.append(dict(iter=it, locked=k, cond_est=est, cond_exact=kappa,
                        variant=variant, chol_failed=bool(failed),
                        qr_shift=shift_value(X) if variant == "shifted" else None,
                        matvecs=int(m.sum()), deg_max=int(m.max()),
                        deg_min=int(m.min()), newly_locked=newly,
                        c=c, e=e, gamma=gamma, lam1=lam1))
        k = j
        theta_act = theta[newly:]
        r_act = r[newly:]
        if k >= nev:
            break
        lam1 = lam[0] if k > 0 else float(theta[0])
        gamma = float(theta_act[0])
        alpha = float(theta[-1])
        beta = upper_bound_check(theta, r, beta)
        c = 0.5 * (alpha + beta)
        e = 0.5 * (beta - alpha)
        if deg_opt:
            m = optimised_degrees(theta_act, r_act, tol, c, e, min_deg, max_deg)
        else:
            m = np.full(L - k, deg, dtype=np.int64)
    evals = np.array(lam[:nev])
    # not converged: report the current Ritz values for the rest
    if k < nev:
        evals = np.concatenate([evals, theta_act[: nev - k]])
        res = np.concatenate([np.array(res_locked), r_act[: nev - k]])
    else:
        res = np.array(res_locked[:nev])
    return ChaseResult(evals=evals, evecs=Vbuf, resid=res, iters=it,
                       matvecs=matvecs, converged=k, bounds=(bounds), log=log)
