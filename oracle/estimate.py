"""Condition-number estimate of the filtered block and the QR-variant choice
(paper estimate (1.1), estimate (1.2) in Sec. 1.3.1; Alg. 3; Cor. 3.5).

Oracle module (test infrastructure only).
"""
import math

from .chebyshev import rho_abs

# Variant codes shared (by value only) with the C interface's enum.
VARIANTS = {"chol1": 1, "chol2": 2, "shifted": 3, "householder": 4}

# Alg. 3 thresholds, stated for double precision.
EST_HI = 1e8
EST_LO = 20.0


def log_cond_estimate(theta_next, m_next, m_max, lam1, c, e, eta=1.0):
    """ln of the estimate kappa_est = eta |rho_{k+1}|^{m_{k+1}} |rho_1|^{m_l - m_{k+1}}
    (estimate (1.2)).  |rho_1| is taken at lam1 (the lowest eigenvalue estimate),
    |rho_{k+1}| at theta_next (the lowest unconverged Ritz value) and m_{k+1} is
    that column's degree; m_max is the largest degree of the pass (m_l).
    With no locked vectors and theta_next = lam1 this is estimate (1.1) with
    m -> m_l.  eta = 1 following the remark after Prop. 3.2.  Evaluated in log
    space so that large degrees do not overflow."""
    lr_next = math.log(rho_abs(theta_next, c, e))
    lr_1 = math.log(rho_abs(lam1, c, e))
    return math.log(eta) + m_next * lr_next + (m_max - m_next) * lr_1


def cond_estimate(theta_next, m_next, m_max, lam1, c, e, eta=1.0):
    """kappa_est itself (may be +inf when it overflows a double)."""
    v = log_cond_estimate(theta_next, m_next, m_max, lam1, c, e, eta)
    return math.exp(v) if v < 709.0 else float("inf")


def select_variant(est, hi=EST_HI, lo=EST_LO):
    """Alg. 3: est > 1e8 -> shifted CholeskyQR2; est < 20 -> CholeskyQR;
    otherwise CholeskyQR2."""
    if est > hi:
        return "shifted"
    if est < lo:
        return "chol1"
    return "chol2"
