"""Chebyshev polynomials and the sigma-scaled recurrence (paper Sec. 2.1-2.2).

Oracle module (test infrastructure only).
"""
import math

import numpy as np


def cheb_closed(m, t):
    """C_m(t) from its closed forms (Sec. 2.1, the definition of C_m and its extension).

    |t| <= 1: cos(m arccos t).  t > 1: cosh(m arccosh t).  For t < -1 the
    parity C_m(-t) = (-1)^m C_m(t) of the polynomial is used.
    """
    t = float(t)
    if abs(t) <= 1.0:
        return math.cos(m * math.acos(t))
    v = math.cosh(m * math.acosh(abs(t)))
    return v if (t > 0 or m % 2 == 0) else -v


def rho_abs(x, c, e):
    """|rho| of the point x for the interval [c - e, c + e] (the interval map of Sec. 2.1, Def. of
    the convergence ratio in Sec. 2.2).

    With t = (x - c)/e: |rho| = max |t +- sqrt(t^2 - 1)| = |t| + sqrt(t^2 - 1)
    for |t| > 1; inside the interval the supremum of |rho| is 1.
    """
    t = (x - c) / e
    if abs(t) <= 1.0:
        return 1.0
    return abs(t) + math.sqrt(t * t - 1.0)


def sigma_sequence(mmax, c, e, gamma):
    """sigma_1..sigma_mmax of the scaled recurrence (Sec. 2.2):
    sigma_1 = e / (gamma - c), sigma_i = 1 / (2/sigma_1 - sigma_{i-1}).
    Returned as a list indexed from 1 (entry 0 unused)."""
    s = [0.0] * (mmax + 1)
    if mmax >= 1:
        s[1] = e / (gamma - c)
    for i in range(2, mmax + 1):
        s[i] = 1.0 / (2.0 / s[1] - s[i - 1])
    return s


def scaled_poly_recurrence(m, x, c, e, gamma):
    """p_m(x) = C_m((x-c)/e) / C_m((gamma-c)/e) evaluated with the scalar
    version of the sigma-scaled three-term recurrence of Alg. 4 (Sec. 2.2)."""
    s = sigma_sequence(max(m, 1), c, e, gamma)
    if m == 0:
        return 1.0
    p_prev = 1.0
    p_cur = (s[1] / e) * (x - c)
    for i in range(2, m + 1):
        p_new = (2.0 * s[i] / e) * (x - c) * p_cur - s[i - 1] * s[i] * p_prev
        p_prev, p_cur = p_cur, p_new
    return p_cur


def scaled_poly_closed(m, x, c, e, gamma):
    """p_m(x) = C_m(t_x)/C_m(t_gamma) from the closed forms (Thm. in Sec. 2.1)."""
    return cheb_closed(m, (x - c) / e) / cheb_closed(m, (gamma - c) / e)


def scaled_poly_closed_vec(m, xs, c, e, gamma):
    """Vectorised p_m over an array of points (used by tests as the spectral
    closed form of the filter, the spectral form of p(A)V in Sec. 2.3)."""
    return np.array([scaled_poly_closed(m, float(x), c, e, gamma) for x in np.ravel(xs)])
