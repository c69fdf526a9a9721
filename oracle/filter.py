"""Chebyshev filter with per-vector degrees (paper Alg. 4 and the per-vector
stopping rule at the end of Sec. 2.2).

Oracle module (test infrastructure only).
"""
import numpy as np

from .chebyshev import sigma_sequence


def chebyshev_filter(H, V, degrees, c, e, gamma):
    """Return (p_{m_1}(H) v_1, ..., p_{m_l}(H) v_l) for the columns of V.

    Alg. 4: V1 = (sigma_1/e)(H - cI)V;  Vi = (2 sigma_i/e)(H - cI)V(i-1)
    - sigma_{i-1} sigma_i V(i-2), with sigma from Sec. 2.2.  Column a stops
    being filtered once its degree m_a is reached (Sec. 2.2, last paragraph):
    its output is the iterate of step m_a.  The columns may come in any
    order; degrees must be >= 1.  ``gamma`` is the point where p(gamma) = 1
    (the estimate of the lowest eigenvalue).
    """
    m = np.asarray(degrees, dtype=np.int64)
    if V.shape[1] != m.size:
        raise ValueError("one degree per column")
    if m.size == 0:
        return V.copy()
    if np.any(m < 1):
        raise ValueError("degrees must be >= 1")
    mmax = int(m.max())
    s = sigma_sequence(mmax, c, e, gamma)
    out = np.empty_like(V)
    x_prev = V.copy()
    x_cur = (s[1] / e) * (H @ V - c * V)
    fin = m == 1
    out[:, fin] = x_cur[:, fin]
    for i in range(2, mmax + 1):
        act = m >= i
        x_new = np.zeros_like(V)
        x_new[:, act] = (2.0 * s[i] / e) * (H @ x_cur[:, act] - c * x_cur[:, act]) \
            - s[i - 1] * s[i] * x_prev[:, act]
        fin = m == i
        out[:, fin] = x_new[:, fin]
        x_prev, x_cur = x_cur, x_new
    return out


def matvecs(degrees):
    """MatVecs of one filter call: the sum of the per-column degrees
    (footnote on MatVecs in Sec. 4.4)."""
    return int(np.sum(np.asarray(degrees, dtype=np.int64)))
