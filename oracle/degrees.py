"""Per-vector polynomial degrees (paper Sec. 2.2 last paragraph; Sec. 4.3).

Oracle module (test infrastructure only).

Sec. 2.2 filters each vector with its own degree, chosen as the smallest
one that brings that vector's residual to the tolerance, and Sec. 4.3 uses
an initial degree of 20 and a cap of 36; no formula is given.  Pinned by a property, not by the
paper (tests: the predicted degree brings a vector whose unwanted components
lie in the damped interval to tol, and one degree fewer than the bare
prediction does not); the margin of 2 is a reading.  The reading used here:
a column whose residual is r and whose Ritz value has convergence ratio
1/|rho| needs about ln(r/tol)/ln|rho| more filter steps, so
m_a = ceil(ln(r_a/tol) / ln|rho(theta_a)|) + margin, clamped to
[min_deg, max_deg], with a margin of 2 degrees (the convergence-ratio model
predicts only the decay rate; aimed exactly at tol the residuals settle at
about tol and then need many one-degree passes to cross it);
|rho| = 1 (a Ritz value inside the damped interval) gives max_deg; a residual
already below tol gives min_deg.  Only the clamp range and the ascending order
used by the filter are fixed by the paper.
"""
import math

import numpy as np

from .chebyshev import rho_abs


def optimised_degrees(theta, resid, tol, c, e, min_deg, max_deg, margin=2):
    out = np.empty(len(theta), dtype=np.int64)
    for a, (th, r) in enumerate(zip(theta, resid)):
        if r <= tol:
            out[a] = min_deg
            continue
        rho = rho_abs(float(th), c, e)
        if rho <= 1.0:
            out[a] = max_deg
            continue
        d = math.ceil(math.log(r / tol) / math.log(rho)) + margin
        out[a] = min(max(d, min_deg), max_deg)
    return out
