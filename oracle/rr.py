"""Rayleigh-Ritz projection and residual norms (paper Alg. 1, the residual of Sec. 2.3.1).

Oracle module (test infrastructure only).
"""
import numpy as np
import scipy.linalg as sla


def rayleigh_ritz(H, Q):
    """Alg. 1 Rayleigh-Ritz on an orthonormal block Q: A~ = Q^H H Q, solve
    A~ W = W Lambda~ (ascending), V = Q W.  Also returns H V = (H Q) W, which
    the residuals need.  A~ is symmetrised explicitly."""
    W = H @ Q
    A = Q.conj().T @ W
    A = 0.5 * (A + A.conj().T)
    theta, Z = sla.eigh(A)
    return theta, Q @ Z, W @ Z


def residual_norms(HV, V, theta):
    """the residual of Sec. 2.3.1: ||A v_a - theta_a v_a||_2 / ||v_a||_2 for every column a."""
    R = HV - V * theta[np.newaxis, :]
    return np.linalg.norm(R, axis=0) / np.linalg.norm(V, axis=0)
