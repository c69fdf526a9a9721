"""Helpers shared by the GPU tests: host <-> device copies of column-major
matrices and comparison utilities."""
import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def to_dev(A, dev):
    """numpy (N x L) -> column-major device tensor with the same values."""
    import torch
    A = np.asarray(A)
    if A.ndim == 1:
        return torch.from_numpy(A.copy()).to(dev)
    return torch.from_numpy(np.ascontiguousarray(A.T)).to(dev).T


def to_host(t):
    if t.dim() == 1:
        return t.cpu().numpy()
    return np.ascontiguousarray(t.T.cpu().numpy().T)


def phase_align(Q, Qref):
    """Rotate the columns of Q by unit phases to best match Qref."""
    d = np.sum(Q.conj() * Qref, axis=0)
    ph = np.where(np.abs(d) > 0, d / np.abs(d), 1.0)
    return Q * ph[np.newaxis, :]


def col_rel_err(A, B):
    """max over columns of max|A - B| / max|B| (element by element, scaled
    per column)."""
    num = np.max(np.abs(A - B), axis=0)
    den = np.maximum(np.max(np.abs(B), axis=0), 1e-300)
    return float(np.max(num / den))


def eig_rel_err(got, ref):
    """max_i |got_i - ref_i| / |ref_i|: the error of every eigenvalue relative
    to itself (the wanted eigenvalues of the test spectra are bounded away
    from zero)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.max(np.abs(got - ref) / np.abs(ref)))
