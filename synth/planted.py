"""Planted-spectrum Hermitian matrices and Gaussian start blocks.

numpy versions (CPU; what the oracle consumes and what small GPU tests copy
to the device) and torch versions (built directly in device memory for the
large workloads, where a host QR of an N = 20000 complex matrix would take
minutes).  The two versions use different random streams: a given seed gives
the same spectrum family but not the same matrix.
"""
import numpy as np


def spectrum(family, N, rng, n_low=None):
    """Sorted planted eigenvalues of a family (see the package docstring)."""
    if family == "uniform":
        lam = rng.uniform(-1.0, 1.0, N)
    elif family == "dft":
        nl = max(1, int(round(0.05 * N))) if n_low is None else n_low
        lam = np.concatenate([rng.uniform(-2.0, -1.0, nl), rng.uniform(-1.0, 50.0, N - nl)])
    elif family == "stress":
        nl = 200 if n_low is None else n_low
        lam = np.concatenate([rng.uniform(-1.0, -0.999, nl), rng.uniform(-0.5, 1e3, N - nl)])
    else:
        raise ValueError(family)
    return np.sort(lam)


def _gauss(rng, shape, cplx):
    if cplx:
        re = rng.standard_normal(shape)
        im = rng.standard_normal(shape)
        return (re + 1j * im) / np.sqrt(2.0)
    return rng.standard_normal(shape)


def planted_numpy(N, family, seed, cplx=False, n_low=None):
    """(H, lambda): H = Q diag(lambda) Q^H, Hermitian to the last bit.
    Draw order: the Gaussian matrix first, then the spectrum."""
    rng = np.random.default_rng(seed)
    G = _gauss(rng, (N, N), cplx)
    Q, _ = np.linalg.qr(G)
    lam = spectrum(family, N, rng, n_low)
    H = (Q * lam[np.newaxis, :]) @ Q.conj().T
    H = 0.5 * (H + H.conj().T)
    return np.asfortranarray(H), lam


def start_block(N, L, seed, cplx=False):
    """Gaussian N x L start block: real N(0,1), complex (N(0,1)+iN(0,1))/sqrt(2)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(_gauss(rng, (N, L), cplx))


def lanczos_start(N, seed, cplx=False):
    rng = np.random.default_rng(seed)
    return _gauss(rng, (N,), cplx)


def lanczos_starts(N, nvec, seed, cplx=False):
    """N x nvec Gaussian start vectors, one per Lanczos run (Fortran order)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(_gauss(rng, (N, nvec), cplx))


def perturbation_numpy(N, seed, cplx=True):
    """E = (G + G^H) / (2 sqrt(N)) with Gaussian G (E|g|^2 = 1)."""
    rng = np.random.default_rng(seed)
    G = _gauss(rng, (N, N), cplx)
    E = (G + G.conj().T) / (2.0 * np.sqrt(N))
    return np.asfortranarray(E)


# ---------------------------------------------------------------- torch -----

def _torch():
    import torch
    return torch


def planted_torch(N, family, seed, cplx, device, n_low=None):
    """(H, lambda) built in device memory with torch: Gaussian G, Q from
    torch.linalg.qr (Householder QR), lambda drawn on the host with numpy from
    the same seed, H = (Q diag(lambda)) Q^H, Hermitised.  H is returned as a
    column-major (Fortran-order) tensor: its transpose is contiguous."""
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    dt = torch.complex128 if cplx else torch.float64
    G = torch.randn((N, N), dtype=dt, device=device, generator=gen)
    Q, _ = torch.linalg.qr(G)
    del G
    rng = np.random.default_rng(seed)
    lam = spectrum(family, N, rng, n_low)
    lam_t = torch.from_numpy(lam).to(device)
    QL = Q * lam_t.to(dt)[None, :]
    H = QL @ Q.conj().T.contiguous()
    del QL, Q
    H = 0.5 * (H + H.conj().T)
    # column-major storage: the memory of H.T (row-major) is H column-major
    Hc = H.T.contiguous().T
    del H
    return Hc, lam


def start_block_torch(N, L, seed, cplx, device):
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    dt = torch.complex128 if cplx else torch.float64
    V = torch.randn((L, N), dtype=dt, device=device, generator=gen)
    return V.T  # column-major N x L view


def perturbation_torch(N, seed, cplx, device):
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    dt = torch.complex128 if cplx else torch.float64
    G = torch.randn((N, N), dtype=dt, device=device, generator=gen)
    E = (G + G.conj().T) / (2.0 * np.sqrt(N))
    return E.T.contiguous().T
