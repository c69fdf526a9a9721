"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only draws random numbers and builds test matrices with a
planted spectrum, H = Q diag(lambda) Q^H with Q from the Householder QR of a
Gaussian matrix.  It holds none of the eigensolver's arithmetic (no filter,
no QR variant, no Rayleigh-Ritz), so both sides can take their inputs from it
without sharing any of the method.

Spectral families (stand-ins for the paper's DFT/BSE matrices of Table 2,
which are not available):
  uniform   lambda ~ U[-1, 1]                               (real, N = 1000)
  dft       5% of lambda ~ U[-2, -1] (a dense low cluster), the rest U[-1, 50]
  stress    n_low of lambda ~ U[-1, -0.999], the rest U[-0.5, 1e3]
"""
from .planted import (spectrum, planted_numpy, start_block, lanczos_start,
                      lanczos_starts, perturbation_numpy, planted_torch, start_block_torch,
                      perturbation_torch)

__all__ = ["spectrum", "planted_numpy", "start_block", "lanczos_start", "lanczos_starts",
           "perturbation_numpy", "planted_torch", "start_block_torch",
           "perturbation_torch"]
