"""Tolerances shared by the GPU parity tests (relative L-infinity, max|u - u_ref| / max|u_ref|).

* FP64 device vs the oracle's FLGF (the same linear operator, another rounding order):
  max(1e-12, Lambda^3 eps_64).  Rounding of node values is amplified by up to the
  Lebesgue constant cubed through the three tensor passes of Interp: the bound of Sec. 2.5
  (Eq. leb), whose own figure is Lambda^3 eps = 1.25e-12 at n_max = 10.  Lambda is that of
  p equispaced nodes for p <= 10, and the largest Lebesgue function of the 10-node windows
  for the n_I = 17 scheme.  The bar exceeds 1e-12 only there: 1.26e-12 at p = 10 and at
  p = 17 (observed at most 9.3e-13 and 4.6e-13).
* FP32 path vs the oracle's FLGF: 1e-6, the bar of the FP32 path (its FP64 node values and
  final add keep the rest of the budget for the FP32 transforms and products).
"""
import numpy as np

from oracle import flgf

FP32_BAR = 1e-6


def lebesgue(p, nmax=None):
    """Largest Lebesgue function of the interpolation stencils of p equispaced nodes on
    [0, p-1] (dense sampling); with nmax < p, of the nmax-node windows the oracle uses."""
    t = np.linspace(0, p - 1, 20001)
    if nmax is None:
        return float(np.max(np.sum(np.abs(flgf.lagrange(p, t)), axis=0)))
    return float(np.max(np.sum(np.abs(flgf.lagrange(p, t, nmax)), axis=0)))


def fp64_tol(p):
    nmax = 10 if p > 10 else None
    return max(1e-12, lebesgue(p, nmax) ** 3 * 2.22e-16)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
