"""Oracle: far-field asymptotic expansion A^q of the 3D 7-point lattice Green's function.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only tests/, the smoke check and the CPU-baseline leg of the benchmark use it.

Paper, Sec. 2.1 (Eq. lgf1, Eq. lgf2): G(n) is the inverse Fourier integral of
1/sigma(xi) with sigma(xi) = 2 sum_i cos(xi_i) - 6, and A^q is the unique rational
function with G(n) = A^q(n) + O(|n|^(-2q-1)).  The paper prints only q = 2 and
defers higher orders to the literature; this module derives every order from
Eq. lgf1 with exact rational arithmetic:

  * sigma(xi) = -(|xi|^2 - delta(xi)),
    delta(xi) = sum_i sum_{k>=2} 2 (-1)^k xi_i^(2k) / (2k)!      (Taylor of 2 - 2 cos)
  * 1/sigma = -sum_{m>=0} delta^m / |xi|^(2m+2); the part homogeneous of degree
    2j - 2 in xi collects [delta^m]_{2m+2j} / |xi|^(2m+2) for m = 0..j.
  * A monomial xi^alpha (all exponents even) becomes the operator (i d)^alpha
    = (-1)^(|alpha|/2) d^alpha acting on F_k, the inverse transform of |xi|^(-2k):
    F_1 = 1/(4 pi r), Laplacian(F_k) = -F_(k-1), F_k = c_k r^(2k-3).
  * Order j therefore contributes T_j(x) = P_j(x) / (pi r^(6j+1)) with P_j a
    homogeneous polynomial of degree 4j, and A^q = sum_{j<q} T_j.

The q = 2 case must reproduce the paper's printed Eq. lgf2 exactly (pinned in the
tests against a fixture transcribed from the paper).
"""
from fractions import Fraction
from functools import lru_cache
import math

import numpy as np

__all__ = ["derive_terms", "asymptotic_G", "term_polynomial"]


def _pmul(a, b, maxdeg=None):
    out = {}
    for ea, ca in a.items():
        for eb, cb in b.items():
            e = (ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2])
            if maxdeg is not None and sum(e) > maxdeg:
                continue
            out[e] = out.get(e, 0) + ca * cb
    return {e: c for e, c in out.items() if c != 0}


def _padd(a, b, scale=1):
    out = dict(a)
    for e, c in b.items():
        out[e] = out.get(e, 0) + scale * c
    return {e: c for e, c in out.items() if c != 0}


_R2 = {(2, 0, 0): Fraction(1), (0, 2, 0): Fraction(1), (0, 0, 2): Fraction(1)}


def _deriv(Q, e, axis):
    """d/dx_axis of Q(x) r^e, returned as (Q', e - 2): (dQ r^2 + e x_axis Q) r^(e-2)."""
    dQ = {}
    for m, c in Q.items():
        if m[axis] > 0:
            mm = list(m)
            mm[axis] -= 1
            dQ[tuple(mm)] = dQ.get(tuple(mm), 0) + c * m[axis]
    out = _pmul(dQ, _R2)
    xQ = {}
    for m, c in Q.items():
        mm = list(m)
        mm[axis] += 1
        xQ[tuple(mm)] = c * e
    return _padd(out, xQ), e - 2


@lru_cache(maxsize=None)
def _deriv_power(alpha, e):
    """d^alpha r^e as (polynomial dict, exponent); alpha a tuple of 3 orders."""
    if alpha == (0, 0, 0):
        return ({(0, 0, 0): Fraction(1)}, e)
    # peel one derivative off the last non-zero axis
    axis = max(i for i in range(3) if alpha[i] > 0)
    prev = list(alpha)
    prev[axis] -= 1
    Q, ee = _deriv_power(tuple(prev), e)
    return _deriv(dict(Q), ee, axis)


def _delta_poly(maxdeg):
    """delta(xi) truncated at total degree maxdeg."""
    d = {}
    k = 2
    while 2 * k <= maxdeg:
        coef = Fraction(2 * (-1) ** k, math.factorial(2 * k))
        for axis in range(3):
            m = [0, 0, 0]
            m[axis] = 2 * k
            d[tuple(m)] = d.get(tuple(m), 0) + coef
        k += 1
    return d


def _gamma(k):
    """c_k * pi for F_k = c_k r^(2k-3): gamma_1 = 1/4, gamma_k = -gamma_(k-1)/((2k-3)(2k-2))."""
    g = Fraction(1, 4)
    for kk in range(2, k + 1):
        g = -g / ((2 * kk - 3) * (2 * kk - 2))
    return g


@lru_cache(maxsize=None)
def term_polynomial(j):
    """P_j (exact rationals): order-j term T_j(x) = P_j(x) / (pi r^(6j+1))."""
    maxdeg = 4 * j
    delta = _delta_poly(2 * j + 4)
    total = {}
    dm = {(0, 0, 0): Fraction(1)}  # delta^m, truncated
    for m in range(0, j + 1):
        if m > 0:
            dm = _pmul(dm, delta, maxdeg=2 * j + 2 * m + 4 * j)
        want = 2 * m + 2 * j
        part = {}
        for alpha, c in dm.items():
            if sum(alpha) != want:
                continue
            sign = -1 if (sum(alpha) // 2) % 2 else 1
            Q, e = _deriv_power(alpha, 2 * m - 1)
            assert e == -2 * m - 4 * j - 1
            part = _padd(part, Q, scale=sign * c)
        # F_(m+1) = gamma_(m+1)/pi r^(2m-1); bring r^(-2m-4j-1) to r^(-6j-1)
        for _ in range(j - m):
            part = _pmul(part, _R2)
        total = _padd(total, part, scale=-_gamma(m + 1))
    for mono in total:
        assert sum(mono) == maxdeg
    return total


def derive_terms(q):
    """List of P_0..P_(q-1)."""
    return [term_polynomial(j) for j in range(q)]


def asymptotic_G(x, q):
    """A^q evaluated at real points x (array [..., 3]), float64.

    Each term is evaluated on the unit direction xhat = x/r, so that
    T_j = P_j(xhat) / (pi r^(2j+1)).
    """
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt(np.sum(x * x, axis=-1))
    xh = x / r[..., None]
    out = np.zeros_like(r)
    for j in range(q):
        P = term_polynomial(j)
        val = np.zeros_like(r)
        for (a, b, c), coef in P.items():
            val += float(coef) * xh[..., 0] ** a * xh[..., 1] ** b * xh[..., 2] ** c
        out += val / (math.pi * r ** (2 * j + 1))
    return out
