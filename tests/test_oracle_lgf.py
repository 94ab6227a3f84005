"""Pins of the oracle's lattice Green's function against facts that do not depend
on its own quadrature: closed forms, the defining difference equation, an
independent reduced Fourier integral, a library Bessel routine and the paper's
printed asymptotic term."""
import json
import math
import os

import numpy as np
import pytest

from oracle import asymptotic, lgf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def table():
    return lgf.bessel_table(24)


def test_watson_origin_value(table):
    # G(0) = -W/6 with W the Watson integral in Glasser-Zucker closed form
    W = (math.sqrt(6) / (32 * math.pi ** 3) * math.gamma(1 / 24) * math.gamma(5 / 24)
         * math.gamma(7 / 24) * math.gamma(11 / 24))
    assert abs(table[0, 0, 0] - (-W / 6)) < 2e-15
    assert abs(table[0, 0, 0] - (-0.2527)) < 1e-4  # the value quoted for the method


def test_first_neighbour(table):
    assert abs(table[1, 0, 0] - (table[0, 0, 0] + 1.0 / 6.0)) < 2e-15


def test_discrete_laplacian_is_delta(table):
    # [L G](n) = delta(n) (Sec. 2.1, Eq. dpoisson with f = delta); the octant table is
    # mirrored to the full box so every interior point has its 6 neighbours.
    R = table.shape[0]
    full = np.empty((2 * R - 1,) * 3)
    idx = np.abs(np.arange(-(R - 1), R))
    full[:] = table[idx[:, None, None], idx[None, :, None], idx[None, None, :]]
    LG = lgf.laplacian(full)[2:-2, 2:-2, 2:-2]  # interior, aligned with full[1:-1,...]
    c = R - 2
    delta = np.zeros_like(LG)
    delta[c, c, c] = 1.0
    assert np.max(np.abs(LG - delta)) < 1e-14


def test_symmetry_48(table):
    # the table integrates a >= b >= c only; check mirror/permutation consistency of
    # values the Laplacian identity links across the permutation boundaries
    rng = np.random.default_rng(3)
    for _ in range(50):
        a, b, c = rng.integers(0, table.shape[0], 3)
        vals = {table[i, j, k] for (i, j, k) in
                [(a, b, c), (a, c, b), (b, a, c), (b, c, a), (c, a, b), (c, b, a)]}
        assert len(vals) == 1


def _reduced_2d(n1, n2, n3):
    """Eq. lgf1 with the xi_3 integral done in closed form:
    G(n) = -(1/4pi^2) int int cos(n1 x1) cos(n2 x2) lam^|n3| / sqrt(a^2 - 4),
    a = 6 - 2cos x1 - 2cos x2, lam = (a - sqrt(a^2-4))/2, in polar coordinates."""
    from scipy import integrate

    def f(r, th):
        x1, x2 = r * math.cos(th), r * math.sin(th)
        a = 6 - 2 * math.cos(x1) - 2 * math.cos(x2)
        s = math.sqrt(a * a - 4) if a > 2 else 0.0
        if s == 0.0:
            return 0.0
        lam = (a - s) / 2
        return r * math.cos(n1 * x1) * math.cos(n2 * x2) * lam ** abs(n3) / s

    tot = 0.0
    for lo, hi, rmax in [(0, math.pi / 4, lambda th: math.pi / math.cos(th)),
                         (math.pi / 4, math.pi / 2, lambda th: math.pi / math.sin(th))]:
        v, _ = integrate.dblquad(f, lo, hi, 0, rmax, epsabs=1e-14, epsrel=1e-13)
        tot += v
    return -4 * tot / (4 * math.pi ** 2)


@pytest.mark.filterwarnings("ignore")
@pytest.mark.parametrize("n", [(0, 0, 0), (1, 1, 0), (1, 1, 1), (2, 0, 0), (3, 1, 2), (5, 4, 0), (8, 0, 0)])
def test_independent_fourier_integral(table, n):
    ref = _reduced_2d(*n)
    assert abs(table[n] - ref) < 5e-13


def test_quadrature_converged():
    base = lgf.bessel_table(20)
    for kw in (dict(panel=0.125), dict(order=30), dict(xmax=1e6)):
        other = lgf.bessel_table(20, **kw)
        assert np.max(np.abs(other - base) / np.abs(base)) < 5e-15, kw


def test_scaled_bessel_against_library():
    from scipy.special import ive
    for x in (1e-6, 0.3, 2.0, 17.5, 400.0, 3.0e4):
        vals = lgf.scaled_bessel(x, 40)
        ref = ive(np.arange(41), x)
        mask = ref > 1e-200  # far below anything the integral can feel
        rel = np.abs(vals[mask] - ref[mask]) / ref[mask]
        assert np.max(rel) < 1e-13, x


def test_asymptotic_q2_matches_paper():
    g = json.load(open(os.path.join(GOLDEN, "asymptotic_q2.json")))
    from fractions import Fraction
    for j, mons in enumerate(g["terms"]):
        want = {(m[0], m[1], m[2]): Fraction(m[3], m[4]) for m in mons}
        got = asymptotic.term_polynomial(j)
        assert got == want


def test_asymptotic_error_rate():
    # G = A^q + O(|n|^(-2q-1)) (Sec. 2.1): doubling |n| on an axis divides the
    # error by about 2^(2q+1)
    T = lgf.bessel_table(48)
    for q in (1, 2, 3):
        e1 = abs(lgf.asymptotic_values([12.0, 0, 0], q) - T[12, 0, 0])
        e2 = abs(lgf.asymptotic_values([24.0, 0, 0], q) - T[24, 0, 0])
        rate = math.log2(e1 / e2)
        assert abs(rate - (2 * q + 1)) < 0.35, (q, rate)


def test_asymptotic_overlap_shell():
    # the far table switches to A^8 at max|n_i| >= 48; both agree there
    T = lgf.bessel_table(48)
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 48, (4000, 3))
    idx[:, 0] = rng.integers(32, 48, 4000)
    a = lgf.asymptotic_values(idx.astype(float), lgf.Q_TABLE)
    g = T[idx[:, 0], idx[:, 1], idx[:, 2]]
    assert np.max(np.abs(a - g) / np.abs(g)) < 5e-15
