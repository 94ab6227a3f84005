"""Pins of the oracle's second lattice kernel: the LGF G_kappa of the screened operator
L - kappa (kappa > 0), the Bessel integral of Appendix A with the factor e^{-kappa t}
(Sec. 5: the method applies to any non-oscillatory lattice kernel).  Each check is against
something other than the oracle's own formula:

  * the discrete equation  sum_{+-e_i} G(n +- e_i) - (6 + kappa) G(n) = delta(n);
  * the sum rule  sum_n G_kappa(n) = -1/kappa  (the symbol at xi = 0);
  * an independent reduced 2D Fourier integral of Eq. lgf1 with the denominator shifted by
    -kappa (the xi_3 integral done in closed form), evaluated by scipy's dblquad;
  * the weak-screening limit G_kappa - G_0 -> sqrt(kappa) / (4 pi) near the origin;
  * the direct sum inverts L - kappa; a manufactured solution passes through it exactly;
  * the FLGF with the screened kernel: exact with no far field and with lattice nodes on
    a single level, convergent in p at full depth, and reproducing a manufactured
    solution.
"""
import numpy as np
import pytest

from oracle import flgf, lgf as olgf
from paper_1402_6081_amd import workloads as W


def _full(T):
    R = T.shape[0]
    a = np.abs(np.arange(-(R - 1), R))
    return T[a[:, None, None], a[None, :, None], a[None, None, :]]


@pytest.mark.parametrize("kappa", [0.25, 1.0, 4.0])
def test_discrete_equation(kappa):
    G = _full(olgf.screened_table(16, kappa))  # index [z, y, x] symmetric, centre 15
    res = (G[2:, 1:-1, 1:-1] + G[:-2, 1:-1, 1:-1] + G[1:-1, 2:, 1:-1] + G[1:-1, :-2, 1:-1]
           + G[1:-1, 1:-1, 2:] + G[1:-1, 1:-1, :-2] - (6.0 + kappa) * G[1:-1, 1:-1, 1:-1])
    c = res.shape[0] // 2
    res[c, c, c] -= 1.0
    assert np.max(np.abs(res)) < 1e-13


@pytest.mark.parametrize("kappa,R", [(1.0, 45), (4.0, 25), (0.25, 90)])
def test_sum_rule(kappa, R):
    # R is chosen so that the terms left out are below 1e-17 (decay e^{-mu |n|}, cosh mu =
    # 1 + kappa/2 along the axes)
    s = float(np.sum(_full(olgf.screened_table(R, kappa))))
    assert abs(s + 1.0 / kappa) * kappa < 1e-13


def _reduced_2d(n, kappa):
    from scipy.integrate import dblquad
    n1, n2, n3 = (abs(int(v)) for v in n)

    def f(x2, x1):
        a = 6.0 + kappa - 2.0 * np.cos(x1) - 2.0 * np.cos(x2)
        r = np.sqrt(a * a - 4.0)
        lam = 0.5 * (a - r)
        return np.cos(n1 * x1) * np.cos(n2 * x2) * lam ** n3 / r

    v, _ = dblquad(f, 0.0, np.pi, 0.0, np.pi, epsabs=1e-14, epsrel=1e-13)
    return -v / np.pi ** 2


@pytest.mark.parametrize("kappa", [0.5, 3.0])
def test_reduced_2d_fourier_integral(kappa):
    T = olgf.screened_table(8, kappa)
    for n in [(0, 0, 0), (1, 0, 0), (1, 1, 0), (2, 1, 1), (3, 0, 2), (5, 4, 1)]:
        ref = _reduced_2d(n, kappa)
        got = T[n[0], n[1], n[2]]
        assert abs(got - ref) <= 1e-11 * abs(ref), (n, got, ref)


def test_weak_screening_limit():
    kappa = olgf.KAPPA_MIN
    Tk = olgf.lgf_table(4, kappa)
    T0 = olgf.bessel_table(4)
    shift = np.sqrt(kappa) / (4.0 * np.pi)
    for n in [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 1, 0)]:
        d = Tk[n] - T0[n]
        assert abs(d / shift - 1.0) < 0.1, (n, d, shift)


def test_spacing_table_matches_unit_table():
    kappa, h = 2.0, 3
    A = olgf.lattice_table(6, kappa, h)
    B = olgf.lgf_table(16, kappa)
    idx = np.arange(6) * h
    assert np.max(np.abs(A - B[np.ix_(idx, idx, idx)]) / np.abs(B[np.ix_(idx, idx, idx)])) < 1e-14


def test_direct_sum_inverts_the_operator():
    kappa = 1.5
    rng = np.random.default_rng(5)
    Z = np.zeros((6, 6, 6))
    Z[1:5, 1:5, 1:5] = rng.standard_normal((4, 4, 4))
    src = np.argwhere(Z != 0)[:, ::-1]  # (x, y, z)
    fv = Z[src[:, 2], src[:, 1], src[:, 0]]
    g = np.stack(np.meshgrid(np.arange(-2, 8), np.arange(-2, 8), np.arange(-2, 8), indexing="ij"), -1)
    tgt = g.reshape(-1, 3)[:, ::-1]
    u = olgf.direct_sum(src, fv, tgt, kappa).reshape(10, 10, 10)  # [z, y, x]
    Lu = (u[2:, 1:-1, 1:-1] + u[:-2, 1:-1, 1:-1] + u[1:-1, 2:, 1:-1] + u[1:-1, :-2, 1:-1]
          + u[1:-1, 1:-1, 2:] + u[1:-1, 1:-1, :-2] - (6.0 + kappa) * u[1:-1, 1:-1, 1:-1])
    ref = np.zeros((8, 8, 8))
    ref[1:7, 1:7, 1:7] = Z  # Lu index i is the lattice coordinate i - 1
    assert np.max(np.abs(Lu - ref)) < 1e-12 * np.max(np.abs(Z))


def _manufactured(blocks, n, kappa, rng):
    """u_rand ~ U[-1, 1], zero on the boundary points, and f = (L - kappa) u_rand, which
    vanishes off the active grid, so G_kappa * f = u_rand exactly."""
    u = W.random_manufactured(blocks, n, rng)
    b = np.asarray(blocks, dtype=np.int64)
    ext = b.max(axis=0) + 1
    D = np.zeros((ext[2] * n, ext[1] * n, ext[0] * n))
    for i, (bx, by, bz) in enumerate(b.tolist()):
        D[bz * n:(bz + 1) * n, by * n:(by + 1) * n, bx * n:(bx + 1) * n] = u[i]
    LD = olgf.laplacian(D, kappa)[1:-1, 1:-1, 1:-1]
    f = np.empty_like(u)
    for i, (bx, by, bz) in enumerate(b.tolist()):
        f[i] = LD[bz * n:(bz + 1) * n, by * n:(by + 1) * n, bx * n:(bx + 1) * n]
    return u, f


def test_direct_sum_manufactured_solution():
    kappa, n = 0.8, 4
    rng = np.random.default_rng(11)
    blocks = W.eden_layout(6, rng)
    u, f = _manufactured(blocks, n, kappa, rng)
    P = W.points_of(blocks, n).reshape(-1, 3)
    got = olgf.direct_sum(P, f.reshape(-1), P, kappa)
    assert np.max(np.abs(got - u.reshape(-1))) < 1e-12


def _exact(blocks, f, n, kappa):
    P = W.points_of(blocks, n).reshape(-1, 3)
    return olgf.direct_sum(P, f.reshape(-1), P, kappa).reshape(f.shape)


def test_flgf_no_far_field_is_exact():
    kappa = 1.0
    rng = np.random.default_rng(12)
    blocks = W.cube_layout(2)
    f = rng.standard_normal((8, 8, 8, 8))
    got = flgf.solve(blocks, f, 8, 9, 0, kappa=kappa)
    ref = _exact(blocks, f, 8, kappa)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_flgf_lattice_nodes_single_level_is_exact():
    # p = n + 1 with one level: Reg puts the block on the nodes, the level-1 kernel is the
    # exact G_kappa at lattice offsets, Interp takes the nodes back: no approximation
    kappa = 0.5
    rng = np.random.default_rng(13)
    blocks = W.eden_layout(14, rng)
    f = rng.standard_normal((len(blocks), 4, 4, 4))
    got = flgf.solve(blocks, f, 4, 5, 1, kappa=kappa)
    ref = _exact(blocks, f, 4, kappa)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_flgf_converges_in_p_at_full_depth():
    kappa = 0.3
    rng = np.random.default_rng(14)
    blocks = W.eden_layout(40, rng)
    f, _ = W.zero_mean_gaussians(blocks, 8, rng, 6)
    ref = _exact(blocks, f, 8, kappa)
    errs = [float(np.max(np.abs(flgf.solve(blocks, f, 8, p, 0, kappa=kappa) - ref)) / np.max(np.abs(ref)))
            for p in (3, 5, 9)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


def test_flgf_manufactured_solution():
    kappa, n = 0.6, 8
    rng = np.random.default_rng(15)
    blocks = W.eden_layout(30, rng)
    u, f = _manufactured(blocks, n, kappa, rng)
    got = flgf.solve(blocks, f, n, n + 1, 0, kappa=kappa)
    assert np.max(np.abs(got - u)) < 1e-6


def test_screened_kernel_needs_lattice_nodes():
    with pytest.raises(ValueError):
        flgf.FLGF(W.cube_layout(2), 8, 6, 0, kappa=1.0)
    with pytest.raises(ValueError):
        olgf.lgf_table(4, 1e-4)
