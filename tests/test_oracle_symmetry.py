"""The identity the symmetry-reduced kernel spectra rest on, checked on the oracle's own
kernel tiles (Sec. 2.1: the LGF is invariant under axis reflections and permutations;
Sec. 3.2: unique kernel vectors per level).

With g a signed permutation of the axes, (g v)_i = s_i v_{perm(i)}, the tile of offset g D
is the tile of D with its offsets mapped by g^-1, so its spectrum at frequency omega is the
spectrum of D at g^-1 omega (indices mod M).  In the stored half spectrum (x frequency
<= M/2) a frequency outside the half is read as the conjugate at its negative.  The class
count of the 27 level-0 offsets is the paper's 4."""
import itertools

import numpy as np

from oracle import flgf


def group():
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            yield perm, signs


def act(g, v):
    perm, s = g
    return tuple(s[i] * v[perm[i]] for i in range(3))


def pull_back(g, wx, wy, wz, M):
    """nu = g^-1 omega for arrays of frequency components: g nu = omega."""
    perm, s = g
    w = (wx, wy, wz)
    nu = [None, None, None]
    for i in range(3):
        nu[perm[i]] = (s[i] * w[i]) % M
    return nu


KERNELS = [
    # (tile edge m, kernel of the offsets, offsets D)
    (4, flgf.near_kernel_fn(4), [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1)]),      # level 0, exact G
    (5, flgf.far_kernel_fn(4, 5, 2), [(2, 1, 0), (3, 2, 1), (3, 3, 0)]),            # nodes on the lattice
    (6, flgf.far_kernel_fn(4, 6, 1), [(2, 0, 0), (3, 2, 1), (2, 2, 1)]),            # asymptotic kernel
]


def test_kernel_spectra_follow_the_symmetry():
    for m, fn, offsets in KERNELS:
        M = 2 * m
        wz, wy, wx = np.meshgrid(np.arange(M), np.arange(M), np.arange(M), indexing="ij")
        for D in offsets:
            base = np.fft.fftn(flgf.kernel_block(D, m, fn))  # [kz, ky, kx]
            scale = np.max(np.abs(base))
            for g in group():
                k = np.fft.fftn(flgf.kernel_block(act(g, D), m, fn))
                nx, ny, nz = pull_back(g, wx, wy, wz, M)
                assert np.max(np.abs(k - base[nz, ny, nx])) < 1e-13 * scale, (m, D, g)


def test_half_spectrum_read_with_conjugation():
    # the stored half [kz][ky][kx <= M/2]: a pulled-back frequency with x component above
    # M/2 is read as the conjugate at -nu
    m, fn = 5, flgf.far_kernel_fn(4, 5, 2)
    M, H = 2 * m, m + 1
    wz, wy, wx = np.meshgrid(np.arange(M), np.arange(M), np.arange(H), indexing="ij")
    D = (3, 2, 1)
    half = np.fft.rfftn(flgf.kernel_block(D, m, fn))  # [kz, ky, kx <= M/2]
    for g in group():
        want = np.fft.rfftn(flgf.kernel_block(act(g, D), m, fn))
        nx, ny, nz = pull_back(g, wx, wy, wz, M)
        cj = nx > M // 2
        nx, ny, nz = np.where(cj, (M - nx) % M, nx), np.where(cj, (M - ny) % M, ny), np.where(cj, (M - nz) % M, nz)
        got = np.where(cj, np.conj(half[nz, ny, nx]), half[nz, ny, nx])
        assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(half)), g


def test_class_counts():
    # orbits of the offsets in [-R, R]^3 under the 48 signed permutations: the 27 level-0
    # offsets fall into the paper's 4 classes; radius 3 gives 20 (16 outside the near range)
    for R, want in ((1, 4), (3, 20)):
        pts = list(itertools.product(range(-R, R + 1), repeat=3))
        orbits = {tuple(sorted((abs(c) for c in D), reverse=True)) for D in pts}
        assert len(orbits) == want
        # each orbit is closed under the group
        for D in pts:
            assert all(tuple(sorted((abs(c) for c in act(g, D)), reverse=True)) ==
                       tuple(sorted((abs(c) for c in D), reverse=True)) for g in group())
    far = {tuple(sorted((abs(c) for c in D), reverse=True)) for D in itertools.product(range(-3, 4), repeat=3)
           if max(abs(c) for c in D) > 1}
    assert len(far) == 16
