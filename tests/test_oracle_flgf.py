"""Pins of the oracle's exact direct sum (oracle A) and of its step-by-step FLGF
(oracle B) against facts fixed by the paper and by the mathematics."""
import numpy as np
import pytest

from oracle import flgf, lgf
from paper_1402_6081_amd import workloads as W


def _flat_points(blocks, n):
    return W.points_of(blocks, n).reshape(-1, 3)


def _exact(blocks, n, f):
    P = _flat_points(blocks, n)
    return lgf.direct_sum(P, f.reshape(-1), P).reshape(f.shape)


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def _dense_from_blocks(blocks, n, vals):
    b = np.asarray(blocks) - np.min(blocks, axis=0)
    ext = b.max(axis=0) + 1
    D = np.zeros((ext[2] * n, ext[1] * n, ext[0] * n))
    for i, (bx, by, bz) in enumerate(b.tolist()):
        D[bz * n:(bz + 1) * n, by * n:(by + 1) * n, bx * n:(bx + 1) * n] = vals[i]
    return D


def _blocks_from_dense(blocks, n, D):
    b = np.asarray(blocks) - np.min(blocks, axis=0)
    out = np.zeros((len(b), n, n, n))
    for i, (bx, by, bz) in enumerate(b.tolist()):
        out[i] = D[bz * n:(bz + 1) * n, by * n:(by + 1) * n, bx * n:(bx + 1) * n]
    return out


def _manufactured(blocks, n, seed):
    """u_rand and f = L u_rand restricted to the layout (Sec. 4.1): since u_rand is 0 on
    boundary points, L u_rand vanishes outside the active grid, so G * f = u_rand."""
    rng = np.random.default_rng(seed)
    u = W.random_manufactured(blocks, n, rng)
    D = _dense_from_blocks(blocks, n, u)
    LD = lgf.laplacian(D)
    # L u_rand outside the bounding box must vanish (boundary points are 0)
    assert np.max(np.abs(LD[0])) == 0 and np.max(np.abs(LD[-1])) == 0
    f = _blocks_from_dense(blocks, n, LD[1:-1, 1:-1, 1:-1])
    # and inside the box, outside the active blocks, too
    active = _dense_from_blocks(blocks, n, np.ones_like(u))
    outside = LD[1:-1, 1:-1, 1:-1][active == 0]
    assert outside.size == 0 or np.max(np.abs(outside)) == 0
    return u, f


# ----------------------------------------------------------------------------- oracle A

@pytest.mark.parametrize("layout", ["cube", "eden"])
def test_direct_sum_inverts_laplacian(layout):
    n = 4
    blocks = W.cube_layout(3) if layout == "cube" else W.eden_layout(14, np.random.default_rng(5))
    u, f = _manufactured(blocks, n, 11)
    ua = _exact(blocks, n, f)
    assert _rel(ua, u) < 1e-12


def test_direct_sum_point_source():
    # f = delta_m gives u = G(. - m): the direct sum reduces to a table lookup
    blocks = W.cube_layout(2)
    n = 4
    f = np.zeros((8, n, n, n))
    f[3, 1, 2, 0] = 1.0
    P = _flat_points(blocks, n)
    m = W.points_of(blocks, n)[3, 1, 2, 0]
    u = _exact(blocks, n, f).reshape(-1)
    assert np.max(np.abs(u - lgf.lgf(P - m))) < 1e-16


# ----------------------------------------------------------------------------- interpolation

@pytest.mark.parametrize("n,p", [(8, 6), (16, 8), (8, 9), (4, 3), (16, 10)])
def test_block_matrix_reproduces_polynomials(n, p):
    # Lagrange interpolation on p nodes is exact for degree <= p-1 (Sec. 2.5):
    # sum_k A[k, j] q(k) = q(j (p-1)/n)
    A = flgf.block_matrix(n, p)
    t = np.arange(n) * (p - 1) / n
    for deg in range(p):
        q = lambda s: (s - 0.37) ** deg
        assert np.max(np.abs(A.T @ q(np.arange(p)) - q(t))) < 1e-9 * max(1.0, (p - 1) ** deg)


@pytest.mark.parametrize("p", [2, 3, 6, 8, 10])
def test_child_matrices_reproduce_polynomials(p):
    C = flgf.child_matrices(p)
    for c in (0, 1):
        t = (c * (p - 1) + np.arange(p)) / 2.0
        for deg in range(p):
            q = lambda s: (s - 1.3) ** deg
            assert np.max(np.abs(C[c].T @ q(np.arange(p)) - q(t))) < 1e-9 * max(1.0, (p - 1) ** deg)


def test_identity_when_p_is_n_plus_one():
    # p = n + 1: level-1 nodes coincide with grid points (Sec. 4)
    A = flgf.block_matrix(8, 9)
    assert np.max(np.abs(A[:8] - np.eye(8))) < 1e-15 and np.max(np.abs(A[8])) < 1e-15


def test_reg_is_adjoint_of_interp():
    rng = np.random.default_rng(0)
    A = flgf.block_matrix(8, 6)
    f = rng.standard_normal((2, 8, 8, 8))
    v = rng.standard_normal((2, 6, 6, 6))
    lhs = np.sum(flgf.reg_block(A, f) * v)
    rhs = np.sum(f * flgf.interp_block(A, v))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# ----------------------------------------------------------------------------- lists

@pytest.mark.parametrize("seed,levels", [(0, 0), (1, 0), (2, 2), (3, 3), (4, 1)])
def test_lists_cover_every_pair_once(seed, levels):
    rng = np.random.default_rng(seed)
    blocks = W.eden_layout(60, rng)
    t = flgf.Tree(blocks, levels)
    nb = len(t.blocks)
    count = np.zeros((nb, nb), dtype=int)
    np.add.at(count, (t.near[0], t.near[1]), 1)
    # leaves under each interval, by walking parents
    anc = {1: np.arange(nb)}
    for l in range(1, t.L):
        anc[l + 1] = t.parent[l][anc[l]]
    for l in range(1, t.L + 1):
        tgt, src, _ = t.ilist[l]
        hit = np.zeros((t.coords[l].shape[0],) * 2, dtype=int)
        np.add.at(hit, (tgt, src), 1)
        count += hit[anc[l][:, None], anc[l][None, :]]
    assert np.all(count == 1)


def test_interaction_list_size_bounded_by_189():
    t = flgf.Tree(W.cube_layout(16), 0)
    for l in range(1, t.L):
        tgt = t.ilist[l][0]
        if tgt.size:
            assert np.bincount(tgt).max() <= 189


# ----------------------------------------------------------------------------- oracle B

def test_no_far_field_is_exact():
    # few blocks: only the block-wise FFT convolution, error near machine precision
    rng = np.random.default_rng(1)
    blocks = W.cube_layout(2)
    f = rng.standard_normal((8, 8, 8, 8))
    assert _rel(flgf.solve(blocks, f, 8, 6, 0), _exact(blocks, 8, f)) < 1e-14


@pytest.mark.parametrize("layout", ["cube4", "eden"])
def test_lattice_nodes_single_level_is_exact(layout):
    # p = n + 1 and a single level: Reg/Interp are the identity and the level-1
    # kernel is the exact G, so the far field is exact as well
    rng = np.random.default_rng(2)
    blocks = W.cube_layout(4) if layout == "cube4" else W.eden_layout(20, rng)
    n = 4
    f = rng.standard_normal((len(blocks), n, n, n))
    assert _rel(flgf.solve(blocks, f, n, n + 1, 1), _exact(blocks, n, f)) < 1e-14


def test_fft_convolution_against_dense_kernel_sum():
    # Step 2 + Step 3a via FFTs equals the compressed-kernel sum of Eq. ifmm evaluated
    # densely over node pairs (brute force; pins Pad/Trunc/kernel placement)
    rng = np.random.default_rng(4)
    blocks = W.eden_layout(40, rng)
    n, p = 4, 3
    solver = flgf.FLGF(blocks, n, p, 0)
    f = rng.standard_normal((len(blocks), n, n, n))
    _, lv = solver.solve(f, return_levels=True)
    t = solver.tree
    for l in range(1, t.L + 1):
        s, h, lattice = flgf.level_geometry(n, p, l)
        k = np.stack(np.meshgrid(np.arange(p), np.arange(p), np.arange(p), indexing="ij"), -1)
        kxyz = k[..., ::-1].reshape(-1, 3)  # node offsets (x, y, z) in [z, y, x] order
        tgt, src, _ = t.ilist[l]
        v = np.zeros((t.coords[l].shape[0], p ** 3))
        for P, Q in zip(tgt.tolist(), src.tolist()):
            xp = t.coords[l][P] * s + kxyz * h
            xq = t.coords[l][Q] * s + kxyz * h
            K = flgf.kernel_values(xp[:, None, :] - xq[None, :, :], lattice)
            v[P] += K @ lv["ftilde"][l][Q].reshape(-1)
        assert np.max(np.abs(v - lv["vtilde"][l].reshape(v.shape))) < 1e-13 * max(1.0, np.max(np.abs(v)))


def test_near_field_against_dense_sum():
    rng = np.random.default_rng(6)
    blocks = W.eden_layout(12, rng)
    n = 4
    f = rng.standard_normal((len(blocks), n, n, n))
    solver = flgf.FLGF(blocks, n, 3, 0)
    _, lv = solver.solve(f, return_levels=True)
    P = W.points_of(solver.tree.blocks, n)
    tgt, src, _ = solver.tree.near
    ref = np.zeros_like(f)
    for a, b in zip(tgt.tolist(), src.tolist()):
        G = lgf.lgf(P[a].reshape(-1, 1, 3) - P[b].reshape(1, -1, 3))
        ref[a] += (G @ f[b].reshape(-1)).reshape(n, n, n)
    assert np.max(np.abs(ref - lv["vnear"])) < 1e-14 * np.max(np.abs(ref))


def test_truncation_error_decays_geometrically_in_p():
    # p-refinement converges geometrically for p <= n_max (Sec. 2.5)
    c = W.config_small()
    exact = _exact(c["blocks"], c["n"], c["f"])
    errs = [_rel(flgf.solve(c["blocks"], c["f"], c["n"], p, c["levels"]), exact) for p in (4, 6, 8, 10)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 10.0, errs
    assert errs[1] < 1e-5  # p = 6 on the 32^3 case


def test_manufactured_solution_through_flgf():
    blocks = W.cube_layout(4)
    n = 8
    u, f = _manufactured(blocks, n, 7)
    assert _rel(flgf.solve(blocks, f, n, 8, 0), u) < 1e-5
    assert _rel(flgf.solve(blocks, f, n, n + 1, 0), u) < 1e-12


def test_translation_invariance():
    rng = np.random.default_rng(8)
    blocks = W.eden_layout(30, rng)
    f = rng.standard_normal((len(blocks), 4, 4, 4))
    a = flgf.solve(blocks, f, 4, 3, 0)
    b = flgf.solve(blocks + np.array([5, -7, 100]), f, 4, 3, 0)
    assert np.array_equal(a, b)


def test_layout_validation():
    with pytest.raises(ValueError):
        flgf.Tree(np.zeros((0, 3)), 0)
    with pytest.raises(ValueError):
        flgf.Tree(np.array([[0, 0, 0], [0, 0, 0]]), 0)
