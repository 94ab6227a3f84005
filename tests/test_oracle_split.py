"""Pins of the oracle FLGF with separate source and evaluation block sets (B_s != B_e,
Eq. bconv): u^P = sum_{Q in B_s} conv(k^{Q-P}, f^Q) for every P in B_e."""
import numpy as np
import pytest

from oracle import flgf, lgf
from paper_1402_6081_amd import workloads as W


def _exact(src, ev, n, f):
    """Eq. bconv by brute force: exact G over every (evaluation point, source point)."""
    lo = np.minimum(np.min(src, axis=0), np.min(ev, axis=0))
    S = W.points_of(np.asarray(src) - lo, n).reshape(-1, 3)
    T = W.points_of(np.asarray(ev) - lo, n).reshape(-1, 3)
    return lgf.direct_sum(S, f.reshape(-1), T).reshape(len(ev), n, n, n)


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("kind", ["dilated", "subset", "disjoint"])
def test_lists_cover_every_eval_source_pair_once(kind):
    # every (evaluation block, source block) pair is reached by exactly one list entry:
    # the near list at level 0, or the interaction list of one level (via the ancestors)
    rng = np.random.default_rng(11)
    src, ev = W.split_sets(kind, rng)
    for levels in (0, 2):
        t = flgf.Tree(src, levels, ev)
        ns, ne = len(t.blocks), len(t.eval_blocks)
        count = np.zeros((ne, ns), dtype=int)
        np.add.at(count, (t.near[0], t.near[1]), 1)
        anc_s, anc_e = {1: np.arange(ns)}, {1: np.arange(ne)}
        for l in range(1, t.L):
            anc_s[l + 1] = t.parent[l][anc_s[l]]
            anc_e[l + 1] = t.parent_e[l][anc_e[l]]
        for l in range(1, t.L + 1):
            tgt, s, _ = t.ilist[l]
            hit = np.zeros((t.coords_e[l].shape[0], t.coords[l].shape[0]), dtype=int)
            np.add.at(hit, (tgt, s), 1)
            count += hit[anc_e[l][:, None], anc_s[l][None, :]]
        assert np.all(count == 1), (kind, levels)


@pytest.mark.parametrize("kind", ["dilated", "subset", "disjoint"])
def test_lattice_single_level_is_exact(kind):
    # p = n + 1 and one level: Reg/Interp are the identity and the level-1 kernel is the
    # exact G, so the FLGF equals Eq. bconv to rounding
    rng = np.random.default_rng(12)
    src, ev = W.split_sets(kind, rng)
    n = 4
    f = rng.standard_normal((len(src), n, n, n))
    u = flgf.solve(src, f, n, n + 1, 1, eval_blocks=ev)
    assert u.shape == (len(ev), n, n, n)
    assert _rel(u, _exact(src, ev, n, f)) < 1e-13


@pytest.mark.parametrize("kind", ["dilated", "subset", "disjoint"])
def test_full_depth_within_interpolation_error(kind):
    # the multilevel scheme (every level, p nodes per interval edge) converges to Eq. bconv
    # geometrically in p, as in the same-set case (Sec. 2.5): a wrong list, tree or
    # transfer on either side leaves an O(1) error instead
    rng = np.random.default_rng(13)
    src, ev = W.split_sets(kind, rng)
    n = 8
    f = rng.standard_normal((len(src), n, n, n))
    exact = _exact(src, ev, n, f)
    errs = [_rel(flgf.solve(src, f, n, p, 0, eval_blocks=ev), exact) for p in (4, 6, 8)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 10.0, errs
    assert errs[0] < 2e-3 and errs[-1] < 2e-6, errs


def test_equal_sets_reduce_to_the_single_set_solve():
    rng = np.random.default_rng(14)
    blocks = W.eden_layout(40, rng)
    n, p = 4, 3
    f = rng.standard_normal((len(blocks), n, n, n))
    ref = flgf.solve(blocks, f, n, p, 0)
    perm = rng.permutation(len(blocks))
    u = flgf.solve(blocks, f, n, p, 0, eval_blocks=blocks[perm])
    assert np.max(np.abs(u - ref[perm])) <= 1e-15 * np.max(np.abs(ref))


def test_evaluation_restricts_and_source_order_is_free():
    # with the union's anchor and extent held fixed, u on a subset of B_e is the
    # restriction of u on B_e (targets do not interact), and permuting the source blocks
    # together with their fields changes nothing
    rng = np.random.default_rng(15)
    src, ev = W.split_sets("dilated", rng)
    n, p = 4, 3
    f = rng.standard_normal((len(src), n, n, n))
    u = flgf.solve(src, f, n, p, 0, eval_blocks=ev)
    lo, hi = ev.min(axis=0), ev.max(axis=0)
    # every third block, plus each block on a face of the bounding box (anchor and extent)
    keep = [i for i in range(len(ev)) if i % 3 == 0 or np.any(ev[i] == lo) or np.any(ev[i] == hi)]
    assert len(keep) < len(ev)
    sub = flgf.solve(src, f, n, p, 0, eval_blocks=ev[keep])
    assert np.max(np.abs(sub - u[keep])) <= 1e-15 * np.max(np.abs(u))
    perm = rng.permutation(len(src))
    u2 = flgf.solve(src[perm], f[perm], n, p, 0, eval_blocks=ev)
    assert np.max(np.abs(u2 - u)) <= 1e-14 * np.max(np.abs(u))


def test_sources_absent_from_evaluation_are_superposed():
    # linearity across the two sets: sources split into two parts give the sum of the
    # two solves on the same evaluation blocks (same anchor and extent)
    rng = np.random.default_rng(16)
    src, ev = W.split_sets("dilated", rng)
    n, p = 4, 3
    f = rng.standard_normal((len(src), n, n, n))
    fa, fb = f.copy(), f.copy()
    half = np.arange(len(src)) % 2 == 0
    fa[~half] = 0.0
    fb[half] = 0.0
    u = flgf.solve(src, f, n, p, 0, eval_blocks=ev)
    ua = flgf.solve(src, fa, n, p, 0, eval_blocks=ev)
    ub = flgf.solve(src, fb, n, p, 0, eval_blocks=ev)
    assert np.max(np.abs(ua + ub - u)) <= 1e-13 * np.max(np.abs(u))


def test_separate_set_validation():
    src = W.cube_layout(2)
    with pytest.raises(ValueError):
        flgf.Tree(src, 0, np.zeros((0, 3)))
    with pytest.raises(ValueError):
        flgf.Tree(src, 0, np.array([[0, 0, 0], [0, 0, 0]]))
