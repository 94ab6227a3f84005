"""Host-side plan logic (tree, lists, workspace estimate) through lgf_plan_estimate, which
does no device work: checked against the oracle's plain O(N^2) list enumeration and
against closed forms (runs without a GPU)."""
import ctypes
import os

import numpy as np
import pytest

from oracle import flgf
from paper_1402_6081_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1402_6081_amd", "libpaper_lgf.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


@pytest.fixture(scope="module")
def L():
    import torch  # noqa: F401  (shares the HIP runtime with the library)
    from paper_1402_6081_amd import lgf as L
    L.library()
    return L


CASES = [
    ("eden60_full", 60, 0),
    ("eden150_full", 150, 0),
    ("eden150_L2", 150, 2),
    ("eden90_L3", 90, 3),
    ("eden1", 1, 0),
    ("eden2", 2, 0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_lists_match_oracle_tree(L, case):
    label, nb, levels = case
    rng = np.random.default_rng(len(label) * 1000 + nb)
    blocks = W.eden_layout(nb, rng)
    # shift to an arbitrary origin: the plan anchors at the bounding-box minimum
    blocks = blocks + np.array([-7, 3, 100], dtype=np.int32)
    info = L.plan_estimate(blocks, 8, 6, levels, "f64")
    tree = flgf.Tree(blocks, levels)
    assert info["levels"] == tree.L
    assert info["near_pairs"] == len(tree.near[0])
    top = 0
    for lvl in range(1, tree.L + 1):
        assert info["intervals"][lvl] == tree.coords[lvl].shape[0], lvl
        assert info["far_pairs"][lvl] == len(tree.ilist[lvl][0]), lvl
        if len(tree.ilist[lvl][0]):
            top = lvl
    assert info["top_level"] == top
    assert info["intervals"][0] == nb and info["npoints"] == nb * 512


@pytest.mark.parametrize("k,levels,expect", [
    (4, 2, [1000, 3096, 0]),                     # 32^3 of 8^3 blocks, 2 levels
    (8, 4, [10648, 53352, 3096, 0, 0]),          # 128^3 of 16^3 blocks, 4 levels
    (16, 0, [97336, 584136, 53352, 3096, 0]),    # 256^3 of 16^3 blocks, full depth
])
def test_cube_pair_counts(L, k, levels, expect):
    """Near pairs of a k^3 cube of blocks: (3k - 2)^3 (each axis contributes
    k + 2 (k - 1) ordered pairs with |d| <= 1).  The interaction-list counts per level are
    the ones the oracle's tree enumerates on the same cubes (checked here for k <= 8)."""
    info = L.plan_estimate(W.cube_layout(k), 16, 8, levels, "f32")
    assert info["near_pairs"] == (3 * k - 2) ** 3 == expect[0]
    for lvl, cnt in enumerate(expect[1:], start=1):
        assert info["far_pairs"][lvl] == cnt, lvl
    if k <= 8:
        tree = flgf.Tree(W.cube_layout(k), levels)
        for lvl in range(1, tree.L + 1):
            assert len(tree.ilist[lvl][0]) == info["far_pairs"][lvl]


def test_interaction_list_size_bound(L):
    """No interval has more than 189 = 6^3 - 3^3 interaction-list entries (Sec. 3.1)."""
    info = L.plan_estimate(W.cube_layout(16), 16, 8, 0, "f32")
    for lvl in range(1, info["levels"] + 1):
        assert info["far_pairs"][lvl] <= 189 * info["intervals"][lvl]


def test_workspace_estimate_scales(L):
    a = L.plan_estimate(W.cube_layout(4), 16, 8, 0, "f32")["workspace_bytes"]
    b = L.plan_estimate(W.cube_layout(4), 16, 8, 0, "f64")["workspace_bytes"]
    c = L.plan_estimate(W.cube_layout(8), 16, 8, 0, "f32")["workspace_bytes"]
    # level-0 spectra dominate: 2 N_B + 1 items of 16^2 * 17 (padded to 64) complex values
    s0 = 32 * 32 * 17
    assert a > (2 * 64 + 1) * s0 * 8
    assert 1.6 < b / a < 2.1
    assert 7.0 < c / a < 9.0


def test_layout_errors(L):
    with pytest.raises(L.LGFError) as e:
        L.plan_estimate(np.array([[0, 0, 0], [1, 0, 0], [0, 0, 0]]), 8, 6)
    assert e.value.name == "LGF_ERR_LAYOUT"
    with pytest.raises(L.LGFError) as e:
        L.plan_estimate(np.array([[0, 0, 0], [1 << 21, 0, 0]]), 8, 6)
    assert e.value.name == "LGF_ERR_LAYOUT"
    for n, p in ((10, 6), (12, 11), (16, 13), (8, 12)):  # n unsupported; p > 10 only as n + 1 for n = 12, 16
        with pytest.raises(L.LGFError) as e:
            L.plan_estimate(np.array([[0, 0, 0]]), n, p)
        assert e.value.name == "LGF_ERR_ARG"
    for n, p in ((6, 7), (12, 13), (12, 8), (16, 17)):  # the scheme family n_I = n + 1 and others
        assert L.plan_estimate(np.array([[0, 0, 0], [3, 0, 0]]), n, p)["n"] == n


def test_server_config_errors(L):
    lib = L.library()
    h = ctypes.c_void_p()
    bad = [L.ServerConfig(0, 0, 0, 16, 8, 0, 1),    # no slots
           L.ServerConfig(0, 4, 0, 10, 8, 0, 1),    # n unsupported
           L.ServerConfig(-1, 4, 0, 16, 8, 0, 1),   # negative budget
           L.ServerConfig(0, 4, 0, 16, 8, 0, 7)]    # unknown precision
    for cfg in bad:
        assert lib.lgf_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 1
    assert lib.lgf_server_submit(None, None, 1, None, None, None, None) == 1
    assert lib.lgf_server_destroy(None) == 0
    assert lib.lgf_graph_create(None, None, None, None, ctypes.byref(h)) == 1
    t = L.Tuning(0, 4, 0, 0, 0, 0)
    assert lib.lgf_plan_set_tuning(None, ctypes.byref(t)) == 1
    assert lib.lgf_plan_get_tuning(None, ctypes.byref(t)) == 1
    assert lib.lgf_plan_create_batch(None, None, 0, 8, 6, 0, 0, None, ctypes.byref(h)) == 1


SPLIT_CASES = [(k, lv) for k in ("dilated", "subset", "disjoint") for lv in (0, 2)]


@pytest.mark.parametrize("kind,levels", SPLIT_CASES)
def test_split_lists_match_oracle_tree(L, kind, levels):
    """Separate source and evaluation blocks: the plan's list sizes are the oracle's lists
    (evaluation targets x source intervals), its intervals those of the union of the two
    trees."""
    rng = np.random.default_rng(21)
    src, ev = W.split_sets(kind, rng)
    shift = np.array([4, -9, 31], dtype=np.int32)
    info = L.plan_estimate(src + shift, 8, 6, levels, "f64", eval_blocks=ev + shift)
    tree = flgf.Tree(src, levels, ev)
    assert info["levels"] == tree.L
    assert info["source_blocks"] == len(src) and info["eval_blocks"] == len(ev)
    assert info["near_pairs"] == len(tree.near[0])
    top = 0
    for lvl in range(1, tree.L + 1):
        union = np.unique(np.vstack([tree.coords[lvl], tree.coords_e[lvl]]), axis=0)
        assert info["intervals"][lvl] == union.shape[0], lvl
        assert info["far_pairs"][lvl] == len(tree.ilist[lvl][0]), lvl
        if len(tree.ilist[lvl][0]):
            top = lvl
    assert info["top_level"] == top
    assert info["nblocks"] == info["intervals"][1]


def test_split_with_equal_sets_matches_single_set(L):
    rng = np.random.default_rng(22)
    blocks = W.eden_layout(120, rng)
    perm = rng.permutation(len(blocks))
    a = L.plan_estimate(blocks, 8, 6, 0, "f32")
    b = L.plan_estimate(blocks, 8, 6, 0, "f32", eval_blocks=blocks[perm])
    for k in ("nblocks", "levels", "top_level", "near_pairs", "far_pairs", "intervals"):
        assert a[k] == b[k], k
    # the split plan adds only its evaluation -> level-1 map
    assert b["workspace_bytes"] == a["workspace_bytes"] + 4 * len(blocks)


def test_split_layout_errors(L):
    src = W.cube_layout(2)
    for ev, name in ((np.array([[0, 0, 0], [0, 0, 0]]), "LGF_ERR_LAYOUT"),
                     (np.zeros((0, 3)), "LGF_ERR_LAYOUT"),
                     (np.array([[0, 0, 0], [1 << 21, 0, 0]]), "LGF_ERR_LAYOUT")):
        with pytest.raises(L.LGFError) as e:
            L.plan_estimate(src, 8, 6, eval_blocks=ev)
        assert e.value.name == name
    with pytest.raises(L.LGFError) as e:
        L.plan_estimate(np.array([[1, 1, 1], [1, 1, 1]]), 8, 6, eval_blocks=src)
    assert e.value.name == "LGF_ERR_LAYOUT"
    info = L.PlanInfo()
    lib = L.library()
    st = lib.lgf_plan_estimate_split(src.ctypes.data, len(src), None, 4, 8, 6, 0, 0, ctypes.byref(info))
    assert st == 1  # LGF_ERR_ARG


def test_lattice_scheme_arguments(L):
    """p = n + 1 = 17 (the paper's scheme at n = 16, stencils of n_max = 10 nodes) is
    accepted; other p above 10 are not."""
    blocks = W.cube_layout(4)
    info = L.plan_estimate(blocks, 16, 17, 0, "f64")
    tree = flgf.Tree(blocks, 0)
    assert info["near_pairs"] == len(tree.near[0])
    for lvl in range(1, tree.L + 1):
        assert info["far_pairs"][lvl] == len(tree.ilist[lvl][0])
    for n, p in ((8, 17), (16, 11), (16, 16), (16, 18), (4, 17)):
        with pytest.raises(L.LGFError) as e:
            L.plan_estimate(blocks, n, p)
        assert e.value.name == "LGF_ERR_ARG", (n, p)


def test_lattice_scheme_workspace(L):
    """Level 1 of the lattice scheme keeps no spectra of its own (it reads the blocks'), and
    levels >= 2 add a two-phase transform intermediate: 17 * 34 * 18 complex per interval
    of the largest such level."""
    blocks = W.cube_layout(8)
    info = L.plan_estimate(blocks, 16, 17, 0, "f64")
    nb, n2 = info["intervals"][1], info["intervals"][2]
    S0 = 32 * 32 * 17
    S2 = (34 * 34 * 18 + 63) // 64 * 64
    spectra_part = (2 * nb + 1) * S0 * 16 + nb * S0 * 16 + (2 * n2 + 1) * S2 * 16
    scratch = n2 * 17 * 34 * 18 * 16
    assert info["workspace_bytes"] > spectra_part + scratch
    assert info["workspace_bytes"] < 1.2 * (spectra_part + scratch)
