"""GPU parity of plans with separate source and evaluation blocks (lgf_plan_create_split,
Eq. bconv with B_s != B_e) through the C ABI.

Tolerances as for the single-set plans: FP64 against the oracle's FLGF (separate source
and evaluation trees) within max(1e-12, Lambda_p^3 eps_64); FP32 against FP64 and the
oracle within 1e-6 of max|u| over the evaluation blocks, on smooth sources.  Properties that hold at any size are checked bit for bit: a split
plan equals the single-set plan of the union with zero sources outside B_s, restricted to
B_e, and equal sets through the split entry equal the single-set plan."""
import json
import os
import sys
import zlib

import numpy as np
import pytest
import torch

from oracle import flgf, lgf as olgf
from paper_1402_6081_amd import workloads as W
from tolerances import FP32_BAR, fp64_tol, rel

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_1402_6081_amd.lgf as L
    L.library()
    return L


def split_solve(L, src, ev, f, n, p, levels, precision="f64", graph=False):
    dt = torch.float64 if precision == "f64" else torch.float32
    plan = L.Plan(src, n, p, levels, precision, eval_blocks=ev)
    fd = torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0", dt)
    if graph:
        u = torch.empty(plan.out_shape(), dtype=dt, device="cuda:0")
        g = plan.graph(fd, u)
        for _ in range(3):
            u.fill_(float("nan"))
            g.launch()
            torch.cuda.synchronize()
        g.close()
    else:
        u = plan.solve(fd)
        torch.cuda.synchronize()
    assert tuple(u.shape) == (len(ev), n, n, n)
    out = u.double().cpu().numpy()
    plan.close()
    return out


CASES = [
    ("dilated", 8, 6, 0),
    ("subset", 8, 6, 0),
    ("disjoint", 8, 6, 0),
    ("dilated", 4, 3, 2),
    ("disjoint", 16, 8, 0),
    ("subset", 8, 9, 1),
]


@pytest.mark.parametrize("case", CASES, ids=["%s_n%d_p%d_L%d" % c for c in CASES])
def test_split_fp64_matches_oracle(L, case):
    kind, n, p, levels = case
    rng = np.random.default_rng(zlib.crc32(("split%s%d%d%d" % case).encode()))
    src, ev = W.split_sets(kind, rng)
    f = rng.standard_normal((len(src), n, n, n))
    _say("case: split", case, "sources", len(src), "evaluation", len(ev))
    ref = flgf.solve(src, f, n, p, levels, eval_blocks=ev)
    got = split_solve(L, src, ev, f, n, p, levels)
    e = rel(got, ref)
    _say("   rel Linf vs oracle = %.3e (tol %.1e)" % (e, fp64_tol(p)))
    assert e < fp64_tol(p)


@pytest.mark.parametrize("kind", ["dilated", "subset", "disjoint"])
def test_split_fp32_within_1e6_of_fp64(L, kind):
    # the FP32 path with separate sets against the device's FP64 solve and against the
    # oracle's FLGF, relative to max|u| over the evaluation blocks B_e
    rng = np.random.default_rng(zlib.crc32(("split32" + kind).encode()))
    src, ev = W.split_sets(kind, rng)
    n, p = 16, 8
    f, _ = W.zero_mean_gaussians(src, n, rng, 4)
    _say("case: split FP32", kind)
    u64 = split_solve(L, src, ev, f, n, p, 0, "f64")
    u32 = split_solve(L, src, ev, f, n, p, 0, "f32", graph=True)
    ref = flgf.solve(src, f, n, p, 0, eval_blocks=ev)
    _, scale = _union_reference(L, src, ev, f, n, p, 0, "f64")
    e_union = float(np.max(np.abs(u32 - u64)) / scale)
    e64, e_or = rel(u32, u64), rel(u32, ref)
    _say("   FP32 vs FP64: %.3e of max|u| over B_e (%.3e of max|u| over the union); vs oracle FLGF %.3e"
         % (e64, e_union, e_or))
    assert e64 <= FP32_BAR
    assert e_or <= FP32_BAR


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_split_with_equal_sets_is_the_single_set_plan(L, prec):
    rng = np.random.default_rng(31)
    blocks = W.eden_layout(80, rng)
    perm = rng.permutation(len(blocks))
    n, p = 16, 8
    f = rng.standard_normal((len(blocks), n, n, n))
    _say("case: split entry with equal sets", prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = L.Plan(blocks, n, p, 0, prec)
    ref = plan.solve(torch.from_numpy(f).to("cuda:0", dt))
    torch.cuda.synchronize()
    got = split_solve(L, blocks, blocks[perm], f, n, p, 0, prec)
    assert np.array_equal(got, ref.double().cpu().numpy()[perm])
    plan.close()


def _union_reference(L, src, ev, f, n, p, levels, prec):
    """Single-set plan over B_s + (B_e minus B_s) with zero sources on the added blocks:
    u restricted to B_e (in B_e's order), and max|u| over the whole union."""
    s = {tuple(b): i for i, b in enumerate(src.tolist())}
    extra = [b for b in ev.tolist() if tuple(b) not in s]
    union = np.concatenate([src, np.asarray(extra, dtype=np.int32).reshape(-1, 3)], axis=0)
    pos = {tuple(b): i for i, b in enumerate(union.tolist())}
    fu = np.zeros((len(union), n, n, n))
    fu[:len(src)] = f
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = L.Plan(union, n, p, levels, prec)
    u = plan.solve(torch.from_numpy(fu).to("cuda:0", dt))
    torch.cuda.synchronize()
    full = u.double().cpu().numpy()
    plan.close()
    return full[[pos[tuple(b)] for b in ev.tolist()]], float(np.max(np.abs(full)))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_split_equals_union_with_zero_sources(L, prec):
    # at a size past the oracle's reach: a sphere of sources inside a 12^3-block cube of
    # evaluation blocks, and a cube of sources evaluated on a spherical shell
    n, p = 16, 8
    rng = np.random.default_rng(41)
    for label, src, ev in (("sphere in cube", W.sphere_layout(12), W.cube_layout(12)),
                           ("cube on shell", W.cube_layout(10), W.shell_layout(12) - 1)):
        f, _ = W.zero_mean_gaussians(src, n, rng, 16)
        _say("case: split vs union,", label, prec, "sources", len(src), "evaluation", len(ev))
        got = split_solve(L, src, ev, f, n, p, 0, prec, graph=True)
        ref, _ = _union_reference(L, src, ev, f, n, p, 0, prec)
        assert np.array_equal(got, ref), label


def test_split_config_full_size(L):
    """The separate-set vortex-ring workload (779 source blocks, 4096 evaluation blocks of
    16^3, p = 8, full depth) at full size: FP64 against the oracle's FLGF and exact sum at
    64 stored targets (tests/golden/split_config_samples.json, written by
    make_split_samples.py from the oracle alone); FP32 against FP64 over the whole field and
    against the oracle at the same targets."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "split_config_samples.json")))
    c = W.config_split()
    assert gold["workload"] == c["name"] and gold["source_blocks"] == len(c["blocks"])
    _say("case: split config full size, FP64 + FP32")
    idx = np.asarray(gold["flat_index"])
    u64 = split_solve(L, c["blocks"], c["eval_blocks"], c["f"], c["n"], c["p"], c["levels"], "f64").reshape(-1)
    scale = gold["max_abs_u"]
    assert abs(np.max(np.abs(u64)) - scale) <= 1e-12 * scale
    flgf_ref, exact = np.asarray(gold["flgf"]), np.asarray(gold["exact"])
    err_b = float(np.max(np.abs(u64[idx] - flgf_ref)) / scale)
    trunc = float(np.max(np.abs(flgf_ref - exact)) / np.max(np.abs(exact)))
    err_a = float(np.max(np.abs(u64[idx] - exact)) / np.max(np.abs(exact)))
    _say("  vs oracle FLGF %.3g, vs exact %.3g (oracle FLGF vs exact %.3g)" % (err_b, err_a, trunc))
    assert err_b <= fp64_tol(c["p"])
    assert err_a <= trunc + 1e-12
    u32 = split_solve(L, c["blocks"], c["eval_blocks"], c["f"], c["n"], c["p"], c["levels"], "f32",
                      graph=True).reshape(-1)
    err32 = float(np.max(np.abs(u32 - u64)) / np.max(np.abs(u64)))
    err32_b = float(np.max(np.abs(u32[idx] - flgf_ref)) / scale)
    err32_a = float(np.max(np.abs(u32[idx] - exact)) / np.max(np.abs(exact)))
    _say("  FP32 vs FP64 %.3g; at the stored targets vs oracle FLGF %.3g, vs exact %.3g" % (err32, err32_b, err32_a))
    assert err32 <= FP32_BAR
    assert err32_b <= FP32_BAR
    assert err32_a <= trunc + FP32_BAR


def test_split_rejects_mismatched_fields(L):
    rng = np.random.default_rng(51)
    src, ev = W.split_sets("dilated", rng)
    plan = L.Plan(src, 8, 6, 0, "f64", eval_blocks=ev)
    f = torch.zeros((len(src), 8, 8, 8), dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError):
        plan.solve(f, torch.empty_like(f))  # u must have the evaluation blocks' shape
    with pytest.raises(ValueError):
        plan.solve(torch.zeros((len(ev), 8, 8, 8), dtype=torch.float64, device="cuda:0"))
    info = plan.info()
    assert info["source_blocks"] == len(src) and info["eval_blocks"] == len(ev)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_split_schedules_same_bits(L, prec):
    # the one-stream schedules (overlap 2 and 3) run the levels' transforms and M2L as
    # multi-level launches; the three-branch schedule launches level by level: same bits,
    # eager and as graphs
    rng = np.random.default_rng(71)
    src, ev = W.split_sets("dilated", rng)
    n, p = 8, 6
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = L.Plan(src, n, p, 0, prec, eval_blocks=ev)
    f = torch.from_numpy(rng.standard_normal((len(src), n, n, n))).to("cuda:0", dt)
    info = plan.info()
    _say("case: split schedules", prec, "levels", info["levels"], "top", info["top_level"])
    assert info["top_level"] >= 2  # several far levels: the merged launches have more than one segment
    plan.set_tuning(overlap=1)
    ref = plan.solve(f).clone()
    torch.cuda.synchronize()
    for ov in (2, 3):
        plan.set_tuning(overlap=ov)
        assert torch.equal(plan.solve(f), ref), ov
        u = torch.empty(plan.out_shape(), dtype=dt, device="cuda:0")
        g = plan.graph(f, u)
        for _ in range(2):
            u.fill_(float("nan"))
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(u, ref), ("graph", ov)
            _ = plan.solve(f)  # eager work between replays
            torch.cuda.synchronize()
        g.close()
    plan.close()
