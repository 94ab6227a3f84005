"""GPU tests of batched solves, HIP-graph replay and the kernel-variant autotuner.

A batch plan is the union of independent per-layout trees, so every problem of a
batch must come out exactly as it does from its own plan: the per-target summation
orders of all kernels are the same in both.  The comparison is therefore bitwise,
and one member of each batch is also checked against the oracle.
"""
import sys
import zlib

import numpy as np
import pytest
import torch

from oracle import flgf
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


def _layouts(seed, sizes):
    rng = np.random.default_rng(seed)
    out = []
    for s in sizes:
        if s == "cube2":
            out.append(W.cube_layout(2))
        else:
            out.append(W.eden_layout(int(s), rng))
    return out


def _fields(layouts, n, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((b.shape[0], n, n, n)) for b in layouts]


BATCHES = [
    # label, sizes, n, p, levels, precision
    ("mixed_n8_p6_full_f64", [40, 1, 9, "cube2", 120, 3], 8, 6, 0, "f64"),
    ("mixed_n8_p6_full_f32", [40, 1, 9, "cube2", 120, 3], 8, 6, 0, "f32"),
    ("mixed_n4_p5_L2_f64", [60, 7, "cube2", 25], 4, 5, 2, "f64"),
    ("mixed_n8_p9_L3_f64", [90, 2, 30], 8, 9, 3, "f64"),
    ("many_n4_p3_full_f32", [3, 5, 8, 13, 21, 34, 55, 89, 1, 2], 4, 3, 0, "f32"),
]


@pytest.mark.parametrize("case", BATCHES, ids=[c[0] for c in BATCHES])
def test_batch_equals_individual_solves(L, case):
    label, sizes, n, p, levels, prec = case
    seed = zlib.crc32(label.encode())
    _say("case: batch", label, "seed", seed)
    lays = _layouts(seed, sizes)
    fs = _fields(lays, n, seed + 1)
    dt = torch.float64 if prec == "f64" else torch.float32
    bp = L.Plan.batch(lays, n, p, levels, prec)
    assert bp.offsets == list(np.concatenate([[0], np.cumsum([b.shape[0] for b in lays])]))
    fb = torch.from_numpy(np.concatenate(fs)).to("cuda:0", dt)
    ub = bp.solve(fb)
    torch.cuda.synchronize()
    parts = [x.double().cpu().numpy() for x in bp.split(ub)]
    for i, (b, f) in enumerate(zip(lays, fs)):
        pl = L.Plan(b, n, p, levels, prec)
        ui = pl.solve(torch.from_numpy(f).to("cuda:0", dt))
        torch.cuda.synchronize()
        ui = ui.double().cpu().numpy()
        pl.close()
        assert np.array_equal(parts[i], ui), "problem %d (%d blocks) differs: %g" % (
            i, b.shape[0], np.max(np.abs(parts[i] - ui)))
    bp.close()
    # the largest member against the oracle (FP64 batches)
    if prec == "f64":
        k = int(np.argmax([b.shape[0] for b in lays]))
        ref = flgf.solve(lays[k], fs[k], n, p, levels)
        e = rel(parts[k], ref)
        _say("   largest member vs oracle FLGF %.3e (tol %.1e)" % (e, fp64_tol(p)))
        assert e < fp64_tol(p)


def test_batch_info_sums_members(L):
    _say("case: batch plan summary")
    lays = _layouts(7, [30, 12, 5])
    bp = L.Plan.batch(lays, 8, 6, 0, "f64")
    inf = bp.info()
    near = far1 = 0
    for b in lays:
        pl = L.Plan(b, 8, 6, 0, "f64")
        i = pl.info()
        near += i["near_pairs"]
        far1 += i["far_pairs"][1]
        pl.close()
    assert inf["nblocks"] == sum(b.shape[0] for b in lays)
    assert inf["near_pairs"] == near
    assert inf["far_pairs"][1] == far1
    bp.close()


GRAPH_CASES = [
    ("eden60_n8_p6_f64", 60, 8, 6, "f64"),       # small plan: far chain on the second stream
    ("eden400_n8_p6_f32", 400, 8, 6, "f32"),     # large plan: single stream
    ("eden300_n4_p5_L2_f64", 300, 4, 5, "f64"),  # truncated top level (CSR Prod)
]


@pytest.mark.parametrize("case", GRAPH_CASES, ids=[c[0] for c in GRAPH_CASES])
def test_graph_replays_match_eager(L, case):
    label, nb, n, p, prec = case
    levels = 2 if "_L2" in label else 0
    seed = zlib.crc32(label.encode())
    _say("case: graph", label, "seed", seed)
    rng = np.random.default_rng(seed)
    blocks = W.eden_layout(nb, rng)
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = L.Plan(blocks, n, p, levels, prec)
    f = torch.zeros(plan.shape(), dtype=dt, device="cuda:0")
    u = torch.zeros_like(f)
    schedule = {"f64": 1, "f32": 3}[prec] if "_L2" not in label else 2
    plan.set_tuning(overlap=schedule)
    g = plan.graph(f, u)
    plan.set_tuning()  # eager solves below use the default schedule: results must not depend on it
    for r in range(4):
        fr = torch.from_numpy(rng.standard_normal(plan.shape())).to("cuda:0", dt)
        f.copy_(fr)
        u.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        got = u.clone()
        # eager work between replays: an unrelated reduction and an eager solve
        junk = torch.randn(1 << 20, device="cuda:0").sum().item()
        assert np.isfinite(junk)
        ref = plan.solve(fr)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), "replay %d differs" % r
    g.close()
    plan.close()


def test_batch_graph(L):
    _say("case: graph of a batch plan")
    lays = _layouts(11, [50, 4, 17])
    fs = _fields(lays, 8, 12)
    bp = L.Plan.batch(lays, 8, 6, 0, "f32")
    f = torch.from_numpy(np.concatenate(fs)).to("cuda:0", torch.float32)
    u = torch.empty_like(f)
    g = bp.graph(f, u)
    for _ in range(3):
        u.zero_()
        g.launch()
        torch.cuda.synchronize()
        ref = bp.solve(f)
        torch.cuda.synchronize()
        assert torch.equal(u, ref)
    g.close()
    bp.close()


def test_autotune_keeps_results(L):
    _say("case: autotune eden200 n8 p8 f32")
    rng = np.random.default_rng(5)
    blocks = W.eden_layout(200, rng)
    plan = L.Plan(blocks, 8, 8, 0, "f32")
    f = torch.from_numpy(rng.standard_normal(plan.shape())).to("cuda:0", torch.float32)
    before = plan.solve(f)
    torch.cuda.synchronize()
    choice = plan.autotune(f, reps=2)
    assert choice["fft0_threads"] in (0, 128, 256, 512)
    assert choice["near_waves"] in (2, 4, 8)
    assert choice["far_waves"] in (0, 1, 2, 4, 8, 16)
    assert choice["far_children"] in (0, 1, 2, 4, 8)
    assert choice["overlap"] in (0, 1, 2, 3)
    assert choice["near_prefetch"] in (0, 1)
    after = plan.solve(f)
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    # a new plan of the same shape class picks the remembered choice
    plan2 = L.Plan(blocks, 8, 8, 0, "f32")
    assert plan2.tuning() == choice
    plan2.close()
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_every_variant_same_bits(L, prec):
    """All kernel variants the autotuner chooses among give identical results."""
    rng = np.random.default_rng(9)
    blocks = W.eden_layout(150, rng)
    for n in (8, 16):
        _say("case: kernel variants", prec, "n", n)
        plan = L.Plan(blocks, n, 6, 0, prec)
        f = torch.from_numpy(rng.standard_normal(plan.shape())).to("cuda:0", plan.dtype)
        plan.set_tuning(far_waves=2, far_children=8, overlap=2)
        ref = plan.solve(f)
        torch.cuda.synchronize()
        variants = [dict(fft0_threads=ft) for ft in (0, 128, 256, 512)]
        variants += [dict(near_waves=nw, near_prefetch=pf) for nw in (2, 4, 8) for pf in (0, 1)]
        variants += [dict(far_waves=fw, far_children=fc) for fw in (0, 1, 2, 4, 8, 16) for fc in (0, 1, 2, 4, 8)]
        variants += [dict(overlap=ov) for ov in (1, 2, 3)]
        for v in variants:
            plan.set_tuning(**v)
            got = plan.solve(f)
            torch.cuda.synchronize()
            assert torch.equal(ref, got), v
        with pytest.raises(L.LGFError):
            plan.set_tuning(fft0_threads=64)
        plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_wide_m2l_lists_same_bits(L, prec, monkeypatch):
    """The M2L's 32-bit source-list entries, which levels of 65535 or more items take
    (forced here at a small size by LGF_M2L_WIDE_LISTS=1), give the bits of the 16-bit
    entries in every M2L variant and schedule."""
    rng = np.random.default_rng(19)
    blocks = W.eden_layout(150, rng)
    _say("case: wide M2L lists", prec)
    plan = L.Plan(blocks, 8, 6, 0, prec)
    f = torch.from_numpy(rng.standard_normal(plan.shape())).to("cuda:0", plan.dtype)
    variants = [dict(far_waves=fw, far_children=fc, overlap=2) for fw in (0, 1, 4, 16) for fc in (0, 1, 8)]
    variants += [dict(far_waves=0, far_children=0, overlap=ov) for ov in (1, 3)]
    refs = []
    for v in variants:
        plan.set_tuning(**v)
        refs.append(plan.solve(f).clone())
    monkeypatch.setenv("LGF_M2L_WIDE_LISTS", "1")
    for v, ref in zip(variants, refs):
        plan.set_tuning(**v)
        got = plan.solve(f)
        torch.cuda.synchronize()
        assert torch.equal(ref, got), v
    monkeypatch.delenv("LGF_M2L_WIDE_LISTS")
    plan.close()


def test_batch_workload_fp32_against_fp64_and_exact(L):
    """The batched workload: 64 Eden layouts of U{8..512} blocks of 16^3, p = 8, one batch
    plan.  Every solve of the FP32 batch against the FP64 batch (<= 1e-6); 4 sampled solves
    of both precisions against the oracle's FLGF over the whole layout (FP64 <= 1e-12, FP32
    <= 1e-6) and against the exact direct sum at 256 targets (<= FLGF truncation + 1e-12,
    FP32 + 1e-6)."""
    from oracle import lgf as olgf
    _say("case: 64-layout batch workload, FP32 vs FP64, 4 solves vs exact")
    rng = np.random.default_rng(4)
    sizes = rng.integers(8, 513, size=64)
    lays = [W.eden_layout(int(s), rng) for s in sizes]
    fs = [W.zero_mean_gaussians(b, 16, rng, max(1, b.shape[0] // 8))[0] for b in lays]
    out = {}
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        bp = L.Plan.batch(lays, 16, 8, 0, prec)
        u = bp.solve(torch.from_numpy(np.concatenate(fs)).to("cuda:0", dt))
        torch.cuda.synchronize()
        out[prec] = [x.double().cpu().numpy() for x in bp.split(u)]
        bp.close()
    worst = max(rel(a, b) for a, b in zip(out["f32"], out["f64"]))
    _say("  worst FP32 vs FP64 over 64 solves: %.3g" % worst)
    assert worst <= FP32_BAR
    for k in rng.choice(64, 4, replace=False):
        # the oracle's FLGF on the whole layout, and the exact sum at 256 sampled targets
        ref = flgf.solve(lays[k], fs[k], 16, 8, 0).reshape(-1)
        P = W.points_of(lays[k], 16).reshape(-1, 3)
        idx = rng.choice(P.shape[0], 256, replace=False)
        exact = olgf.direct_sum(P, fs[k].reshape(-1), P[idx])
        got = out["f64"][k].reshape(-1)
        g32 = out["f32"][k].reshape(-1)
        scale = float(np.max(np.abs(exact)))
        trunc = float(np.max(np.abs(ref[idx] - exact))) / scale
        err_a = float(np.max(np.abs(got[idx] - exact))) / scale
        err32_a = float(np.max(np.abs(g32[idx] - exact))) / scale
        _say("  solve %d (%d blocks): FP64 vs oracle FLGF %.3g, vs exact %.3g (truncation %.3g); "
             "FP32 vs oracle FLGF %.3g, vs exact %.3g"
             % (k, lays[k].shape[0], rel(got, ref), err_a, trunc, rel(g32, ref), err32_a))
        assert rel(got, ref) <= 1e-12
        assert err_a <= trunc + 1e-12
        assert rel(g32, ref) <= FP32_BAR
        assert err32_a <= trunc + FP32_BAR


def test_plan_busy_on_another_stream(L):
    """One workspace per plan: a solve on a second stream while the first stream's solve is
    still queued is refused (LGF_ERR_BUSY); the same stream, or the second stream once the
    first solve is done, is accepted.  A bounded GPU spin holds the first solve back."""
    rng = np.random.default_rng(71)
    blocks = W.eden_layout(64, rng)
    plan = L.Plan(blocks, 8, 6, 0, "f64")
    f = torch.from_numpy(rng.standard_normal((len(blocks), 8, 8, 8))).to("cuda:0")
    ref = plan.solve(f).clone()
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ua, ub = torch.empty_like(f), torch.empty_like(f)
    with torch.cuda.stream(sa):
        torch.cuda._sleep(50_000_000)  # bounded spin (tens of milliseconds)
    plan.solve(f, ua, stream=sa)
    with pytest.raises(L.LGFError) as e:
        plan.solve(f, ub, stream=sb)
    assert e.value.name == "LGF_ERR_BUSY"
    g = plan.graph(f, ub)  # graph creation synchronises its own stream only
    plan.solve(f, ua, stream=sa)  # same stream: ordered, accepted
    torch.cuda.synchronize()
    plan.solve(f, ub, stream=sb)  # idle again
    g.launch(stream=sb)
    torch.cuda.synchronize()
    assert torch.equal(ua, ref) and torch.equal(ub, ref)
    g.close()
    plan.close()


def test_nonfinite_input_check(L, monkeypatch):
    rng = np.random.default_rng(72)
    blocks = W.eden_layout(20, rng)
    plan = L.Plan(blocks, 8, 6, 0, "f32")
    f = torch.from_numpy(rng.standard_normal((len(blocks), 8, 8, 8))).to("cuda:0", torch.float32)
    good = plan.solve(f).clone()
    f[3, 1, 2, 3] = float("nan")
    monkeypatch.setenv("LGF_CHECK_FINITE", "1")
    with pytest.raises(L.LGFError) as e:
        plan.solve(f)
    assert e.value.name == "LGF_ERR_ARG"
    f[3, 1, 2, 3] = 0.0
    f2 = torch.from_numpy(rng.standard_normal((len(blocks), 8, 8, 8))).to("cuda:0", torch.float32)
    assert torch.isfinite(plan.solve(f2)).all()
    monkeypatch.delenv("LGF_CHECK_FINITE")
    plan.close()
    assert torch.isfinite(good).all()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_schedules_same_bits(L, prec):
    # a batch whose members have different depths: the union's top levels carry empty
    # lists for the shallow members (zeroed fields) and the one-stream schedules launch
    # the transforms and M2L of all levels at once; all three schedules give the same bits
    _say("case: batch schedules", prec)
    lays = _layouts(23, [60, 1, "cube2", 7, 200])
    fs = _fields(lays, 8, 24)
    bp = L.Plan.batch(lays, 8, 6, 0, prec)
    f = torch.from_numpy(np.concatenate(fs)).to("cuda:0", bp.dtype)
    bp.set_tuning(overlap=1)
    ref = bp.solve(f).clone()
    torch.cuda.synchronize()
    for ov in (2, 3):
        bp.set_tuning(overlap=ov)
        got = bp.solve(f)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), ov
    bp.close()
