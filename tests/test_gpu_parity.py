"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by
element, on seeded inputs.

Tolerances (relative L-infinity, max|u - u_ref| / max|u_ref|):
  * FP64 solve vs oracle B (same FLGF operator, different rounding order):
    max(1e-12, Lambda_p^3 eps_64).  Both sides evaluate the same linear operator in
    FP64; rounding differences of node values are amplified by up to the Lebesgue
    constant Lambda_p^3 of p equispaced nodes in 3D (Sec. 2.5, Eq. leb: the paper's
    own bound Lambda^3 eps = 1.25e-12 at n_max = 10).
  * FP64 solve vs oracle A (exact direct sum): eps_trunc + 1e-12, eps_trunc being
    the oracle-B-vs-oracle-A difference on the same input.
  * FP32 path vs oracle B and vs the device's FP64 solve: 1e-6 (the FP32 bar); vs the
    exact sum: eps_trunc + 1e-6.
  * Device LGF table vs the oracle's Bessel table: 1e-14 relative.
"""
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


def gpu_solve(L, blocks, f, n, p, levels, precision="f64"):
    plan = L.Plan(blocks, n, p, levels, precision)
    dt = torch.float64 if precision == "f64" else torch.float32
    fd = torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0", dt)
    u = plan.solve(fd)
    torch.cuda.synchronize()
    out = u.double().cpu().numpy()
    plan.close()
    return out


def test_device_green_table(L):
    _say("case: device Green's function table R=32")
    G = L.green_table(32)
    ref = olgf.bessel_table(32)
    assert np.max(np.abs(G - ref) / np.abs(ref)) < 1e-14


def test_device_far_kernel(L):
    _say("case: device far kernel A^8")
    rng = np.random.default_rng(0)
    pts = rng.uniform(-200, 200, (5000, 3))
    pts = pts[np.max(np.abs(pts), axis=1) > 8]
    got = L.far_kernel(pts)
    ref = olgf.asymptotic_values(pts, flgf.Q_FAR)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-14


CASES = [
    # (label, layout builder, n, p, levels)
    ("cube2_n8_p6_nofar", lambda r: W.cube_layout(2), 8, 6, 0),
    ("cube4_n8_p6_L2", lambda r: W.cube_layout(4), 8, 6, 2),
    ("eden30_n8_p6_full", lambda r: W.eden_layout(30, r), 8, 6, 0),
    ("eden40_n4_p3_full", lambda r: W.eden_layout(40, r), 4, 3, 0),
    ("eden40_n4_p5_full", lambda r: W.eden_layout(40, r), 4, 5, 0),
    ("eden40_n4_p7_full", lambda r: W.eden_layout(40, r), 4, 7, 0),
    ("cube4_n16_p8_full", lambda r: W.cube_layout(4), 16, 8, 0),
    ("eden20_n16_p10_full", lambda r: W.eden_layout(20, r), 16, 10, 0),
    ("eden30_n8_p9_L1_lattice", lambda r: W.eden_layout(30, r), 8, 9, 1),
    ("cube5_n4_p2_L2_truncated", lambda r: W.cube_layout(5), 4, 2, 2),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_solve_fp64_matches_oracle(L, case):
    label, mk, n, p, levels = case
    rng = np.random.default_rng(zlib.crc32(label.encode()))
    blocks = mk(rng)
    f = rng.standard_normal((len(blocks), n, n, n))
    _say("case:", label, "blocks", len(blocks))
    ref = flgf.solve(blocks, f, n, p, levels)
    got = gpu_solve(L, blocks, f, n, p, levels)
    e = rel(got, ref)
    _say("   rel Linf vs oracle B = %.3e (tol %.1e)" % (e, fp64_tol(p)))
    assert e < fp64_tol(p)


def test_small_config_against_exact(L):
    c = W.config_small()
    _say("case: 32^3 cube, n=8 p=6 2 levels, 4 Gaussians vs exact direct sum")
    ref_b = flgf.solve(c["blocks"], c["f"], c["n"], c["p"], c["levels"])
    P = W.points_of(c["blocks"], c["n"]).reshape(-1, 3)
    ref_a = olgf.direct_sum(P, c["f"].reshape(-1), P).reshape(c["f"].shape)
    got = gpu_solve(L, c["blocks"], c["f"], c["n"], c["p"], c["levels"])
    eps_trunc = rel(ref_b, ref_a)
    eb, ea = rel(got, ref_b), rel(got, ref_a)
    _say("   vs B %.3e  vs A %.3e  eps_trunc %.3e" % (eb, ea, eps_trunc))
    assert eb < 1e-12
    assert ea < eps_trunc + 1e-12


def test_medium_config_full_size(L):
    # the 128^3 workload at full size, every point against oracle B
    c = W.config_medium()
    _say("case: 128^3 cube, n=16 p=8 4 levels, 32 zero-net Gaussians, FP64 vs oracle B (all points)")
    ref = flgf.solve(c["blocks"], c["f"], c["n"], c["p"], c["levels"])
    got = gpu_solve(L, c["blocks"], c["f"], c["n"], c["p"], c["levels"])
    e = rel(got, ref)
    _say("   rel Linf vs oracle B = %.3e" % e)
    assert e < 1e-12


FP32_CASES = [
    ("cube4_n8_p6_L2", lambda r: W.cube_layout(4), 8, 6, 2),
    ("eden60_n16_p8_full", lambda r: W.eden_layout(60, r), 16, 8, 0),
    ("eden40_n8_p9_lattice", lambda r: W.eden_layout(40, r), 8, 9, 0),
]


@pytest.mark.parametrize("case", FP32_CASES, ids=[c[0] for c in FP32_CASES])
def test_fp32_path_within_1e6_of_fp64(L, case):
    # FP32 transforms and products, float-float down pass, FP64 tables and final add:
    # max|u32 - u64| / max|u64| <= 1e-6 on smooth (Gaussian) sources
    label, mk, n, p, levels = case
    rng = np.random.default_rng(zlib.crc32(label.encode()))
    blocks = mk(rng)
    f, _ = W.zero_mean_gaussians(blocks, n, rng, max(4, len(blocks) // 8))
    _say("case: FP32", label, "blocks", len(blocks))
    u64 = gpu_solve(L, blocks, f, n, p, levels, "f64")
    u32 = gpu_solve(L, blocks, f, n, p, levels, "f32")
    e = rel(u32, u64)
    _say("   FP32 vs FP64 rel Linf = %.3e" % e)
    assert e < FP32_BAR


def test_medium_config_fp32(L):
    """The 128^3 workload on the FP32 path over the whole field: against the oracle's FLGF
    (FP64, the same operator) and against the device's FP64 solve, both within 1e-6 of
    max|u|."""
    c = W.config_medium()
    _say("case: 128^3 workload FP32 vs oracle FLGF and vs FP64 (all points)")
    ref = flgf.solve(c["blocks"], c["f"], c["n"], c["p"], c["levels"])
    u64 = gpu_solve(L, c["blocks"], c["f"], c["n"], c["p"], c["levels"], "f64")
    u32 = gpu_solve(L, c["blocks"], c["f"], c["n"], c["p"], c["levels"], "f32")
    e_or, e64 = rel(u32, ref), rel(u32, u64)
    _say("   FP32 vs oracle FLGF rel Linf = %.3e, vs FP64 = %.3e" % (e_or, e64))
    assert e_or <= FP32_BAR
    assert e64 <= FP32_BAR


def test_deterministic(L):
    # no atomics and a fixed summation order: two solves are bitwise equal
    rng = np.random.default_rng(9)
    blocks = W.eden_layout(50, rng)
    f = rng.standard_normal((len(blocks), 16, 16, 16))
    for prec in ("f64", "f32"):
        a = gpu_solve(L, blocks, f, 16, 8, 0, prec)
        b = gpu_solve(L, blocks, f, 16, 8, 0, prec)
        assert np.array_equal(a, b), prec


def test_large_config_vortex_ring(L):
    """256^3 vortex-ring workload (16^3 blocks of 16^3, p = 8, full depth) at full size:
    FP64 against the oracle's FLGF and exact direct sum at 64 stored targets
    (tests/golden/large_config_samples.json, written by make_large_samples.py from the
    oracle alone); the FP32 path against FP64 over the whole field and against the oracle's
    FLGF and exact sum at the same targets."""
    import json
    import os
    _say("case: large config 256^3 vortex ring, FP64 + FP32")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "large_config_samples.json")))
    c = W.config_large()
    assert gold["workload"] == c["name"]
    idx = np.asarray(gold["flat_index"])
    u64 = gpu_solve(L, c["blocks"], c["f"], c["n"], c["p"], c["levels"], "f64").reshape(-1)
    scale = gold["max_abs_u"]
    assert abs(np.max(np.abs(u64)) - scale) <= 1e-12 * scale
    flgf_ref = np.asarray(gold["flgf"])
    exact = np.asarray(gold["exact"])
    err_b = float(np.max(np.abs(u64[idx] - flgf_ref)) / scale)
    trunc = float(np.max(np.abs(flgf_ref - exact)) / np.max(np.abs(exact)))
    err_a = float(np.max(np.abs(u64[idx] - exact)) / np.max(np.abs(exact)))
    _say("  vs oracle FLGF %.3g, vs exact %.3g (oracle FLGF vs exact %.3g)" % (err_b, err_a, trunc))
    assert err_b <= fp64_tol(c["p"])
    assert err_a <= trunc + 1e-12
    u32 = gpu_solve(L, c["blocks"], c["f"], c["n"], c["p"], c["levels"], "f32").reshape(-1)
    err32 = float(np.max(np.abs(u32 - u64)) / np.max(np.abs(u64)))
    # the FP32 path against the oracle: its FLGF, and the exact sum within the truncation
    err32_b = float(np.max(np.abs(u32[idx] - flgf_ref)) / scale)
    err32_a = float(np.max(np.abs(u32[idx] - exact)) / np.max(np.abs(exact)))
    _say("  FP32 vs FP64 %.3g; at the stored targets vs oracle FLGF %.3g, vs exact %.3g" % (err32, err32_b, err32_a))
    assert err32 <= FP32_BAR
    assert err32_b <= FP32_BAR
    assert err32_a <= trunc + FP32_BAR


def test_medium_config_tuned_graph(L):
    """The 128^3 workload in the launch configuration the benchmark times: autotuned kernel
    variants, then one graph per schedule (three branches, two, one stream), as the
    benchmark builds them, each replayed with eager solves in between.  Every replay equals
    the eager solve bit for bit; FP64 against the oracle's FLGF at full size, FP32 against
    the oracle and FP64 within 1e-6."""
    _say("case: medium config, autotuned variants, graphs of every schedule, FP64 + FP32")
    c = W.config_medium()
    ref = flgf.solve(c["blocks"], c["f"], c["n"], c["p"], c["levels"])
    out = {}
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        plan = L.Plan(c["blocks"], c["n"], c["p"], c["levels"], prec)
        f = torch.from_numpy(c["f"]).to("cuda:0", dt)
        u = torch.empty_like(f)
        choice = plan.autotune(f, u, reps=2)
        eager = plan.solve(f).clone()
        torch.cuda.synchronize()
        for ov in (1, 3, 2):
            _say("   %s schedule %d" % (prec, ov))
            plan.set_tuning(**dict(choice, overlap=ov))
            g = plan.graph(f, u)
            for _ in range(3):
                u.fill_(float("nan"))
                g.launch()
                torch.cuda.synchronize()
                assert torch.equal(u, eager), (prec, ov)
                plan.solve(f)  # eager work between the replays
                torch.cuda.synchronize()
            g.close()
        out[prec] = u.double().cpu().numpy()
        plan.close()
    assert rel(out["f64"], ref) <= fp64_tol(c["p"])
    assert rel(out["f32"], ref) <= FP32_BAR
    assert rel(out["f32"], out["f64"]) <= FP32_BAR
