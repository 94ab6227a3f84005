"""GPU parity of the screened operator L - kappa (lgf_plan_create_screened), a second
non-oscillatory lattice kernel (Sec. 5), against the oracle: the device's integrated
G_kappa table, FP64 solves against the oracle's FLGF with the same kernel (element by
element, max(1e-12, Lambda^3 eps_64)) and against the exact direct sum (truncation
+ 1e-12), a manufactured solution, the FP32 path (1e-6), graphs and symmetry-reduced
spectra with the screened kernel, and the argument checks."""
import sys
import zlib

import numpy as np
import pytest
import torch

from oracle import flgf, lgf as olgf
from paper_1402_6081_amd import workloads as W
from tolerances import FP32_BAR, fp64_tol, rel
from test_oracle_screened import _manufactured

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


def gpu_solve(L, blocks, f, n, p, levels, kappa, precision="f64", spectra=None):
    plan = L.Plan(blocks, n, p, levels, precision, kappa=kappa, spectra=spectra)
    dt = torch.float64 if precision == "f64" else torch.float32
    u = plan.solve(torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0", dt))
    torch.cuda.synchronize()
    info = plan.info()
    plan.close()
    assert info["kappa"] == kappa
    return u.double().cpu().numpy()


@pytest.mark.parametrize("kappa", [0.25, 1.0, 4.0])
def test_device_screened_table(L, kappa):
    _say("case: device screened LGF table, kappa", kappa)
    G = L.green_table_screened(24, kappa)
    ref = olgf.screened_table(24, kappa)
    # relative 1e-14; values decay by tens of orders of magnitude across the table, and
    # those far below G(0) carry each quadrature's own relative rounding, so they are held
    # to an absolute 1e-17 of |G(0)| (far below anything a convolution with them can feel)
    err = np.abs(G - ref)
    assert np.all(err <= 1e-14 * np.abs(ref) + 1e-17 * abs(ref[0, 0, 0]))
    big = np.abs(ref) > 1e-12 * abs(ref[0, 0, 0])
    assert np.max(err[big] / np.abs(ref[big])) < 1e-14


CASES = [
    # label, layout, n, p, levels, kappa
    ("cube2_n8_p9_k1_nofar", lambda r: W.cube_layout(2), 8, 9, 0, 1.0),
    ("eden30_n8_p9_k05_full", lambda r: W.eden_layout(30, r), 8, 9, 0, 0.5),
    ("eden40_n8_p5_k1_full", lambda r: W.eden_layout(40, r), 8, 5, 0, 1.0),
    ("eden40_n4_p3_k03_full", lambda r: W.eden_layout(40, r), 4, 3, 0, 0.3),
    ("cube5_n4_p5_k2_L2_truncated", lambda r: W.cube_layout(5), 4, 5, 2, 2.0),
    ("eden24_n16_p17_k1_full", lambda r: W.eden_layout(24, r), 16, 17, 0, 1.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_screened_fp64_matches_oracle(L, case):
    label, mk, n, p, levels, kappa = case
    rng = np.random.default_rng(zlib.crc32(label.encode()))
    blocks = mk(rng)
    f = rng.standard_normal((len(blocks), n, n, n))
    _say("case:", label, "blocks", len(blocks))
    ref = flgf.solve(blocks, f, n, p, levels, kappa=kappa)
    got = gpu_solve(L, blocks, f, n, p, levels, kappa)
    e = rel(got, ref)
    _say("   rel Linf vs oracle FLGF = %.3e (tol %.1e)" % (e, fp64_tol(p)))
    assert e < fp64_tol(p)


def test_screened_against_exact_and_fp32(L):
    """A smooth source on a 60-block layout (n = 8, p = 9, kappa = 0.5): FP64 against the
    exact direct sum within the oracle's truncation + 1e-12; FP32 against FP64 and the
    oracle's FLGF within 1e-6."""
    kappa, n, p = 0.5, 8, 9
    rng = np.random.default_rng(81)
    blocks = W.eden_layout(60, rng)
    f, _ = W.zero_mean_gaussians(blocks, n, rng, 8)
    _say("case: screened 60 blocks, exact sum and FP32")
    ref = flgf.solve(blocks, f, n, p, 0, kappa=kappa)
    P = W.points_of(blocks, n).reshape(-1, 3)
    exact = olgf.direct_sum(P, f.reshape(-1), P, kappa).reshape(f.shape)
    u64 = gpu_solve(L, blocks, f, n, p, 0, kappa)
    u32 = gpu_solve(L, blocks, f, n, p, 0, kappa, "f32")
    trunc = rel(ref, exact)
    _say("   FP64 vs oracle FLGF %.3e, vs exact %.3e (truncation %.3e); FP32 vs FP64 %.3e, vs oracle %.3e"
         % (rel(u64, ref), rel(u64, exact), trunc, rel(u32, u64), rel(u32, ref)))
    assert rel(u64, ref) < fp64_tol(p)
    assert rel(u64, exact) <= trunc + 1e-12
    assert rel(u32, u64) <= FP32_BAR
    assert rel(u32, ref) <= FP32_BAR


def test_screened_manufactured_solution(L):
    """u_rand (zero on the boundary points) and f = (L - kappa) u_rand: G_kappa * f = u_rand
    exactly, so the device's error is the method's, as the oracle's FLGF measures it."""
    kappa, n, p = 0.6, 8, 9
    rng = np.random.default_rng(82)
    blocks = W.eden_layout(30, rng)
    u, f = _manufactured(blocks, n, kappa, rng)
    _say("case: screened manufactured solution")
    ref = flgf.solve(blocks, f, n, p, 0, kappa=kappa)
    got = gpu_solve(L, blocks, f, n, p, 0, kappa)
    eps = float(np.max(np.abs(ref - u)))
    err = float(np.max(np.abs(got - u)))
    _say("   oracle error %.3e, device error %.3e" % (eps, err))
    assert eps < 1e-6
    assert err <= eps + 1e-12


def test_kappa_zero_is_the_laplace_plan(L):
    rng = np.random.default_rng(83)
    blocks = W.eden_layout(40, rng)
    f = rng.standard_normal((len(blocks), 8, 8, 8))
    a = gpu_solve(L, blocks, f, 8, 6, 0, 0.0)
    plan = L.Plan(blocks, 8, 6, 0, "f64")
    b = plan.solve(torch.from_numpy(f).to("cuda:0")).cpu().numpy()
    plan.close()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_screened_graph_and_reduced_spectra(L, prec):
    """A screened plan launched as a graph equals its eager solve bit for bit; with
    symmetry-reduced spectra (G_kappa has the 48-fold symmetry too) it equals the full
    tables within their generation rounding."""
    kappa, n, p = 2.0, 8, 9
    rng = np.random.default_rng(84)
    blocks = W.eden_layout(50, rng)
    dt = torch.float64 if prec == "f64" else torch.float32
    f = torch.from_numpy(rng.standard_normal((len(blocks), n, n, n))).to("cuda:0", dt)
    plan = L.Plan(blocks, n, p, 0, prec, kappa=kappa)
    eager = plan.solve(f).clone()
    u = torch.empty_like(f)
    g = plan.graph(f, u)
    for _ in range(3):
        u.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(u, eager)
    g.close()
    plan.close()
    red = L.Plan(blocks, n, p, 0, prec, kappa=kappa, spectra="reduced")
    ur = red.solve(f)
    torch.cuda.synchronize()
    red.close()
    d = rel(ur.double().cpu().numpy(), eager.double().cpu().numpy())
    _say("   %s reduced vs full spectra %.3e" % (prec, d))
    assert d < (1e-13 if prec == "f64" else 1e-6)


def test_screened_argument_errors(L):
    blocks = W.cube_layout(2)
    for n, p, kappa in ((8, 6, 1.0), (8, 8, 1.0), (8, 9, 1e-4), (8, 9, -1.0), (16, 10, 1.0)):
        with pytest.raises(L.LGFError) as e:
            L.Plan(blocks, n, p, 0, "f64", kappa=kappa)
        assert e.value.name == "LGF_ERR_ARG", (n, p, kappa)
    with pytest.raises(L.LGFError):
        L.green_table_screened(8, 1e-5)
