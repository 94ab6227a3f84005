"""GPU tests of the request server (lgf_server_*): results in a concurrent mix equal the
results of the same requests solved alone and the oracle's, solves ordered after the
submitter's stream, admission under an HBM budget, queue limits."""
import sys

import numpy as np
import pytest
import torch

from oracle import flgf
from paper_1402_6081_amd import workloads as W
from tolerances import FP32_BAR, rel

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


def _alone(L, blocks, f, n, p, prec):
    plan = L.Plan(blocks, n, p, 0, prec)
    u = plan.solve(f)
    torch.cuda.synchronize()
    plan.close()
    return u


def _mix(seed, count, lo, hi, repeat_every=4):
    """Layouts with repeats (plan reuse, and concurrent requests of one layout)."""
    rng = np.random.default_rng(seed)
    base = [W.eden_layout(int(s), rng) for s in rng.integers(lo, hi, size=count)]
    lays = []
    for i in range(count):
        lays.append(base[i])
        if i % repeat_every == 0:
            lays.append(base[i])
            lays.append(base[i])
    return lays, rng


@pytest.mark.parametrize("prec,slots", [("f32", 4), ("f64", 3), ("f32", 1)])
def test_server_results_equal_alone(L, prec, slots):
    _say("case: server mix", prec, "slots", slots)
    n, p = 8, 6
    lays, rng = _mix(21 + slots, 10, 4, 160)
    dt = torch.float64 if prec == "f64" else torch.float32
    fs = [torch.from_numpy(rng.standard_normal((b.shape[0], n, n, n))).to("cuda:0", dt) for b in lays]
    refs = [_alone(L, b, f, n, p, prec) for b, f in zip(lays, fs)]
    srv = L.Server(n, p, 0, prec, max_slots=slots)
    us = [torch.full_like(f, float("nan")) for f in fs]
    tickets = [srv.submit(b, f, u) for b, f, u in zip(lays, fs, us)]
    res = [srv.wait(t) for t in tickets]
    for i, (r, u, ref) in enumerate(zip(res, us, refs)):
        assert r["status"] == "LGF_OK", (i, r)
        assert torch.equal(u, ref), "request %d differs from its solve alone" % i
        assert r["latency_ms"] >= r["queue_ms"] >= 0.0 and r["device_ms"] > 0.0
    st = srv.stats()
    assert st["completed"] == len(lays) and st["failed"] == 0
    assert st["plans_created"] <= len(lays)
    assert 0 < st["latency_p50_ms"] <= st["latency_p99_ms"] <= st["latency_max_ms"]
    assert st["points"] == sum(b.shape[0] for b in lays) * n ** 3
    srv.close()


def test_server_budget_admission(L):
    _say("case: server budget admission and eviction")
    n, p, prec = 8, 6, "f32"
    rng = np.random.default_rng(33)
    lays = [W.eden_layout(int(s), rng) for s in (120, 90, 150, 60, 130, 100)]
    fs = [torch.from_numpy(rng.standard_normal((b.shape[0], n, n, n))).to("cuda:0", torch.float32)
          for b in lays]
    refs = [_alone(L, b, f, n, p, prec) for b, f in zip(lays, fs)]  # also caches every spectrum
    ests = [L.plan_estimate(b, n, p, 0, prec)["workspace_bytes"] for b in lays]
    probe = L.Server(n, p, 0, prec, max_slots=1)
    spectra = probe.stats()["spectra_bytes"]
    probe.close()
    budget = spectra + int(2.2 * max(ests))  # at most two plans resident at once
    srv = L.Server(n, p, 0, prec, max_slots=4, budget_bytes=budget)
    us = [torch.full_like(f, float("nan")) for f in fs]
    tickets = [srv.submit(b, f, u) for b, f, u in zip(lays, fs, us)]
    res = [srv.wait(t) for t in tickets]
    for r, u, ref in zip(res, us, refs):
        assert r["status"] == "LGF_OK"
        assert torch.equal(u, ref)
    st = srv.stats()
    nlay = len(lays)
    # every plan was created once and all but the resident ones were evicted again
    assert st["plans_created"] == nlay and st["plans_evicted"] >= 1
    resident = st["plans_created"] - st["plans_evicted"]
    assert resident * min(ests) <= st["plan_bytes"] <= budget - st["spectra_bytes"]
    # a request that cannot fit on its own is refused; the server keeps serving
    big = W.cube_layout(12)
    fb = torch.zeros((big.shape[0], n, n, n), dtype=torch.float32, device="cuda:0")
    ub = torch.empty_like(fb)
    t_big = srv.submit(big, fb, ub)
    t_ok = srv.submit(lays[0], fs[0], us[0])
    assert srv.wait(t_big)["status"] == "LGF_ERR_BUDGET"
    assert srv.wait(t_ok)["status"] == "LGF_OK"
    assert torch.equal(us[0], refs[0])
    srv.close()


def test_server_queue_limit(L):
    _say("case: server queue limit")
    n, p = 8, 6
    rng = np.random.default_rng(44)
    b = W.eden_layout(200, rng)
    f = torch.from_numpy(rng.standard_normal((b.shape[0], n, n, n))).to("cuda:0", torch.float32)
    ref = _alone(L, b, f, n, p, "f32")
    srv = L.Server(n, p, 0, "f32", max_slots=1, max_queue=2)
    us, tickets, busy = [], [], 0
    for _ in range(40):
        u = torch.empty_like(f)
        try:
            tickets.append(srv.submit(b, f, u))
            us.append(u)
        except L.LGFError as e:
            assert e.name == "LGF_ERR_BUSY"
            busy += 1
    assert busy > 0
    for t, u in zip(tickets, us):
        assert srv.wait(t)["status"] == "LGF_OK"
        assert torch.equal(u, ref)
    srv.close()


def test_server_poll_and_layout_error(L):
    _say("case: server poll and a bad layout")
    srv = L.Server(8, 6, 0, "f32", max_slots=2)
    dup = np.array([[0, 0, 0], [0, 0, 0]], dtype=np.int32)
    f = torch.zeros((2, 8, 8, 8), dtype=torch.float32, device="cuda:0")
    u = torch.empty_like(f)
    t = srv.submit(dup, f, u)
    r = None
    for _ in range(200000):
        r = srv.poll(t)
        if r is not None:
            break
    if r is None:
        r = srv.wait(t)
    assert r["status"] == "LGF_ERR_LAYOUT"
    with pytest.raises(L.LGFError):
        srv.poll(t)  # released
    srv.close()


def test_server_serving_config_mix_against_oracle(L):
    """The serving configuration: n = 16, p = 8, FP32, 4 slots; Eden-box layouts with
    bounding-box edges U{2..8} blocks and fill U[0.3, 1], zero-net Gaussian sources as in
    the benchmark's request mix, submitted all at once with repeats (concurrent requests of
    one layout, plan reuse).  Every result equals the same request solved alone, bit for
    bit, and the oracle's FLGF within 1e-6 of max|u|."""
    _say("case: server serving-config mix, n=16 p=8 FP32, 4 slots")
    n, p = 16, 8
    rng = np.random.default_rng(55)
    base = []
    for _ in range(7):
        b = W.eden_box_layout(int(rng.integers(2, 9)), float(rng.uniform(0.3, 1.0)), rng)
        f, _ = W.zero_mean_gaussians(b, n, rng, max(1, b.shape[0] // 8))
        base.append((b, f))
    order = [0, 1, 2, 0, 3, 4, 1, 5, 6, 2, 0]
    dev = torch.device("cuda:0")
    fs = [torch.from_numpy(f).to(dev, torch.float32) for _, f in base]
    alone = [_alone(L, b, f, n, p, "f32") for (b, _), f in zip(base, fs)]
    srv = L.Server(n, p, 0, "f32", max_slots=4)
    us = [torch.full_like(fs[k], float("nan")) for k in order]
    tickets = [srv.submit(base[k][0], fs[k], u) for k, u in zip(order, us)]
    res = [srv.wait(t) for t in tickets]
    for i, (k, r, u) in enumerate(zip(order, res, us)):
        assert r["status"] == "LGF_OK", (i, r)
        assert torch.equal(u, alone[k]), "request %d (layout %d) differs from its solve alone" % (i, k)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(order) and st["failed"] == 0
    for k, (b, f) in enumerate(base):
        ref = flgf.solve(b, f, n, p, 0)
        e = rel(alone[k].double().cpu().numpy(), ref)
        _say("   layout %d: %d blocks, FP32 vs oracle FLGF rel Linf = %.3e" % (k, b.shape[0], e))
        assert e <= FP32_BAR


def test_server_waits_for_submit_stream(L):
    """A request's solve starts only after the work its submitter queued on its stream:
    the source field is written on a side stream behind a bounded spin and submitted at
    once with that stream; the result equals the solve of the finished field."""
    _say("case: server ordering after the submitter's stream")
    n, p = 8, 6
    rng = np.random.default_rng(66)
    b = W.eden_layout(90, rng)
    f_host = torch.from_numpy(rng.standard_normal((b.shape[0], n, n, n))).to(torch.float32)
    f_ok = f_host.to("cuda:0")
    ref = _alone(L, b, f_ok, n, p, "f32")
    srv = L.Server(n, p, 0, "f32", max_slots=2)
    side = torch.cuda.Stream()
    f = torch.zeros_like(f_ok)
    u = torch.full_like(f_ok, float("nan"))
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        torch.cuda._sleep(50_000_000)  # bounded spin (tens of milliseconds)
        f.copy_(f_ok)
        t = srv.submit(b, f, u, stream=side)
    r = srv.wait(t)
    assert r["status"] == "LGF_OK"
    assert torch.equal(u, ref)
    srv.close()
