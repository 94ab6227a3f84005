"""The 128^3 workload in the launch configuration the benchmark times: autotuned kernel
variants and schedule (lgf_plan_autotune, which times eager solves), then one HIP-graph
launch per solve, replayed with eager work between the replays.  FP64 against the oracle's
FLGF at full size within 1e-12; FP32 against FP64 within 1e-6.  Collected last, so that a
failure here cannot hide another test."""
import sys

import numpy as np
import pytest
import torch

from oracle import flgf
from paper_1402_6081_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_medium_config_bench_launch_configuration():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_1402_6081_amd.lgf as L
    L.library()
    _say("case: medium config, autotuned variants, graph launches, FP64 + FP32")
    c = W.config_medium()
    ref = flgf.solve(c["blocks"], c["f"], c["n"], c["p"], c["levels"])
    out = {}
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        plan = L.Plan(c["blocks"], c["n"], c["p"], c["levels"], prec)
        f = torch.from_numpy(c["f"]).to("cuda:0", dt)
        u = torch.empty_like(f)
        choice = plan.autotune(f, u, reps=2)
        _say("   %s tuning %s" % (prec, choice))
        eager = plan.solve(f).clone()
        g = plan.graph(f, u)
        for _ in range(3):
            u.fill_(float("nan"))
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(u, eager)
            plan.solve(f)  # eager work between the replays
            torch.cuda.synchronize()
        out[prec] = u.double().cpu().numpy()
        g.close()
        plan.close()
    e64 = float(np.max(np.abs(out["f64"] - ref)) / np.max(np.abs(ref)))
    e32 = float(np.max(np.abs(out["f32"] - out["f64"])) / np.max(np.abs(out["f64"])))
    _say("   FP64 vs oracle %.3e, FP32 vs FP64 %.3e" % (e64, e32))
    assert e64 <= 1e-12
    assert e32 <= 1e-6
