"""Benchmark: grid points solved per second for u = G * f on one MI355X.

Workload (the metric's configuration, the largest single-solve one): a 256^3 cube as 16^3
blocks of 16^3 points, p = 8 interpolation nodes per interval edge, full tree depth,
sourced by a thin vortex ring (R = 80 cells, Gaussian core sigma = 4, seeded tilt).  The
headline line is the FP64 path; the FP32 path (FP32 transforms and products, FP64 tables,
level inverse transforms and final add) solves the same input beside it, with its rate,
latencies, roofline, and its error against the FP64 result and against the oracle.  An
FP32 rate whose error against FP64 exceeds the 1e-6 bar is withheld (value null,
meets_fp32_bar false).

Timing: the plan's kernel variants are autotuned first (lgf_plan_autotune, a few dozen
eager solves), the graph schedule is chosen by timing one graph of each schedule, then W
untimed warm-up solves and K timed solves bracketed by device synchronisation; the inputs
are resident in HBM before the timed region.  Two passes per precision:
  * eager lgf_solve calls on one stream with every step bracketed by HIP events
    (lgf_profile_*): isolated per-kernel device times (the roofline entry uses the
    dominant one);
  * the tuned solve captured once as a HIP graph (lgf_graph_create) and launched K times:
    the reported rate (value) and per-solve latencies (p50/p99, events around each launch).
Further legs: the 128^3 workload (8^3 blocks, p = 8, 4 levels, 32 Gaussians), the batched
workload (64 Eden layouts in one batch plan), the request server (closed loop for
capacity, then Poisson arrivals at 80% of it for p50/p99 latency), separate source and
evaluation sets, the paper's n_I = n + 1 scheme and symmetry-reduced kernel spectra.

cpu_baseline: the oracle timed on the host: the exact direct sum (Eq. dpoissonsoln) at the
64 stored targets of the 256^3 workload on all cores, and at 4 of them on one core; the
oracle's FLGF solve of the 128^3 workload on one core.  The host's CPU model and core
count are printed with it.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector (packed FP32 instructions)
# The kernels are compiled without packed FP32 instructions, so one FP32 FMA per lane per
# cycle: 256 CUs x 64 lanes x 2 flops x 2.4 GHz, the same as the FP64 vector rate
FP32_ISSUE_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12


def _time_solves(plan, f, u, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.solve(f, u)
    torch.cuda.synchronize()
    plan.profile_enable(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(f, u)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_collect(max(steps, 1))
    return t1 - t0, prof


def _time_graph(plan, f, u, steps, warmup):
    """Whole solves as one HIP-graph launch each; per-launch device latency from events."""
    import torch
    g = plan.graph(f, u)
    for _ in range(warmup):
        g.launch()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        g.launch()
        b.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    g.close()
    return t1 - t0, lat


_SRC = {"prod": ["lgf_prod.hip", "lgf_device.h", "lgf_internal.h"],
        "fft": ["lgf_fft.hip", "lgf_device.h", "lgf_internal.h"],
        "interp": ["lgf_interp.hip", "lgf_device.h", "lgf_internal.h"]}


def _family(step):
    if step.startswith("prod"):
        return "prod"
    if step.startswith("fft"):
        return "fft"
    return "interp"


def _src_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1402_6081_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, prec, step):
    """HBM bytes per launch of `step` from the committed rocprofv3 counter summaries
    (profiles/*.md, FETCH_SIZE + WRITE_SIZE scaled by a copy kernel), or None when no
    summary covers it or the kernel's sources changed since the counters were taken."""
    import glob
    want = _src_hash(_SRC[_family(step)])
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("TRAFFIC "):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if kv.get("workload") == workload and kv.get("prec") == prec and kv.get("step") == step:
                    if kv.get("src") == want:
                        return float(kv["bytes"]), os.path.basename(path)
    return None, None


def _roofline(prof, dtype_peak_tflops, workload=None, prec=None):
    steps = prof["steps"]
    ns = max(prof["nsolves"], 1)
    dom = max(steps, key=lambda s: s["total_ms"])
    avg_s = dom["total_ms"] / ns / 1e3
    gbs = dom["bytes"] / avg_s / 1e9
    tfl = dom["flops"] / avg_s / 1e12
    # bound: compare the step's arithmetic intensity with the machine ridge
    ridge = dtype_peak_tflops * 1e12 / (HBM_PEAK_GBS * 1e9)
    intensity = dom["flops"] / max(dom["bytes"], 1.0)
    if intensity < ridge:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(tfl, 3), "peak": dtype_peak_tflops, "unit": "TFLOP/s",
                "frac": round(tfl / dtype_peak_tflops, 4)}
    traffic, src = measured_traffic(workload, prec, dom["name"]) if workload else (None, None)
    if dtype_peak_tflops == FP32_PEAK_TFLOPS:
        # the same kernel against the FP32 rate the build can issue (no packed instructions)
        roof["fp32_issue_peak_tflops"] = round(FP32_ISSUE_TFLOPS, 1)
        roof["frac_of_fp32_issue_peak"] = round(tfl / FP32_ISSUE_TFLOPS, 4)
        roof["achieved_tflops"] = round(tfl, 3)
    roof.update({"kernel_step": dom["name"], "avg_ms": round(avg_s * 1e3, 5),
                 "algorithmic_bytes": dom["bytes"], "algorithmic_flops": dom["flops"],
                 "traffic": traffic})
    if src:
        roof["traffic_from"] = src
    return roof


def _solve_hbm(prof, ms_per_solve, copy_gbps, workload, prec):
    """HBM rate of a whole solve: the bytes of all its steps (algorithmic, and the
    rocprofv3-measured traffic when every step has a committed counter entry) over the
    solve time, against the measured device-copy bandwidth and the 8 TB/s peak."""
    alg = sum(s["bytes"] for s in prof["steps"])  # per solve
    tr = [measured_traffic(workload, prec, s["name"])[0] for s in prof["steps"]]
    traffic = sum(tr) if tr and all(t is not None for t in tr) else None
    t = ms_per_solve / 1e3
    bytes_ = traffic if traffic is not None else alg
    gbs = bytes_ / t / 1e9
    return {"algorithmic_bytes": round(alg), "traffic": round(traffic) if traffic is not None else None,
            "ms": round(ms_per_solve, 5), "GBps": round(gbs, 1),
            "frac_of_copy": round(gbs / copy_gbps, 4) if copy_gbps else None,
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_from": "traffic" if traffic is not None else "algorithmic"}


def _breakdown(prof):
    ns = max(prof["nsolves"], 1)
    out = []
    for s in prof["steps"]:
        ms = s["total_ms"] / ns
        out.append({"step": s["name"], "avg_ms": round(ms, 5),
                    "GB/s": round(s["bytes"] / (ms / 1e3) / 1e9, 1) if ms > 0 else None,
                    "GFLOP/s": round(s["flops"] / (ms / 1e3) / 1e9, 1) if ms > 0 else None})
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _golden_large():
    """Oracle values at 64 sampled targets of the 256^3 workload (its FLGF and exact sum),
    written by tests/golden/make_large_samples.py from the oracle alone."""
    with open(os.path.join(ROOT, "tests", "golden", "large_config_samples.json")) as fh:
        return json.load(fh)


def cpu_baseline(cfg_large, cfg_medium, gold):
    """The oracle on the host cores: the exact direct sum of the 256^3 workload at the 64
    stored targets with every core, and at 4 targets with one core; the oracle's FLGF on the
    whole 128^3 workload with one core (plan and pre-computation excluded).  Returns the
    baseline entry and the exact values at the 64 targets."""
    from threadpoolctl import threadpool_limits
    from oracle import flgf, lgf as olgf
    ncpu = os.cpu_count() or 1
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    n = cfg_large["n"]
    P = W_points(cfg_large)
    fl = cfg_large["f"].reshape(-1)
    idx = np.asarray(gold["flat_index"])
    t0 = time.perf_counter()
    olgf.lgf_table(257)  # G up to the workload's largest separation, built once
    t_table = time.perf_counter() - t0
    olgf.set_threads(ncpu)
    t0 = time.perf_counter()
    exact = olgf.direct_sum(P, fl, P[idx])
    dt_all = time.perf_counter() - t0
    olgf.set_threads(1)
    t0 = time.perf_counter()
    olgf.direct_sum(P, fl, P[idx[:4]])
    dt_one = time.perf_counter() - t0
    olgf.set_threads(ncpu)
    with threadpool_limits(limits=1):
        solver = flgf.FLGF(cfg_medium["blocks"], cfg_medium["n"], cfg_medium["p"], cfg_medium["levels"])
        t0 = time.perf_counter()
        solver.solve(cfg_medium["f"])
        dt_b = time.perf_counter() - t0
    npts = int(P.shape[0])
    rate_all = len(idx) / dt_all
    entry = {"value": round(rate_all, 3), "unit": "grid points solved/s", "cores": ncpu, "kind": "oracle",
             "cpu_model": _cpu_model(), "nproc": ncpu,
             "sample": "exact direct sum (Eq. dpoissonsoln, Neumaier sums, OpenMP over targets) of the %s "
                       "workload (%d sources) at its 64 stored targets, %d threads, %.2f s; full field "
                       "extrapolated linearly: %.3g s" % (cfg_large["name"], npts, ncpu, dt_all, npts / rate_all),
             "direct_sum_one_core": {"value": round(4 / dt_one, 4), "unit": "grid points solved/s", "cores": 1,
                                     "sample": "4 of the stored targets, %.2f s; full field extrapolated: %.3g s"
                                               % (dt_one, npts * dt_one / 4)},
             "lgf_table_s": round(t_table, 3),
             "oracle_flgf_one_core": {"value": round(cfg_medium["f"].size / dt_b, 1), "unit": "grid points solved/s",
                                      "cores": 1,
                                      "sample": "one oracle FLGF solve (numpy, one thread) of the whole %s workload "
                                                "(%d points), plan and pre-computation excluded, %.2f s"
                                                % (cfg_medium["name"], cfg_medium["f"].size, dt_b)}}
    return entry, exact


def W_points(cfg):
    from paper_1402_6081_amd import workloads as W
    return W.points_of(cfg["blocks"], cfg["n"]).reshape(-1, 3)


FP32_BAR = 1e-6


def _bar(entry, err):
    """Withhold an FP32 rate whose error against FP64 exceeds the bar."""
    entry["rel_linf_err_vs_fp64"] = err
    entry["meets_fp32_bar"] = bool(err <= FP32_BAR)
    if err > FP32_BAR:
        entry["value_over_bar"] = entry["value"]
        entry["value"] = None
    return entry


def _graph_schedule(plan, f, u, choice, launches=20):
    """The autotuner times eager solves; a graph runs the same schedules with other costs
    (the device's own dependency handling instead of host-side events), so the schedule a
    graph is built with is chosen by timing one graph of each (overlap 1, 3, 2) with the
    tuned kernel variants.  Returns the choice (set on the plan) and the per-launch times."""
    ms = {}
    for ov in (1, 3, 2):
        plan.set_tuning(**dict(choice, overlap=ov))
        dt, _ = _time_graph(plan, f, u, launches, 3)
        ms[ov] = dt / launches * 1e3
    best = dict(choice, overlap=min(ms, key=ms.get))
    plan.set_tuning(**best)
    return best, {str(k): round(v, 5) for k, v in ms.items()}


def _measure(plan, f, u, steps, warmup, graph=True, tune=True):
    """Autotune the plan's kernel variants and eager schedule (lgf_plan_autotune), then
      * eager solves on one stream with per-step events: isolated kernel durations for the
        breakdown and the roofline;
      * graph launches with the tuned variants, in the schedule whose graph is fastest
        (_graph_schedule): the rate and latencies."""
    choice = plan.autotune(f, u, reps=10) if tune else plan.tuning()
    plan.set_tuning(**dict(choice, overlap=2))
    dt_e, prof = _time_solves(plan, f, u, steps, warmup)
    plan.set_tuning(**choice)
    if not graph:  # counter-collection runs: eager solves only
        return dict(dt_eager=dt_e, prof=prof, dt_graph=dt_e, lat_graph=np.asarray(prof["solve_ms"]), tuning=choice,
                    eager_tuning=choice, graph_schedule_ms=None)
    gchoice, sched = _graph_schedule(plan, f, u, choice) if tune else (choice, None)
    dt_g, lat = _time_graph(plan, f, u, steps, warmup)
    return dict(dt_eager=dt_e, prof=prof, dt_graph=dt_g, lat_graph=lat, tuning=gchoice, eager_tuning=choice,
                graph_schedule_ms=sched)


def hbm_copy_bandwidth(mib=2048, reps=10):
    """Achievable HBM bandwidth of a plain device copy (read + write bytes / time), for context."""
    import torch
    x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    gbs = 2.0 * x.numel() * 4 * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return round(gbs, 1)


def copy_calibration(mib):
    """Three plain device copies of `mib` MiB (a kernel of known traffic: mib MiB read and
    mib MiB written per launch) so hardware byte counters can be scaled to bytes."""
    import torch
    x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()


def _pct(x):
    return {"p50": round(float(np.percentile(x, 50)), 5), "p99": round(float(np.percentile(x, 99)), 5)}


def medium_bench(L, W, steps, warmup, copy_gbps, graph=True, tune=True, breakdown=None, fp32=True):
    """The 128^3 workload (8^3 blocks of 16^3, p = 8, 4 levels, 32 zero-net Gaussians), FP64
    and FP32, measured as the headline."""
    import torch
    cfg = W.config_medium()
    npts = int(cfg["f"].size)
    out = {"workload": cfg["name"], "points": npts, "unit": "grid points solved/s"}
    u64h = None
    for prec, dt, peak in (("f64", torch.float64, FP64_PEAK_TFLOPS), ("f32", torch.float32, FP32_PEAK_TFLOPS)):
        if prec == "f32" and not fp32:
            break
        plan = L.Plan(cfg["blocks"], cfg["n"], cfg["p"], cfg["levels"], prec)
        f = torch.from_numpy(cfg["f"]).to("cuda:0", dt)
        u = torch.empty_like(f)
        m = _measure(plan, f, u, steps, warmup, graph=graph, tune=tune)
        res = {"value": round(npts * steps / m["dt_graph"], 1), "ms_per_step": round(m["dt_graph"] / steps * 1e3, 5),
               "latency_ms": _pct(m["lat_graph"]), "tuning": m["tuning"],
               "graph_schedule_ms": m["graph_schedule_ms"],
               "eager_ms_per_step": round(m["dt_eager"] / steps * 1e3, 5),
               "roofline": _roofline(m["prof"], peak, cfg["name"], prec)}
        res["solve_hbm"] = _solve_hbm(m["prof"], res["ms_per_step"], copy_gbps, cfg["name"], prec)
        uh = u.double().cpu().numpy()
        if prec == "f64":
            u64h = uh
        else:
            _bar(res, float(np.max(np.abs(uh - u64h)) / np.max(np.abs(u64h))))
        if breakdown is not None:
            breakdown["cube128_" + prec] = _breakdown(m["prof"])
        out[prec] = res
        plan.close()
        del f, u
        torch.cuda.empty_cache()
    return out


def context_bench(L, W, steps=3, warmup=1, seed=7):
    """The paper's own test geometries at its scale (Sec. 4.1-4.2, Table 2): a cube, a sphere
    and a spherical shell of thickness 0.1 D, each about 1e8 points as ~24k blocks of 16^3,
    with a random manufactured solution (u_rand ~ U[-1, 1], zero on the boundary points, f =
    L u_rand, so G * f = u_rand exactly and the error is known in O(N)).  Schemes p = 8 and
    the paper's n_I = n + 1 = 17 (n_max = 10), FP64 and FP32, full depth, default kernel
    variants, eager solves.  The cube is also run as the paper's Table 2 schemes n_I = 7
    (77^3 blocks of 6^3) and n_I = 13 (38^3 blocks of 12^3), about 1e8 points each.
    Reported per case: points/s, the error against u_rand (relative L-infinity, computed on
    the device), plan time against solve time."""
    import torch
    shapes = (("cube29", W.cube_layout(29), 16, (8, 17)), ("sphere36", W.sphere_layout(36), 16, (8, 17)),
              ("shell44", W.shell_layout(44), 16, (8, 17)), ("cube77_n6", W.cube_layout(77), 6, (7,)),
              ("cube38_n12", W.cube_layout(38), 12, (13,)))
    out = {"note": "context only: the paper's Table 2 rates are 1.2e5 points/s per Xeon X5650 core, FP64, "
                   "n_I = 7..28, N = 1e8; here one MI355X, default kernel variants, eager solves",
           "unit": "grid points solved/s"}
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    for name, blocks, n, schemes in shapes:
        t0 = time.perf_counter()
        u_ex, f = W.manufactured_pair(blocks, n, rng)
        t_gen = time.perf_counter() - t0
        npts = int(f.size)
        res = {"blocks": int(len(blocks)), "n": n, "points": npts, "host_generation_s": round(t_gen, 1)}
        ue = torch.from_numpy(u_ex).to(dev)
        scale = float(torch.max(torch.abs(ue)))
        del u_ex
        for p in schemes:
            for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
                fd = torch.from_numpy(f).to(dev, dt)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan = L.Plan(blocks, n, p, 0, prec)
                torch.cuda.synchronize()
                t_plan = time.perf_counter() - t0
                u = torch.empty_like(fd)
                for _ in range(warmup):
                    plan.solve(fd, u)
                torch.cuda.synchronize()
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
                for a, b in ev:
                    a.record()
                    plan.solve(fd, u)
                    b.record()
                torch.cuda.synchronize()
                ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
                err = float(torch.max(torch.abs(u.double() - ue))) / scale
                info = plan.info()
                res["p%d_%s" % (p, prec)] = {"value": round(npts / (ms * 1e-3), 1), "ms_per_solve": round(ms, 3),
                                              "rel_linf_err_vs_exact": err, "plan_s": round(t_plan, 3),
                                              "plan_over_solve": round(t_plan / (ms * 1e-3), 1),
                                              "levels": info["levels"], "workspace_GB": round(info["workspace_bytes"] / 1e9, 2)}
                print("context %s p=%d %s: %.3f ms, err %.3g, plan %.2f s" % (name, p, prec, ms, err, t_plan),
                      file=sys.stderr, flush=True)
                plan.close()
                del fd, u
                torch.cuda.empty_cache()
        del ue
        torch.cuda.empty_cache()
        out[name] = res
    return out


def batch_bench(L, W, steps, warmup, seed=4):
    """64 independent Eden layouts of 8..512 blocks of 16^3, p = 8, FP32: one batch plan,
    one graph launch per batch, against the same 64 solves issued as separate plans."""
    import torch
    rng = np.random.default_rng(seed)
    sizes = rng.integers(8, 513, size=64)
    lays = [W.eden_layout(int(s), rng) for s in sizes]
    fs = []
    for b in lays:
        fb, _ = W.zero_mean_gaussians(b, 16, rng, max(1, b.shape[0] // 8))
        fs.append(fb)
    npts = int(sum(x.size for x in fs))
    dev = torch.device("cuda:0")
    fcat = torch.from_numpy(np.concatenate(fs)).to(dev, torch.float32)
    ucat = torch.empty_like(fcat)
    t0 = time.perf_counter()
    bp = L.Plan.batch(lays, 16, 8, 0, "f32")
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    choice, sched = _graph_schedule(bp, fcat, ucat, bp.autotune(fcat, ucat, reps=2), launches=5)
    dt_g, lat = _time_graph(bp, fcat, ucat, steps, warmup)
    # the same 64 problems as 64 plans enqueued back to back (no batching)
    plans = [L.Plan(b, 16, 8, 0, "f32") for b in lays]
    fl = [x.contiguous() for x in bp.split(fcat)]
    ul = [torch.empty_like(x) for x in fl]
    for _ in range(warmup):
        L.solve_many(plans, fl, ul)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        L.solve_many(plans, fl, ul)
    torch.cuda.synchronize()
    dt_sep = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(bp.split(ucat), ul))
    for pl in plans:
        pl.close()
    bp.close()
    return {"workload": "64 Eden layouts, 8..512 blocks of 16^3 (seed %d), p=8, f32" % seed,
            "points": npts, "blocks": int(sum(b.shape[0] for b in lays)),
            "value": round(npts * steps / dt_g, 1), "unit": "grid points solved/s",
            "ms_per_batch": round(dt_g / steps * 1e3, 5), "latency_ms": _pct(lat),
            "separate_plans_value": round(npts * steps / dt_sep, 1),
            "separate_plans_ms": round(dt_sep / steps * 1e3, 5),
            "batch_equals_separate": bool(same), "plan_s": round(t_plan, 3), "tuning": choice,
            "graph_schedule_ms": sched}


def split_bench(L, W, steps, warmup, graph=True, tune=True, breakdown=None):
    """Separate source and evaluation blocks: the vortex ring's 779 source blocks evaluated
    on the whole 16^3-block cube of 16^3 points (p = 8, full depth), FP64 and FP32, one
    autotuned graph launch per solve; against the single-set plan of the cube with the
    sources zero-padded to it (the same u, bit for bit)."""
    import torch
    cfg = W.config_split()
    src, ev, n = cfg["blocks"], cfg["eval_blocks"], cfg["n"]
    pos = {tuple(b): i for i, b in enumerate(ev.tolist())}
    at = np.asarray([pos[tuple(b)] for b in src.tolist()])
    fpad = np.zeros((len(ev), n, n, n))
    fpad[at] = cfg["f"]
    npts = len(ev) * n ** 3
    out = {"workload": cfg["name"], "source_blocks": int(len(src)), "eval_blocks": int(len(ev)),
           "points": int(npts), "unit": "evaluation points solved/s"}
    for prec, dt, peak in (("f64", torch.float64, FP64_PEAK_TFLOPS), ("f32", torch.float32, FP32_PEAK_TFLOPS)):
        plan = L.Plan(src, n, cfg["p"], cfg["levels"], prec, eval_blocks=ev)
        f = torch.from_numpy(cfg["f"]).to("cuda:0", dt)
        u = torch.empty(plan.out_shape(), dtype=dt, device="cuda:0")
        m = _measure(plan, f, u, steps, warmup, graph=graph, tune=tune)
        res = {"value": round(npts * steps / m["dt_graph"], 1), "ms_per_step": round(m["dt_graph"] / steps * 1e3, 5),
               "latency_ms": _pct(m["lat_graph"]), "tuning": m["tuning"],
               "eager_ms_per_step": round(m["dt_eager"] / steps * 1e3, 5),
               "roofline": _roofline(m["prof"], peak, cfg["name"], prec)}
        uh = u.double().cpu().numpy()
        if prec == "f64":
            u64h = uh
        else:
            _bar(res, float(np.max(np.abs(uh - u64h)) / np.max(np.abs(u64h))))
        if breakdown is not None:
            breakdown["split_fp64" if prec == "f64" else "split_fp32"] = _breakdown(m["prof"])
        plan.close()
        if graph:
            whole = L.Plan(ev, n, cfg["p"], cfg["levels"], prec)
            fw = torch.from_numpy(fpad).to("cuda:0", dt)
            uw = torch.empty_like(fw)
            if tune:
                whole.autotune(fw, uw, reps=2)
            dt_w, _ = _time_graph(whole, fw, uw, steps, warmup)
            res["single_set_ms_per_step"] = round(dt_w / steps * 1e3, 5)
            res["equal_to_single_set"] = bool(torch.equal(u, uw))
            whole.close()
            del fw, uw
        out[prec] = res
        del f, u
        torch.cuda.empty_cache()
    return out


def scheme_bench(L, W, steps, warmup, graph=True, tune=True, breakdown=None):
    """The paper's own scheme family: n_I = n + 1 = 17 nodes per interval edge with stencils of
    the n_max = 10 closest nodes, on the 128^3 cube of 16^3 blocks, full depth; a random
    manufactured solution, so the error against the exact u is reported with the rate."""
    import torch
    cfg = W.config_scheme()
    npts = int(cfg["f"].size)
    out = {"workload": cfg["name"], "points": npts, "n": cfg["n"], "n_I": cfg["p"], "n_max": 10,
           "unit": "grid points solved/s"}
    scale = float(np.max(np.abs(cfg["u_exact"])))
    for prec, dt, peak in (("f64", torch.float64, FP64_PEAK_TFLOPS), ("f32", torch.float32, FP32_PEAK_TFLOPS)):
        plan = L.Plan(cfg["blocks"], cfg["n"], cfg["p"], cfg["levels"], prec)
        f = torch.from_numpy(cfg["f"]).to("cuda:0", dt)
        u = torch.empty_like(f)
        m = _measure(plan, f, u, steps, warmup, graph=graph, tune=tune)
        uh = u.double().cpu().numpy()
        err = float(np.max(np.abs(uh - cfg["u_exact"])) / scale)
        out[prec] = {"value": round(npts * steps / m["dt_graph"], 1), "ms_per_step": round(m["dt_graph"] / steps * 1e3, 5),
                     "latency_ms": _pct(m["lat_graph"]), "tuning": m["tuning"],
                     "eager_ms_per_step": round(m["dt_eager"] / steps * 1e3, 5),
                     "rel_linf_err_vs_exact": err, "workspace_bytes": plan.info()["workspace_bytes"],
                     "roofline": _roofline(m["prof"], peak, cfg["name"], prec)}
        if prec == "f64":
            u64h = uh
        else:
            # a rough manufactured source: the FP32 level-0 transforms lose digits to the
            # cancellation in G * f (the bar holds for smooth sources, not for this one)
            _bar(out[prec], float(np.max(np.abs(uh - u64h)) / np.max(np.abs(u64h))))
        if breakdown is not None:
            breakdown["scheme_fp64" if prec == "f64" else "scheme_fp32"] = _breakdown(m["prof"])
        plan.close()
        del f, u
        torch.cuda.empty_cache()
    return out


def reduced_bench(L, W, steps, warmup, graph=True, tune=True, breakdown=None, scheme=True, compare=True):
    """Symmetry-reduced kernel spectra (one spectrum per class of offsets under the LGF's 48
    signed axis permutations) on the 128^3 workload and on the n_I = n + 1 scheme: the rate
    (tuned, graph-launched as above), the kernel spectra's bytes against the full tables',
    and the difference from the full-table solve of the same input (compare=False: the
    reduced solves only, for counter runs)."""
    import torch
    out = {}
    for cfg in (W.config_medium(), W.config_scheme()) if scheme else (W.config_medium(),):
        npts = int(cfg["f"].size)
        res = {"unit": "grid points solved/s"}
        ref64 = None
        for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
            f = torch.from_numpy(cfg["f"]).to("cuda:0", dt)
            u = torch.empty_like(f)
            plan = L.Plan(cfg["blocks"], cfg["n"], cfg["p"], cfg["levels"], prec, spectra="reduced")
            m = _measure(plan, f, u, steps, warmup, graph=graph, tune=tune)
            ur = u.double().cpu().numpy()
            wl = cfg["name"] + "_reduced"
            r = {"workload": wl, "value": round(npts * steps / m["dt_graph"], 1),
                 "ms_per_step": round(m["dt_graph"] / steps * 1e3, 5), "latency_ms": _pct(m["lat_graph"]),
                 "eager_ms_per_step": round(m["dt_eager"] / steps * 1e3, 5), "tuning": m["tuning"],
                 "spectra_bytes": plan.info()["spectra_bytes"],
                 "roofline": _roofline(m["prof"], FP64_PEAK_TFLOPS if prec == "f64" else FP32_PEAK_TFLOPS, wl, prec)}
            if breakdown is not None and not scheme:
                breakdown["reduced_fp64" if prec == "f64" else "reduced_fp32"] = _breakdown(m["prof"])
            plan.close()
            if compare:
                full = L.Plan(cfg["blocks"], cfg["n"], cfg["p"], cfg["levels"], prec, spectra="full")
                uf = full.solve(f).double().cpu().numpy()
                r["full_spectra_bytes"] = full.info()["spectra_bytes"]
                full.close()
                r["rel_linf_diff_vs_full_tables"] = float(np.max(np.abs(ur - uf)) / np.max(np.abs(uf)))
                if prec == "f64":
                    ref64 = uf
                else:
                    _bar(r, float(np.max(np.abs(ur - ref64)) / np.max(np.abs(ref64))))
            res[prec] = r
            del f, u
            torch.cuda.empty_cache()
        out[cfg["name"]] = res
    return out


def serve_bench(L, W, nreq=192, seed=5, slots=4, load=0.8):
    """Serving: 32 request layouts (bounding box U{2..16} blocks of 16^3, Eden fill
    U[0.3, 1]), p = 8, FP32, through the request server (resident plans, shared spectra).
    Closed loop first (all requests queued at once) gives the capacity; then an open loop
    with Poisson arrivals at `load` x capacity gives the latency percentiles."""
    import torch
    rng = np.random.default_rng(seed)
    mix = W.serving_mix(32, rng)
    dev = torch.device("cuda:0")
    fs = [torch.from_numpy(f).to(dev, torch.float32) for _, f in mix]
    order = rng.integers(0, len(mix), size=nreq)
    us = [torch.empty_like(fs[k]) for k in order]
    srv = L.Server(16, 8, 0, "f32", max_slots=slots)
    # warm-up: every layout's plan becomes resident, every spectrum cached
    for t in [srv.submit(mix[k][0], fs[k], torch.empty_like(fs[k])) for k in range(len(mix))]:
        assert srv.wait(t)["status"] == "LGF_OK"
    srv.reset_stats()
    tickets = [srv.submit(mix[k][0], fs[k], u) for k, u in zip(order, us)]
    for t in tickets:
        assert srv.wait(t)["status"] == "LGF_OK"
    closed = srv.stats()
    cap_rps = closed["completed"] / (closed["points"] / closed["points_per_s"])  # requests/s
    # open loop, Poisson arrivals
    srv.reset_stats()
    gaps = rng.exponential(1.0 / (load * cap_rps), size=nreq)
    t0 = time.perf_counter()
    due = t0
    tickets = []
    for k, u, g in zip(order, us, gaps):
        due += g
        while time.perf_counter() < due:
            pass
        tickets.append(srv.submit(mix[k][0], fs[k], u))
    res = [srv.wait(t) for t in tickets]
    assert all(r["status"] == "LGF_OK" for r in res)
    st = srv.stats()
    srv.close()
    pts_req = [mix[k][1].size for k in order]
    return {"workload": "%d requests over 32 Eden-box layouts (edge U{2..16} blocks of 16^3, fill U[0.3,1]; "
                        "seed %d), p=8, f32, %d slots" % (nreq, seed, slots),
            "points_per_request_mean": round(float(np.mean(pts_req)), 1),
            "closed_loop": {"value": round(closed["points_per_s"], 1), "unit": "grid points solved/s",
                            "requests_per_s": round(cap_rps, 1),
                            "latency_ms": {"p50": round(closed["latency_p50_ms"], 4),
                                           "p99": round(closed["latency_p99_ms"], 4)}},
            "open_loop": {"offered_load": load, "value": round(st["points_per_s"], 1),
                          "unit": "grid points solved/s",
                          "latency_ms": {"p50": round(st["latency_p50_ms"], 4),
                                         "p99": round(st["latency_p99_ms"], 4),
                                         "max": round(st["latency_max_ms"], 4)},
                          "device_ms_p50": round(float(np.percentile([r["device_ms"] for r in res], 50)), 4)},
            "resident_plan_bytes": st["plan_bytes"], "spectra_bytes": st["spectra_bytes"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-medium", action="store_true", help="skip the 128^3 workload")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--no-scheme", action="store_true")
    ap.add_argument("--no-reduced", action="store_true", help="skip the symmetry-reduced spectra runs")
    ap.add_argument("--reduced-only", action="store_true",
                    help="only the 128^3 workload with symmetry-reduced spectra (profiling runs)")
    ap.add_argument("--split-only", action="store_true",
                    help="only the separate-set workload (profiling runs); prints its JSON object")
    ap.add_argument("--context", action="store_true",
                    help="only the paper-scale context run (cube, sphere, shell of ~1e8 points); prints its JSON object")
    ap.add_argument("--scheme-only", action="store_true",
                    help="only the n_I = n + 1 scheme workload (profiling runs); prints its JSON object")
    ap.add_argument("--medium-only", action="store_true",
                    help="only the 128^3 workload (profiling runs); prints its JSON object")
    ap.add_argument("--no-graph", action="store_true", help="eager solves only (counter runs)")
    ap.add_argument("--no-tune", action="store_true", help="default kernel variants, no autotuning")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run 3 plain device copies of MIB MiB (counter calibration)")
    ap.add_argument("--breakdown", default=None, help="write the per-step breakdown JSON here")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported (the solve is not sharded "
              "across GPUs)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1402_6081_amd.lgf as L
    from paper_1402_6081_amd import workloads as W

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    if args.context:
        print(json.dumps({"context": context_bench(L, W)}), flush=True)
        return
    if args.medium_only:
        breakdown = {}
        out = medium_bench(L, W, args.steps, args.warmup, hbm_copy_bandwidth(), graph=not args.no_graph,
                           tune=not args.no_tune, breakdown=breakdown, fp32=not args.no_fp32)
        if args.breakdown:
            with open(args.breakdown, "w") as fh:
                json.dump(breakdown, fh, indent=1)
        print(json.dumps({"cube128": out}), flush=True)
        return
    if args.split_only or args.scheme_only or args.reduced_only:
        breakdown = {}
        if args.reduced_only:  # the 128^3 workload with reduced spectra, no full-table runs
            leg = "reduced_spectra"
            out = reduced_bench(L, W, args.steps, args.warmup, graph=not args.no_graph, tune=not args.no_tune,
                                breakdown=breakdown, scheme=False, compare=False)
        else:
            leg, fn = ("split", split_bench) if args.split_only else ("scheme", scheme_bench)
            out = fn(L, W, args.steps, args.warmup, graph=not args.no_graph, tune=not args.no_tune,
                     breakdown=breakdown)
        if args.breakdown:
            with open(args.breakdown, "w") as fh:
                json.dump(breakdown, fh, indent=1)
        print(json.dumps({leg: out}), flush=True)
        return
    dev = torch.device("cuda:0")
    cfg = W.config_large()
    npts = cfg["f"].size
    f64 = torch.from_numpy(cfg["f"]).to(dev)
    u64 = torch.empty_like(f64)
    t_plan = time.perf_counter()
    plan = L.Plan(cfg["blocks"], cfg["n"], cfg["p"], cfg["levels"], "f64")
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t_plan
    m = _measure(plan, f64, u64, args.steps, args.warmup, graph=not args.no_graph, tune=not args.no_tune)
    print("fp64 measured", flush=True, file=sys.stderr)
    info = plan.info()
    copy_gbps = hbm_copy_bandwidth()

    result = {
        "metric": "grid points solved/s, FP32 vs FP64 path at rel err <=1e-6; p50/p99 solve latency",
        "value": round(npts * args.steps / m["dt_graph"], 1),
        "unit": "grid points solved/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["dt_graph"] / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "points": int(npts), "blocks": int(info["nblocks"]),
                   "n": cfg["n"], "p": cfg["p"], "levels": info["levels"],
                   "launch": "eager lgf_solve" if args.no_graph else "hip graph per solve",
                   "tuning": m["tuning"], "graph_schedule_ms": m["graph_schedule_ms"],
                   "source": "thin vortex ring, R=80, core sigma=4, seeded tilt (seed 2)"},
        "latency_ms": _pct(m["lat_graph"]),
        "eager": {"value": round(npts * args.steps / m["dt_eager"], 1),
                  "ms_per_step": round(m["dt_eager"] / args.steps * 1e3, 5),
                  "latency_ms": _pct(m["prof"]["solve_ms"]),
                  "note": "lgf_solve per step on one stream, with per-step profiling events (roofline source)"},
        "plan_s": round(t_plan, 3),
        "workspace_bytes": info["workspace_bytes"],
        "roofline": _roofline(m["prof"], FP64_PEAK_TFLOPS, cfg["name"], "f64"),
        "hbm_copy_GBps": copy_gbps,
    }
    result["solve_hbm"] = _solve_hbm(m["prof"], result["ms_per_step"], copy_gbps, cfg["name"], "f64")
    breakdown = {"fp64": _breakdown(m["prof"])}
    u64_host = u64.cpu().numpy().reshape(-1)
    plan.close()
    del u64
    u32_host = None
    if not args.no_fp32:
        f32 = f64.float()
        u32 = torch.empty_like(f32)
        plan32 = L.Plan(cfg["blocks"], cfg["n"], cfg["p"], cfg["levels"], "f32")
        m32 = _measure(plan32, f32, u32, args.steps, args.warmup, graph=not args.no_graph, tune=not args.no_tune)
        print("fp32 measured", flush=True, file=sys.stderr)
        u32_host = u32.double().cpu().numpy().reshape(-1)
        err = float(np.max(np.abs(u32_host - u64_host)) / np.max(np.abs(u64_host)))
        result["fp32"] = _bar({"value": round(npts * args.steps / m32["dt_graph"], 1),
                               "unit": "grid points solved/s", "dtype": "f32",
                               "ms_per_step": round(m32["dt_graph"] / args.steps * 1e3, 5),
                               "latency_ms": _pct(m32["lat_graph"]),
                               "eager_ms_per_step": round(m32["dt_eager"] / args.steps * 1e3, 5),
                               "tuning": m32["tuning"], "graph_schedule_ms": m32["graph_schedule_ms"],
                               "workspace_bytes": plan32.info()["workspace_bytes"],
                               "roofline": _roofline(m32["prof"], FP32_PEAK_TFLOPS, cfg["name"], "f32"),
                               "note": "FP32 transforms and products; FP64 kernel tables and spectrum "
                                       "generation, FP64 arithmetic in the level >= 1 inverse transforms "
                                       "(float-float node values), FP64 final add"}, err)
        result["fp32"]["solve_hbm"] = _solve_hbm(m32["prof"], result["fp32"]["ms_per_step"], copy_gbps,
                                                 cfg["name"], "f32")
        breakdown["fp32"] = _breakdown(m32["prof"])
        plan32.close()
        del f32, u32
    del f64
    torch.cuda.empty_cache()
    # accuracy against the oracle at the 64 stored targets (its FLGF, the same operator, and
    # the exact sum, computed live in the cpu_baseline leg)
    gold = _golden_large()
    idx = np.asarray(gold["flat_index"])
    flgf_ref = np.asarray(gold["flgf"])
    scale = float(gold["max_abs_u"])
    acc = {"targets": int(len(idx)), "scale": "max|u| over the field (oracle)",
           "fp64_vs_oracle_flgf": float(np.max(np.abs(u64_host[idx] - flgf_ref)) / scale)}
    if u32_host is not None:
        acc["fp32_vs_oracle_flgf"] = float(np.max(np.abs(u32_host[idx] - flgf_ref)) / scale)
    if not args.no_cpu_baseline:
        result["cpu_baseline"], exact = cpu_baseline(cfg, W.config_medium(), gold)
        print("cpu baseline measured", flush=True, file=sys.stderr)
        es = float(np.max(np.abs(exact)))
        acc["oracle_flgf_vs_exact"] = float(np.max(np.abs(flgf_ref - exact)) / es)
        acc["fp64_vs_exact"] = float(np.max(np.abs(u64_host[idx] - exact)) / es)
        if u32_host is not None:
            acc["fp32_vs_exact"] = float(np.max(np.abs(u32_host[idx] - exact)) / es)
    result["accuracy"] = acc
    del u64_host, u32_host

    if not args.no_medium:
        result["cube128"] = medium_bench(L, W, args.steps, args.warmup, copy_gbps, graph=not args.no_graph,
                                         tune=not args.no_tune, breakdown=breakdown, fp32=not args.no_fp32)
        print("128^3 workload measured", flush=True, file=sys.stderr)

    if not args.no_batch:
        result["batch"] = batch_bench(L, W, max(5, args.steps // 5), 2)
        print("batch measured", flush=True, file=sys.stderr)
    if not args.no_serve:
        result["serve"] = serve_bench(L, W)
        print("serving measured", flush=True, file=sys.stderr)
    if not args.no_split:
        result["split"] = split_bench(L, W, max(5, args.steps // 5), 2, graph=not args.no_graph,
                                      tune=not args.no_tune, breakdown=breakdown)
        print("separate-set solves measured", flush=True, file=sys.stderr)
    if not args.no_scheme:
        result["scheme"] = scheme_bench(L, W, max(5, args.steps // 5), 2, graph=not args.no_graph,
                                        tune=not args.no_tune, breakdown=breakdown)
        print("n_I = n + 1 scheme measured", flush=True, file=sys.stderr)
    if not args.no_reduced:
        result["reduced_spectra"] = reduced_bench(L, W, max(5, args.steps // 5), 2, graph=not args.no_graph,
                                                  tune=not args.no_tune)
        print("symmetry-reduced spectra measured", flush=True, file=sys.stderr)

    result["paper_context"] = {"value": 1.2e5, "unit": "grid points solved/s",
                               "hardware": "1 core Intel Xeon X5650 2.66 GHz, FP64, N = 1e8, n_I = 7..28"}
    if args.breakdown:
        with open(args.breakdown, "w") as fh:
            json.dump(breakdown, fh, indent=1)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
