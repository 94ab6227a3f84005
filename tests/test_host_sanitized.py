"""Host-side checking without a GPU: the plan's tree and lists (lgf_host.cpp) and the request
server's scheduling core (lgf_server_core.h) built on their own with g++ under the address
and undefined-behaviour sanitizers, and the server core also under the thread sanitizer.

* The plan checker builds single-set, separate-set and batch (union) plans for many
  layouts, edge cases included, and runs check_host on each; its counts must equal the
  production library's lgf_plan_estimate (the same code, built by hipcc without
  sanitizers), which tests/test_host_plan.py pins to the oracle's tree.
* The server checker drives ServerCore with a mock executor (scenarios in
  tests/server_core_check.cpp): admission order, slot and plan exclusivity, the HBM budget
  with least-recently-used eviction, oversize refusal, waiting for running work, the queue
  limit, injected failures at every executor step, 8 concurrent clients, shutdown.
"""
import os
import shutil
import subprocess
import zlib

import numpy as np
import pytest

from paper_1402_6081_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1402_6081_amd", "csrc")
OUT = os.path.join(ROOT, "tests", "_host_build")
GXX = shutil.which("g++")
pytestmark = pytest.mark.skipif(GXX is None, reason="needs g++")

SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")


def _build(name, sources, sanitize):
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, name)
    srcs = [os.path.join(ROOT, s) for s in sources]
    if not os.path.exists(exe) or os.path.getmtime(exe) < max(
            os.path.getmtime(f) for f in srcs + [os.path.join(CSRC, "lgf_host.h"),
                                                 os.path.join(CSRC, "lgf_server_core.h")]):
        cmd = [GXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + sanitize, "-pthread",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC] + srcs + ["-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


@pytest.fixture(scope="module")
def plan_checker():
    return _build("host_plan_check_asan", ["paper_1402_6081_amd/csrc/lgf_host.cpp", "tests/host_plan_check.cpp"],
                  "address,undefined")


def _line(kind, n, p, levels, *layouts):
    parts = [kind, str(n), str(p), str(levels)]
    if kind == "batch":
        parts.append(str(len(layouts)))
    parts += [str(len(b)) for b in layouts] if kind != "single" else [str(len(layouts[0]))]
    for b in layouts:
        parts += [str(int(x)) for x in np.asarray(b, dtype=np.int64).reshape(-1)]
    return " ".join(parts)


def _run(exe, lines):
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, env=SAN_ENV, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    out = r.stdout.strip().split("\n")
    assert len(out) == len(lines)
    return out


def _cases():
    rng = np.random.default_rng(zlib.crc32(b"host-sanitized"))
    single = [
        ("one block", W.cube_layout(1), 8, 6, 0),
        ("line", np.array([[i, 0, 0] for i in range(9)], np.int32), 8, 6, 0),
        ("cube4", W.cube_layout(4), 16, 8, 0),
        ("cube5 truncated", W.cube_layout(5), 4, 5, 2),
        ("eden120", W.eden_layout(120, rng), 8, 9, 0),
        ("eden200 p17", W.eden_layout(200, rng), 16, 17, 0),
        ("sphere10", W.sphere_layout(10), 16, 8, 3),
        ("shell14", W.shell_layout(14), 8, 4, 0),
        ("far apart", np.array([[0, 0, 0], [9000, 3, -5], [-7000, 8000, 12]], np.int32), 4, 3, 0),
        ("negative", W.eden_layout(50, rng) - 1000, 8, 10, 0),
        ("p2", W.eden_layout(40, rng), 4, 2, 0),
    ]
    for k in range(6):
        single.append(("eden%d" % k, W.eden_layout(int(rng.integers(2, 300)), rng), [4, 8, 16][k % 3],
                       [2, 5, 8][k % 3], int(rng.integers(0, 4))))
    splits = []
    for kind in ("dilated", "subset", "disjoint"):
        s, e = W.split_sets(kind, rng)
        splits.append(("split " + kind, s, e, 8, 6, 0))
    splits.append(("split far", W.cube_layout(2), W.cube_layout(2) + 40, 8, 8, 0))
    batches = [("batch", [W.eden_layout(int(m), rng) for m in (5, 60, 1, 130)], 8, 6, 0)]
    return single, splits, batches


def test_plan_host_code_under_sanitizers(plan_checker):
    import paper_1402_6081_amd.lgf as L
    single, splits, batches = _cases()
    lines = [_line("single", n, p, lv, b) for _, b, n, p, lv in single]
    lines += [_line("split", n, p, lv, s, e) for _, s, e, n, p, lv in splits]
    lines += [_line("batch", n, p, lv, *bs) for _, bs, n, p, lv in batches]
    out = _run(plan_checker, lines)
    for (label, b, n, p, lv), o in zip(single, out[:len(single)]):
        v = [int(x) for x in o.split()]
        assert v[0] == 0, (label, o)
        ref = L.plan_estimate(b, n, p, lv, "f64")
        ref32 = L.plan_estimate(b, n, p, lv, "f32")
        nb, depth, top, near = v[1:5]
        assert (nb, depth, top, near) == (ref["nblocks"], ref["levels"], ref["top_level"], ref["near_pairs"]), label
        assert (v[9], v[10]) == (ref["workspace_bytes"], ref32["workspace_bytes"]), label
        per = v[11:]
        assert [per[2 * k] for k in range(depth)] == ref["intervals"][1:depth + 1], label
        assert [per[2 * k + 1] for k in range(depth)] == ref["far_pairs"][1:depth + 1], label
    for (label, s, e, n, p, lv), o in zip(splits, out[len(single):len(single) + len(splits)]):
        v = [int(x) for x in o.split()]
        assert v[0] == 0, (label, o)
        ref = L.plan_estimate(s, n, p, lv, "f64", eval_blocks=e)
        assert (v[1], v[2], v[4], v[7], v[8], v[9]) == (ref["nblocks"], ref["levels"], ref["near_pairs"],
                                                       ref["source_blocks"], ref["eval_blocks"],
                                                       ref["workspace_bytes"]), label
    for (label, bs, n, p, lv), o in zip(batches, out[len(single) + len(splits):]):
        v = [int(x) for x in o.split()]
        assert v[0] == 0, (label, o)
        parts = [L.plan_estimate(b, n, p, lv, "f64") for b in bs]
        assert v[1] == sum(q["nblocks"] for q in parts) and v[4] == sum(q["near_pairs"] for q in parts)


def test_plan_host_code_rejects_bad_layouts(plan_checker):
    dup = np.array([[0, 0, 0], [1, 0, 0], [0, 0, 0]], np.int32)
    wide = np.array([[0, 0, 0], [1 << 20, 0, 0]], np.int32)
    deep = np.array([[0, 0, 0], [1 << 17, 0, 0]], np.int32)  # 19 levels, more than supported
    lines = [_line("single", 8, 6, 0, dup), _line("single", 8, 6, 0, wide),
             _line("split", 8, 6, 0, W.cube_layout(2), dup), _line("single", 8, 6, 0, deep)]
    out = _run(plan_checker, lines)
    assert all(o.split()[0] == "2" for o in out), out  # LGF_ERR_LAYOUT
    assert "duplicate" in out[0] and "2^20" in out[1] and "duplicate evaluation block" in out[2]
    assert "deeper" in out[3]


@pytest.mark.parametrize("sanitize", ["address,undefined", "thread"])
def test_server_core_with_mock_executor(sanitize):
    exe = _build("server_core_check_" + sanitize.split(",")[0], ["tests/server_core_check.cpp"], sanitize)
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "all server-core checks passed" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
