"""The allocation-free entry point lgf_far_kernel_noalloc against the allocating
lgf_far_kernel it is a variant of: the same values bit for bit, on two calls in a row (the
second smaller than the first, so it reads nothing the first call left behind), and a call
above the stated maximum refused on the host."""
import ctypes
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_far_kernel_noalloc_matches_allocating_entry():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_1402_6081_amd.lgf as L
    lib = L.library()
    rng = np.random.default_rng(77)
    for npts in (L.FAR_KERNEL_NOALLOC_MAX_POINTS, 5000):
        _say("case: lgf_far_kernel_noalloc, %d points" % npts)
        pts = rng.uniform(-400.0, 400.0, (npts, 3))
        pts[np.max(np.abs(pts), axis=1) < 8] += 16.0  # away from the origin, where A^q is used
        got = L.far_kernel_noalloc(pts)
        ref = L.far_kernel(pts)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))
    # above the maximum: refused before any device work
    n = L.FAR_KERNEL_NOALLOC_MAX_POINTS + 1
    pts = np.ones((n, 3)) * 50.0
    out = np.zeros(n)
    assert lib.lgf_far_kernel_noalloc(pts.ctypes.data, n, out.ctypes.data) == 1  # LGF_ERR_ARG
    assert b"at most" in lib.lgf_last_error()
    assert lib.lgf_far_kernel_noalloc(None, 0, None) == 0
    assert lib.lgf_far_kernel_noalloc(None, 5, None) == 1
    assert not np.any(out)
