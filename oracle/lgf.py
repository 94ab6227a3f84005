"""Oracle: lattice Green's function values and the exact direct sum (plain CPU, FP64).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg of
the benchmark may import this module; the product path never does.

* G(n) for max|n_i| < BESSEL_RADIUS comes from the Bessel integral of Appendix A
  (Eq. lgf3), integrated in liblgf_oracle.so.
* Beyond it, G(n) = A^q(n) with q = Q_TABLE terms (Sec. 2.1, Eq. lgf2); A^q agrees
  with the Bessel values to ~1e-15 relative from max|n_i| >= 32 on (checked by the
  oracle's own tests), so the switch is seamless in FP64.
* direct_sum(): u(t) = sum_m G(t - m) f(m)  (Sec. 2.1, Eq. dpoissonsoln), the exact
  result that the fast method approximates.
* A second non-oscillatory lattice kernel (the method applies to such LGFs, Sec. 5): the
  LGF G_kappa of the screened operator L - kappa, kappa >= KAPPA_MIN, by the Bessel
  integral of Appendix A with the extra factor e^{-kappa t} (no tail term: the factor
  makes the integrand negligible beyond x = 80 / kappa).  It has no asymptotic expansion
  here; every value is integrated.  kappa = 0 is the Laplace LGF above.
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

from . import asymptotic

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lgf_oracle.c")
_LIB = os.path.join(_HERE, "liblgf_oracle.so")

BESSEL_RADIUS = 48   # Bessel-integral region: max|n_i| < 48
Q_TABLE = 8          # terms of A^q used beyond it
KAPPA_MIN = 1e-3     # weakest screening: the integral then stops at x = 1e5 (kappa x / 2 >= 50)

# Quadrature parameters of the Bessel integral (converged: halving the panel width,
# raising the order or moving the split point changes G by <= 1 ulp-ish, see tests).
XMAX = 1.0e5
PANEL = 0.25
ORDER = 20

_lock = threading.Lock()
_lib = None


def build_library(force=False):
    """Compile liblgf_oracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", _LIB, "-lm"])
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build_library()
            L = ctypes.CDLL(_LIB)
            L.oracle_lgf_table.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_void_p]
            L.oracle_lgf_table.restype = ctypes.c_int
            L.oracle_scaled_bessel.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
            L.oracle_lgf_table_screened.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
            L.oracle_lgf_table_screened.restype = ctypes.c_int
            L.oracle_direct_sum.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.c_void_p]
            L.oracle_direct_sum.restype = ctypes.c_int
            L.oracle_asym_eval.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]
            L.oracle_num_threads.restype = ctypes.c_int
            L.oracle_set_threads.argtypes = [ctypes.c_int]
            _lib = L
    return _lib


def num_threads():
    return lib().oracle_num_threads()


def set_threads(n):
    """Threads the direct sum and table loops use from now on (OpenMP)."""
    lib().oracle_set_threads(int(n))


def bessel_table(R, xmax=XMAX, panel=PANEL, order=ORDER):
    """G on the full octant [0,R)^3 by the Bessel integral (Appendix A)."""
    out = np.zeros((R, R, R), dtype=np.float64)
    rc = lib().oracle_lgf_table(int(R), float(xmax), float(panel), int(order), out.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle_lgf_table failed")
    return out


def _check_kappa(kappa):
    kappa = float(kappa)
    if not (kappa == 0.0 or kappa >= KAPPA_MIN):
        raise ValueError("kappa must be 0 (Laplace) or >= %g" % KAPPA_MIN)
    return kappa


def screened_table(R, kappa, h=1, xmax=XMAX, panel=PANEL, order=ORDER):
    """G_kappa(h a, h b, h c) on the octant 0 <= a, b, c < R by the Bessel integral with
    the screening factor (kappa >= KAPPA_MIN)."""
    kappa = _check_kappa(kappa)
    if kappa == 0.0:
        raise ValueError("screened_table needs kappa > 0 (the Laplace table is bessel_table)")
    out = np.zeros((R, R, R), dtype=np.float64)
    rc = lib().oracle_lgf_table_screened(int(R), int(h), kappa, float(xmax), float(panel), int(order),
                                         out.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle_lgf_table_screened failed (%d)" % rc)
    return out


def scaled_bessel(x, K):
    """e^{-x} I_k(x) for k = 0..K (Miller recurrence, used by the Bessel integral)."""
    out = np.zeros(K + 1, dtype=np.float64)
    lib().oracle_scaled_bessel(float(x), int(K), out.ctypes.data)
    return out


_asym_cache = {}


def _asym_arrays(q):
    if q not in _asym_cache:
        starts, exps, coefs = [0], [], []
        for j in range(q):
            P = asymptotic.term_polynomial(j)
            for e, c in sorted(P.items()):
                exps.append(e)
                coefs.append(float(c))
            starts.append(len(coefs))
        _asym_cache[q] = (np.asarray(starts, dtype=np.int32),
                          np.ascontiguousarray(np.asarray(exps, dtype=np.int32).reshape(-1, 3)),
                          np.asarray(coefs, dtype=np.float64))
    return _asym_cache[q]


def asymptotic_values(points, q=Q_TABLE):
    """A^q at real points [..., 3] (x, y, z), float64."""
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64))
    shape = pts.shape[:-1]
    pts = pts.reshape(-1, 3)
    starts, exps, coefs = _asym_arrays(q)
    out = np.zeros(pts.shape[0], dtype=np.float64)
    if pts.shape[0]:
        lib().oracle_asym_eval(pts.ctypes.data, pts.shape[0], q, starts.ctypes.data,
                               exps.ctypes.data, coefs.ctypes.data, out.ctypes.data)
    return out.reshape(shape)


_table_cache = {}


def lgf_table(R, kappa=0.0):
    """Full-octant table G[a, b, c], 0 <= a, b, c < R (Bessel near, A^Q_TABLE far); with
    kappa > 0 the screened LGF G_kappa, integrated everywhere."""
    R = int(R)
    kappa = _check_kappa(kappa)
    if kappa > 0.0:
        return lattice_table(R, kappa, 1)
    with _lock:
        hit = _table_cache.get(R)
    if hit is not None:
        return hit
    Rb = min(R, BESSEL_RADIUS)
    T = np.empty((R, R, R), dtype=np.float64)
    T[:Rb, :Rb, :Rb] = bessel_table(Rb)
    if R > Rb:
        # points with max index >= Rb, unique up to permutation: a >= b >= c
        a, b, c = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
        far = np.maximum(np.maximum(a, b), c) >= Rb
        canon = far & (a >= b) & (b >= c)
        idx = np.argwhere(canon)
        vals = asymptotic_values(idx.astype(np.float64), Q_TABLE)
        for perm in [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]:
            T[idx[:, perm[0]], idx[:, perm[1]], idx[:, perm[2]]] = vals
    with _lock:
        _table_cache[R] = T
    return T


_lattice_cache = {}


def lattice_table(R, kappa, h):
    """G_kappa(h a, h b, h c), 0 <= a, b, c < R (kappa > 0), cached."""
    key = (int(R), float(kappa), int(h))
    with _lock:
        hit = _lattice_cache.get(key)
    if hit is not None:
        return hit
    T = screened_table(int(R), kappa, int(h))
    with _lock:
        _lattice_cache[key] = T
    return T


def lgf(points, kappa=0.0):
    """G at integer points [..., 3] (G_kappa with kappa > 0)."""
    pts = np.asarray(points, dtype=np.int64)
    ab = np.abs(pts)
    R = int(ab.max()) + 1 if ab.size else 1
    T = lgf_table(max(R, 2), kappa)
    return T[ab[..., 0], ab[..., 1], ab[..., 2]]


def lgf_lattice(points, kappa, h):
    """G_kappa at integer points [..., 3] that are multiples of h (kappa > 0), from a
    table at spacing h."""
    pts = np.asarray(points, dtype=np.int64)
    if np.any(pts % h):
        raise ValueError("points are not multiples of the spacing")
    ab = np.abs(pts) // h
    R = int(ab.max()) + 1 if ab.size else 1
    T = lattice_table(max(R, 2), kappa, h)
    return T[ab[..., 0], ab[..., 1], ab[..., 2]]


def direct_sum(src, f, tgt, kappa=0.0):
    """u(t) = sum_m G(t - m) f(m) over integer source points src [N,3] (x,y,z),
    source values f [N], integer targets tgt [T,3].  Brute force, Neumaier sums.  With
    kappa > 0, G is the screened operator's LGF G_kappa."""
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32))
    tgt = np.ascontiguousarray(np.asarray(tgt, dtype=np.int32))
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
    lo = np.minimum(src.min(axis=0), tgt.min(axis=0))
    hi = np.maximum(src.max(axis=0), tgt.max(axis=0))
    R = int(np.max(hi - lo)) + 1
    T = lgf_table(max(R, 2), kappa)
    u = np.zeros(tgt.shape[0], dtype=np.float64)
    bad = lib().oracle_direct_sum(T.ctypes.data, T.shape[0], src.ctypes.data, f.ctypes.data,
                                  src.shape[0], tgt.ctypes.data, tgt.shape[0], u.ctypes.data)
    if bad:
        raise RuntimeError("direct_sum: separation beyond table")
    return u


def laplacian(U, kappa=0.0):
    """[L U](n) = sum_{+-e_i} U(n +- e_i) - 6 U(n) (Sec. 2.1, Eq. dpoisson), minus kappa U(n)
    for the screened operator, on a dense array U[z, y, x] that is zero outside it; returns
    an array one cell larger on every side (index shift +1)."""
    U = np.asarray(U, dtype=np.float64)
    P = np.zeros(tuple(s + 4 for s in U.shape))
    P[2:-2, 2:-2, 2:-2] = U
    out = -(6.0 + kappa) * P[1:-1, 1:-1, 1:-1]
    out += P[2:, 1:-1, 1:-1] + P[:-2, 1:-1, 1:-1]
    out += P[1:-1, 2:, 1:-1] + P[1:-1, :-2, 1:-1]
    out += P[1:-1, 1:-1, 2:] + P[1:-1, 1:-1, :-2]
    return out
