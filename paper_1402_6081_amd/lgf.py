"""Python binding of the C ABI in include/lgf.h (argument marshalling only).

Every step of a solve runs in the HIP kernels of libpaper_lgf.so; this module only
passes torch device pointers and streams through ctypes.  There is no CPU fallback:
if the library is not built, or no GPU is visible, the calls raise.
"""
import ctypes
import os

import numpy as np
import torch  # imported before the library so both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpaper_lgf.so")

F64, F32 = 0, 1
_STATUS = {0: "LGF_OK", 1: "LGF_ERR_ARG", 2: "LGF_ERR_LAYOUT", 3: "LGF_ERR_OOM", 4: "LGF_ERR_BUDGET",
           5: "LGF_ERR_DEVICE", 6: "LGF_ERR_BUSY"}


class LGFError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status
        self.name = _STATUS.get(status, str(status))


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("nblocks", ctypes.c_int64), ("npoints", ctypes.c_int64),
        ("n", ctypes.c_int32), ("p", ctypes.c_int32),
        ("levels", ctypes.c_int32), ("top_level", ctypes.c_int32),
        ("near_pairs", ctypes.c_int64), ("far_pairs", ctypes.c_int64 * 16),
        ("intervals", ctypes.c_int64 * 16), ("workspace_bytes", ctypes.c_int64),
        ("spectra_bytes", ctypes.c_int64), ("precision", ctypes.c_int32),
        ("source_blocks", ctypes.c_int64), ("eval_blocks", ctypes.c_int64),
        ("spectra_mode", ctypes.c_int32), ("kappa", ctypes.c_double),
    ]


TUNING_FIELDS = ("fft0_threads", "near_waves", "near_prefetch", "far_waves", "far_children", "overlap")


class Tuning(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in TUNING_FIELDS]


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("n", ctypes.c_int32), ("p", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


class RequestResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("nblocks", ctypes.c_int64), ("latency_ms", ctypes.c_double),
                ("queue_ms", ctypes.c_double), ("device_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("failed", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("points", ctypes.c_int64), ("plans_created", ctypes.c_int64), ("plans_evicted", ctypes.c_int64),
                ("plan_bytes", ctypes.c_int64), ("spectra_bytes", ctypes.c_int64),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double), ("points_per_s", ctypes.c_double)]


class StepProfile(ctypes.Structure):
    _fields_ = [
        ("nsteps", ctypes.c_int32), ("nsolves", ctypes.c_int32),
        ("name", (ctypes.c_char * 32) * 64), ("total_ms", ctypes.c_double * 64),
        ("bytes", ctypes.c_double * 64), ("flops", ctypes.c_double * 64),
    ]


EXPORTS = ["lgf_plan_create", "lgf_plan_create_screened", "lgf_plan_estimate", "lgf_plan_create_split", "lgf_plan_estimate_split",
           "lgf_plan_create_batch", "lgf_plan_solve_offsets", "lgf_solve", "lgf_solve_many",
           "lgf_graph_create", "lgf_graph_launch", "lgf_graph_destroy", "lgf_plan_autotune", "lgf_plan_get_tuning",
           "lgf_plan_set_tuning", "lgf_server_create", "lgf_server_submit", "lgf_server_poll", "lgf_server_wait",
           "lgf_server_stats", "lgf_server_reset_stats", "lgf_server_destroy",
           "lgf_plan_query", "lgf_plan_destroy", "lgf_set_memory_budget", "lgf_memory_in_use",
           "lgf_spectra_cache_trim", "lgf_set_spectra_mode", "lgf_get_spectra_mode", "lgf_last_error",
           "lgf_green_table", "lgf_green_table_screened", "lgf_far_kernel", "lgf_far_kernel_noalloc",
           "lgf_profile_enable",
           "lgf_profile_collect"]

_lib = None


def library():
    """Load libpaper_lgf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpaper_lgf.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.lgf_plan_create.argtypes = [vp, i64, i32, i32, i32, ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.lgf_plan_create_screened.argtypes = [vp, i64, i32, i32, i32, ctypes.c_double, ctypes.c_int, vp,
                                               ctypes.POINTER(vp)]
        L.lgf_plan_create_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i64), i32, i32, i32, i32,
                                            ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.lgf_plan_solve_offsets.argtypes = [vp, ctypes.POINTER(i64), i32, ctypes.POINTER(i32)]
        L.lgf_plan_estimate.argtypes = [vp, i64, i32, i32, i32, ctypes.c_int, ctypes.POINTER(PlanInfo)]
        L.lgf_plan_create_split.argtypes = [vp, i64, vp, i64, i32, i32, i32, ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.lgf_plan_estimate_split.argtypes = [vp, i64, vp, i64, i32, i32, i32, ctypes.c_int,
                                              ctypes.POINTER(PlanInfo)]
        L.lgf_solve.argtypes = [vp, vp, vp, vp]
        L.lgf_graph_create.argtypes = [vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.lgf_graph_launch.argtypes = [vp, vp]
        L.lgf_graph_destroy.argtypes = [vp]
        L.lgf_plan_autotune.argtypes = [vp, vp, vp, vp, i32]
        L.lgf_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.lgf_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.lgf_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
        L.lgf_server_submit.argtypes = [vp, vp, i64, vp, vp, vp, ctypes.POINTER(i64)]
        L.lgf_server_poll.argtypes = [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(RequestResult)]
        L.lgf_server_wait.argtypes = [vp, i64, ctypes.POINTER(RequestResult)]
        L.lgf_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.lgf_server_reset_stats.argtypes = [vp]
        L.lgf_server_destroy.argtypes = [vp]
        L.lgf_solve_many.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp]
        L.lgf_plan_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.lgf_plan_destroy.argtypes = [vp]
        L.lgf_set_memory_budget.argtypes = [i64]
        L.lgf_set_spectra_mode.argtypes = [i32]
        L.lgf_memory_in_use.restype = i64
        L.lgf_last_error.restype = ctypes.c_char_p
        L.lgf_green_table.argtypes = [i32, vp]
        L.lgf_green_table_screened.argtypes = [i32, ctypes.c_double, vp]
        L.lgf_far_kernel.argtypes = [vp, i64, vp]
        L.lgf_far_kernel_noalloc.argtypes = [vp, i64, vp]
        L.lgf_profile_enable.argtypes = [vp, i32]
        L.lgf_profile_collect.argtypes = [vp, ctypes.POINTER(StepProfile), vp, i32]
        for name in EXPORTS:
            if name in ("lgf_memory_in_use", "lgf_last_error"):
                continue
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise LGFError(status, library().lgf_last_error().decode())


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the LGF solver runs only on the device")


def _layout(blocks):
    return np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 3))


class Plan:
    """lgf_plan_create / lgf_solve / lgf_plan_query / lgf_plan_destroy.

    With `eval_blocks` (lgf_plan_create_split) f lives on `blocks` (B_s) and u on
    `eval_blocks` (B_e).  With `kappa` > 0 (lgf_plan_create_screened) the operator is the
    screened L - kappa."""

    def __init__(self, blocks, n, p, levels=0, precision="f64", stream=None, _layouts=None, eval_blocks=None,
                 spectra=None, kappa=0.0):
        """spectra: "full" or "reduced" kernel spectra for this plan (None: the process-wide
        mode, set_spectra_mode)."""
        self.kappa = float(kappa)
        if self.kappa != 0.0 and (_layouts is not None or eval_blocks is not None):
            raise ValueError("the screened operator is for single-set plans")
        _require_gpu()
        prev = None
        if spectra is not None:
            prev = get_spectra_mode()
            set_spectra_mode(spectra)
        try:
            self._create(blocks, n, p, levels, precision, stream, _layouts, eval_blocks)
        finally:
            if prev is not None:
                set_spectra_mode(prev)

    def _create(self, blocks, n, p, levels, precision, stream, _layouts, eval_blocks):
        self.n, self.p = int(n), int(p)
        self.precision = precision
        prec = {"f64": F64, "f32": F32}[precision]
        self.dtype = torch.float64 if prec == F64 else torch.float32
        h = ctypes.c_void_p()
        self.eval_blocks = None
        if _layouts is None and eval_blocks is not None:
            b, e = _layout(blocks), _layout(eval_blocks)
            _check(library().lgf_plan_create_split(b.ctypes.data, b.shape[0], e.ctypes.data, e.shape[0], self.n,
                                                   self.p, int(levels), prec, _stream_handle(stream),
                                                   ctypes.byref(h)))
            self.eval_blocks = e
        elif _layouts is None and self.kappa != 0.0:
            b = _layout(blocks)
            _check(library().lgf_plan_create_screened(b.ctypes.data, b.shape[0], self.n, self.p, int(levels),
                                                      self.kappa, prec, _stream_handle(stream), ctypes.byref(h)))
        elif _layouts is None:
            b = _layout(blocks)
            _check(library().lgf_plan_create(b.ctypes.data, b.shape[0], self.n, self.p, int(levels), prec,
                                             _stream_handle(stream), ctypes.byref(h)))
        else:
            lay = [np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1, 3)) for x in _layouts]
            ptrs = (ctypes.c_void_p * len(lay))(*[x.ctypes.data for x in lay])
            nbs = (ctypes.c_int64 * len(lay))(*[x.shape[0] for x in lay])
            _check(library().lgf_plan_create_batch(ptrs, nbs, len(lay), self.n, self.p, int(levels), prec,
                                                   _stream_handle(stream), ctypes.byref(h)))
            b = np.concatenate(lay, axis=0)
        self.blocks = b
        self._h = h
        cnt = ctypes.c_int32()
        _check(library().lgf_plan_solve_offsets(h, None, 0, ctypes.byref(cnt)))
        offs = (ctypes.c_int64 * (cnt.value + 1))()
        _check(library().lgf_plan_solve_offsets(h, offs, cnt.value + 1, ctypes.byref(cnt)))
        self.offsets = [int(x) for x in offs]

    @classmethod
    def batch(cls, layouts, n, p, levels=0, precision="f64", stream=None, spectra=None):
        """One plan over independent layouts (lgf_plan_create_batch); fields concatenated in order."""
        return cls(None, n, p, levels, precision, stream, _layouts=list(layouts), spectra=spectra)

    def split(self, x):
        """Views of a batch field [sum N_B, n, n, n] per problem."""
        return [x[a:b] for a, b in zip(self.offsets[:-1], self.offsets[1:])]

    @property
    def handle(self):
        return self._h

    def shape(self):
        """Shape of f (the source blocks)."""
        return (self.blocks.shape[0], self.n, self.n, self.n)

    def out_shape(self):
        """Shape of u (the evaluation blocks; the source blocks unless the sets differ)."""
        nb = self.blocks.shape[0] if self.eval_blocks is None else self.eval_blocks.shape[0]
        return (nb, self.n, self.n, self.n)

    def solve(self, f, u=None, stream=None):
        """u = G * f on the plan's layout; f is a contiguous device tensor [N_s, n, n, n],
        u [N_e, n, n, n] (allocated when None)."""
        if self._h is None:
            raise RuntimeError("plan destroyed")
        self._check_field(f, "f")
        if u is None:
            u = torch.empty(self.out_shape(), dtype=self.dtype, device=f.device)
        else:
            self._check_field(u, "u")
        _check(library().lgf_solve(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                   _stream_handle(stream)))
        return u

    def _check_field(self, x, name):
        shape = self.shape() if name == "f" else self.out_shape()
        if not (x.is_cuda and x.is_contiguous() and x.dtype == self.dtype and tuple(x.shape) == shape):
            raise ValueError("%s must be a contiguous %s device tensor of shape %s" % (name, self.dtype, shape))

    def graph(self, f, u, stream=None):
        """Capture one solve reading f and writing u as a HIP graph (lgf_graph_create)."""
        self._check_field(f, "f")
        self._check_field(u, "u")
        return Graph(self, f, u, stream)

    def autotune(self, f, u=None, reps=3, stream=None):
        """Pick the fastest kernel variants for this plan (lgf_plan_autotune); returns the choice."""
        self._check_field(f, "f")
        if u is None:
            u = torch.empty(self.out_shape(), dtype=self.dtype, device=f.device)
        self._check_field(u, "u")
        _check(library().lgf_plan_autotune(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                           _stream_handle(stream), int(reps)))
        return self.tuning()

    def tuning(self):
        t = Tuning()
        _check(library().lgf_plan_get_tuning(self._h, ctypes.byref(t)))
        return {k: getattr(t, k) for k in TUNING_FIELDS}

    def set_tuning(self, fft0_threads=0, near_waves=4, near_prefetch=0, far_waves=0, far_children=0, overlap=0):
        t = Tuning(int(fft0_threads), int(near_waves), int(near_prefetch), int(far_waves), int(far_children),
                   int(overlap))
        _check(library().lgf_plan_set_tuning(self._h, ctypes.byref(t)))

    def info(self):
        inf = PlanInfo()
        _check(library().lgf_plan_query(self._h, ctypes.byref(inf)))
        d = {k: getattr(inf, k) for k, _ in PlanInfo._fields_}
        d["far_pairs"] = list(inf.far_pairs)
        d["intervals"] = list(inf.intervals)
        return d

    def profile_enable(self, max_solves):
        _check(library().lgf_profile_enable(self._h, int(max_solves)))

    def profile_collect(self, max_solves=4096):
        """Per-step device times of the solves recorded since profile_enable."""
        prof = StepProfile()
        per_solve = np.zeros(max_solves, dtype=np.float64)
        _check(library().lgf_profile_collect(self._h, ctypes.byref(prof), per_solve.ctypes.data, max_solves))
        steps = []
        for j in range(prof.nsteps):
            steps.append(dict(name=bytes(prof.name[j]).split(b"\0")[0].decode(), total_ms=prof.total_ms[j],
                              bytes=prof.bytes[j], flops=prof.flops[j]))
        return dict(nsolves=prof.nsolves, steps=steps, solve_ms=per_solve[:min(prof.nsolves, max_solves)])

    def close(self):
        if self._h is not None:
            library().lgf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _info_dict(inf):
    d = {k: getattr(inf, k) for k, _ in PlanInfo._fields_}
    d["far_pairs"] = list(inf.far_pairs)
    d["intervals"] = list(inf.intervals)
    return d


def plan_estimate(blocks, n, p, levels=0, precision="f64", eval_blocks=None):
    """lgf_plan_estimate (lgf_plan_estimate_split with eval_blocks): the plan summary of a
    layout, computed on the host only."""
    b = _layout(blocks)
    inf = PlanInfo()
    prec = {"f64": F64, "f32": F32}[precision]
    if eval_blocks is None:
        _check(library().lgf_plan_estimate(b.ctypes.data, b.shape[0], int(n), int(p), int(levels), prec,
                                           ctypes.byref(inf)))
    else:
        e = _layout(eval_blocks)
        _check(library().lgf_plan_estimate_split(b.ctypes.data, b.shape[0], e.ctypes.data, e.shape[0], int(n),
                                                 int(p), int(levels), prec, ctypes.byref(inf)))
    return _info_dict(inf)


class Graph:
    """An executable HIP graph of one solve (lgf_graph_create / launch / destroy).

    It keeps references to its plan and buffers so they outlive the graph."""

    def __init__(self, plan, f, u, stream=None):
        self.plan, self.f, self.u = plan, f, u
        h = ctypes.c_void_p()
        _check(library().lgf_graph_create(plan.handle, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                          _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        if self._h is None:
            raise RuntimeError("graph destroyed")
        _check(library().lgf_graph_launch(self._h, _stream_handle(stream)))
        return self.u

    def close(self):
        if self._h is not None:
            library().lgf_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """lgf_server_*: a request loop with HBM-budget admission and resident plans."""

    def __init__(self, n, p, levels=0, precision="f32", max_slots=4, budget_bytes=0, max_queue=0, spectra=None):
        """spectra: "full" or "reduced" kernel spectra for every plan the server creates
        (None: the process-wide mode at creation, set_spectra_mode)."""
        _require_gpu()
        prev = None
        if spectra is not None:
            prev = get_spectra_mode()
            set_spectra_mode(spectra)
        try:
            self._create(n, p, levels, precision, max_slots, budget_bytes, max_queue)
        finally:
            if prev is not None:
                set_spectra_mode(prev)

    def _create(self, n, p, levels, precision, max_slots, budget_bytes, max_queue):
        self.n = int(n)
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        cfg = ServerConfig(int(budget_bytes), int(max_slots), int(max_queue), self.n, int(p), int(levels),
                           {"f64": F64, "f32": F32}[precision])
        h = ctypes.c_void_p()
        _check(library().lgf_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, blocks, f, u, stream=None):
        """Queue u = G * f on `blocks`; returns a ticket.  f, u stay referenced until done.
        The solve runs after the work queued on `stream` (default: torch's current stream)
        before this call, so f may still be in flight there."""
        b = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 3))
        shape = (b.shape[0], self.n, self.n, self.n)
        for x in (f, u):
            if not (x.is_cuda and x.is_contiguous() and x.dtype == self.dtype and tuple(x.shape) == shape):
                raise ValueError("fields must be contiguous %s device tensors of shape %s" % (self.dtype, shape))
        t = ctypes.c_int64()
        _check(library().lgf_server_submit(self._h, b.ctypes.data, b.shape[0], ctypes.c_void_p(f.data_ptr()),
                                           ctypes.c_void_p(u.data_ptr()), _stream_handle(stream), ctypes.byref(t)))
        self._keep[t.value] = (f, u)
        return t.value

    @staticmethod
    def _result(r):
        return dict(status=_STATUS.get(r.status, r.status), nblocks=r.nblocks, latency_ms=r.latency_ms,
                    queue_ms=r.queue_ms, device_ms=r.device_ms)

    def wait(self, ticket):
        r = RequestResult()
        _check(library().lgf_server_wait(self._h, int(ticket), ctypes.byref(r)))
        self._keep.pop(ticket, None)
        return self._result(r)

    def poll(self, ticket):
        r = RequestResult()
        d = ctypes.c_int32()
        _check(library().lgf_server_poll(self._h, int(ticket), ctypes.byref(d), ctypes.byref(r)))
        if not d.value:
            return None
        self._keep.pop(ticket, None)
        return self._result(r)

    def stats(self):
        st = ServerStats()
        _check(library().lgf_server_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def reset_stats(self):
        _check(library().lgf_server_reset_stats(self._h))

    def close(self):
        if self._h is not None:
            library().lgf_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_many(plans, fs, us, stream=None):
    n = len(plans)
    hp = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    hf = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
    hu = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
    _check(library().lgf_solve_many(hp, hf, hu, n, _stream_handle(stream)))
    return us


def green_table(R):
    """G[a, b, c] for 0 <= a, b, c < R from the library's FP64 device table."""
    _require_gpu()
    out = np.zeros((R, R, R), dtype=np.float64)
    _check(library().lgf_green_table(int(R), out.ctypes.data))
    return out


def green_table_screened(R, kappa):
    """G_kappa[a, b, c] for 0 <= a, b, c < R from the library's FP64 device integration."""
    _require_gpu()
    out = np.zeros((R, R, R), dtype=np.float64)
    _check(library().lgf_green_table_screened(int(R), float(kappa), out.ctypes.data))
    return out


def far_kernel(points):
    """The library's A^q far kernel at real points [..., 3]."""
    _require_gpu()
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64))
    shape = pts.shape[:-1]
    pts = pts.reshape(-1, 3)
    out = np.zeros(pts.shape[0], dtype=np.float64)
    _check(library().lgf_far_kernel(pts.ctypes.data, pts.shape[0], out.ctypes.data))
    return out.reshape(shape)


FAR_KERNEL_NOALLOC_MAX_POINTS = 262144  # LGF_FAR_KERNEL_NOALLOC_MAX_POINTS of lgf.h


def far_kernel_noalloc(points):
    """far_kernel through lgf_far_kernel_noalloc (no device allocation; at most
    FAR_KERNEL_NOALLOC_MAX_POINTS points per call)."""
    _require_gpu()
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64))
    shape = pts.shape[:-1]
    pts = pts.reshape(-1, 3)
    out = np.zeros(pts.shape[0], dtype=np.float64)
    _check(library().lgf_far_kernel_noalloc(pts.ctypes.data, pts.shape[0], out.ctypes.data))
    return out.reshape(shape)


def set_memory_budget(nbytes):
    _check(library().lgf_set_memory_budget(int(nbytes)))


def memory_in_use():
    return int(library().lgf_memory_in_use())


def trim_spectra_cache():
    _check(library().lgf_spectra_cache_trim())


SPECTRA_MODES = {"full": 0, "reduced": 1}


def set_spectra_mode(mode):
    """Kernel spectra of plans created afterwards: "full" (one per offset) or "reduced"
    (one per symmetry class of offsets), lgf_set_spectra_mode."""
    _check(library().lgf_set_spectra_mode(SPECTRA_MODES[mode]))


def get_spectra_mode():
    m = int(library().lgf_get_spectra_mode())
    return {v: k for k, v in SPECTRA_MODES.items()}[m]
