"""Python binding of libphiks (the C ABI declared in include/phiks.h).

Argument marshalling only: every step of the computation runs inside libphiks
(host planner in C++, all vector work in HIP kernels on gfx950).  Device buffers are
raw device addresses; ``DeviceArray`` allocates them through the library itself, so
that the process uses the one HIP runtime the library was built against (a second,
differently versioned HIP runtime in the same process -- e.g. one bundled with
another framework -- would be shadowed by soname and is not supported).  Streams are
raw ``hipStream_t`` handles (0 = the null stream).  The library must have been built
(``python paper_2210_07667_amd/build.py``); importing this module fails loudly
otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PHIKS_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("PHIKS_LIBRARY") or os.path.join(_HERE, "libphiks.so")

PHIKS_OK = 0
PHIKS_EINVAL = -1
PHIKS_ENOPLAN = -2
PHIKS_ENOMEM = -3
PHIKS_EDEVICE = -4
PHIKS_EWORKSPACE = -5
PHIKS_ENONFINITE = -6
PHIKS_ETIMEDOUT = -7
PHIKS_SAME_VECTOR = 0
PHIKS_LINCOMB = 1
PHIKS_FP64 = 0
PHIKS_FP32 = 1
PHIKS_BF16X3 = 2
PHIKS_VOP_AXPBY = 0
PHIKS_VOP_RATIONAL = 1
PHIKS_VOP_CUBIC = 2
PHIKS_VOP_BRUSS_U = 3
PHIKS_VOP_BRUSS_V = 4
PHIKS_MATRIX_NODE = 0
PHIKS_MATRIX_LEVEL = 1
NOALLOC_SCRATCH_BYTES = 64 << 20     # PHIKS_NOALLOC_SCRATCH_BYTES
PHIKS_RECT_BENDIXSON = 0
PHIKS_RECT_NORM_CENTERED = 1

# every exported entry point of include/phiks.h
SYMBOLS = ("phiks_plan", "phiks_apply", "phiks_combine", "phiks_workspace_size",
           "phiks_plan_info", "phiks_plan_destroy", "phiks_status_string",
           "phiks_last_error", "phiks_plan_params", "phiks_gll", "phiks_rectangle",
           "phiks_remainder", "phiks_tucker", "phiks_kernel_timing",
           "phiks_kernel_timing_read", "phiks_device_count", "phiks_device_alloc",
           "phiks_device_free", "phiks_memcpy_htod", "phiks_memcpy_dtoh",
           "phiks_device_synchronize", "phiks_memcpy_dtod", "phiks_batch_plan",
           "phiks_batch_apply", "phiks_batch_workspace_size", "phiks_batch_info",
           "phiks_batch_destroy", "phiks_server_create", "phiks_server_register", "phiks_server_submit",
           "phiks_server_wait", "phiks_server_stats", "phiks_server_destroy",
           "phiks_vector_op", "phiks_plan_complex", "phiks_plan_params_complex",
           "phiks_server_lane", "phiks_server_select_evictions", "phiks_server_clock",
           "phiks_apply_noalloc", "phiks_plan_matrix", "phiks_batch_dryrun", "phiks_batch_tuning",
           "phiks_planner_options", "phiks_range_rectangle", "phiks_stream_create",
           "phiks_stream_destroy", "phiks_stream_order", "phiks_stream_synchronize")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python paper_2210_07667_amd/build.py` (no CPU fallback exists)")

_lib = ctypes.CDLL(LIB_PATH)

_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_dpp = ctypes.POINTER(_dp)
_vp = ctypes.c_void_p

_lib.phiks_plan.restype = ctypes.c_int
_lib.phiks_plan.argtypes = [ctypes.c_int, _i64p, _dpp, ctypes.c_double, ctypes.c_int,
                            ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, ctypes.c_int,
                            _vp, ctypes.POINTER(_vp)]
_lib.phiks_apply.restype = ctypes.c_int
_lib.phiks_apply.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.phiks_apply_noalloc.restype = ctypes.c_int
_lib.phiks_apply_noalloc.argtypes = [_vp, _vp, _vp, _vp]
_lib.phiks_plan_matrix.restype = ctypes.c_int
_lib.phiks_plan_matrix.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp]
_lib.phiks_combine.restype = ctypes.c_int
_lib.phiks_combine.argtypes = [_vp, ctypes.POINTER(_vp), _vp, _vp, ctypes.c_size_t, _vp]
_lib.phiks_workspace_size.restype = ctypes.c_int
_lib.phiks_workspace_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
_lib.phiks_plan_info.restype = ctypes.c_int
_lib.phiks_plan_info.argtypes = [_vp] + [ctypes.POINTER(ctypes.c_int)] * 4
_lib.phiks_plan_destroy.restype = None
_lib.phiks_plan_destroy.argtypes = [_vp]
_lib.phiks_status_string.restype = ctypes.c_char_p
_lib.phiks_status_string.argtypes = [ctypes.c_int]
_lib.phiks_last_error.restype = ctypes.c_char_p
_lib.phiks_last_error.argtypes = []
_lib.phiks_plan_params.restype = ctypes.c_int
_lib.phiks_plan_params.argtypes = [ctypes.c_int, _i64p, _dpp, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp]
_lib.phiks_plan_params.argtypes += [ctypes.POINTER(ctypes.c_int)] * 3
_lib.phiks_tucker.restype = ctypes.c_int
_lib.phiks_tucker.argtypes = [ctypes.c_int, _i64p, ctypes.POINTER(_vp), _vp, _vp, _vp,
                              ctypes.c_size_t, _vp]
_lib.phiks_kernel_timing.restype = ctypes.c_int
_lib.phiks_kernel_timing.argtypes = [ctypes.c_int]
_lib.phiks_kernel_timing_read.restype = ctypes.c_int
_lib.phiks_kernel_timing_read.argtypes = [_dp, _i64p, _dp]
_lib.phiks_gll.restype = ctypes.c_int
_lib.phiks_gll.argtypes = [ctypes.c_int, _dp, _dp]
_lib.phiks_rectangle.restype = ctypes.c_int
_lib.phiks_rectangle.argtypes = [ctypes.c_int64, _dp, _dp]
_lib.phiks_range_rectangle.restype = ctypes.c_int
_lib.phiks_range_rectangle.argtypes = [ctypes.c_int64, _dp, ctypes.c_int, _dp]


class PlannerOptions(ctypes.Structure):
    """phiks_planner_options_t: the planner's q range, s limit and rectangle kind."""
    _fields_ = [("q_min", ctypes.c_int), ("q_max", ctypes.c_int), ("s_max", ctypes.c_int),
                ("rect", ctypes.c_int)]

    def as_tuple(self):
        return (self.q_min, self.q_max, self.s_max, self.rect)


_lib.phiks_planner_options.restype = ctypes.c_int
_lib.phiks_planner_options.argtypes = [ctypes.POINTER(PlannerOptions), ctypes.POINTER(PlannerOptions)]
_lib.phiks_remainder.restype = ctypes.c_int
_lib.phiks_remainder.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 _dp]

_lib.phiks_batch_plan.restype = ctypes.c_int
_lib.phiks_batch_plan.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_i64p),
                                  ctypes.POINTER(_dpp), _dp, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, _dp, ctypes.c_int, _vp, ctypes.POINTER(_vp)]
_lib.phiks_batch_apply.restype = ctypes.c_int
_lib.phiks_batch_apply.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp,
                                   ctypes.c_size_t, _vp]
_lib.phiks_batch_workspace_size.restype = ctypes.c_int
_lib.phiks_batch_workspace_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
_lib.phiks_batch_info.restype = ctypes.c_int
_lib.phiks_batch_info.argtypes = [_vp, ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 4
_lib.phiks_batch_destroy.restype = None
_lib.phiks_batch_destroy.argtypes = [_vp]
_lib.phiks_batch_tuning.restype = ctypes.c_int
_lib.phiks_batch_tuning.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
_lib.phiks_batch_dryrun.restype = ctypes.c_int
_lib.phiks_batch_dryrun.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_i64p),
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p, _i64p, _i64p]



class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("completed", "ticks", "cache_hits", "cache_misses",
                                              "evictions", "cache_bytes", "cached_plans",
                                              "timed_out")]


_lib.phiks_server_create.restype = ctypes.c_int
_lib.phiks_server_create.argtypes = [ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(_vp)]
_lib.phiks_server_register.restype = ctypes.c_int
_lib.phiks_server_register.argtypes = [_vp, ctypes.c_int, _i64p, _dpp, _i64p]
_lib.phiks_server_submit.restype = ctypes.c_int
_lib.phiks_server_submit.argtypes = [_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                     _vp, _vp, _i64p]
_lib.phiks_server_wait.restype = ctypes.c_int
_lib.phiks_server_wait.argtypes = [_vp, ctypes.c_int64, _dp, _dp]
_lib.phiks_server_clock.restype = ctypes.c_double
_lib.phiks_server_clock.argtypes = []
_lib.phiks_server_lane.restype = ctypes.c_int
_lib.phiks_server_lane.argtypes = [ctypes.c_int64, ctypes.c_int]
_lib.phiks_server_stats.restype = ctypes.c_int
_lib.phiks_server_stats.argtypes = [_vp, ctypes.POINTER(ServerStats)]
_lib.phiks_server_destroy.restype = None
_lib.phiks_server_destroy.argtypes = [_vp]
_ip = ctypes.POINTER(ctypes.c_int)
_szp = ctypes.POINTER(ctypes.c_size_t)
_lib.phiks_server_select_evictions.restype = ctypes.c_int
_lib.phiks_server_select_evictions.argtypes = [ctypes.c_int, _szp, _ip,
                                               ctypes.POINTER(ctypes.c_uint64), ctypes.c_size_t,
                                               ctypes.c_size_t, ctypes.c_size_t, _ip, _ip]
_lib.phiks_plan_complex.restype = ctypes.c_int
_lib.phiks_plan_complex.argtypes = [ctypes.c_int, _i64p, _dpp, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp,
                                    _vp, ctypes.POINTER(_vp)]
_lib.phiks_plan_params_complex.restype = ctypes.c_int
_lib.phiks_plan_params_complex.argtypes = [ctypes.c_int, _i64p, _dpp, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_int, _dp]
_lib.phiks_plan_params_complex.argtypes += [ctypes.POINTER(ctypes.c_int)] * 3
_lib.phiks_vector_op.restype = ctypes.c_int
_lib.phiks_vector_op.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, _vp, ctypes.c_double,
                                 _vp, _vp, _vp]


class PhiksError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.phiks_status_string(status).decode()
        detail = _lib.phiks_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}){': ' + detail if detail else ''}")
        self.status = status


def _check(status: int, where: str) -> None:
    if status != PHIKS_OK:
        raise PhiksError(status, where)


def status_string(status: int) -> str:
    return _lib.phiks_status_string(status).decode()


def _host_mats(A: Sequence[np.ndarray]):
    mats = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in A]
    for m in mats:
        if m.ndim != 2 or m.shape[0] != m.shape[1]:
            raise ValueError("each A_mu must be a square matrix")
    n = (ctypes.c_int64 * len(mats))(*[m.shape[0] for m in mats])
    ptrs = (_dp * len(mats))(*[m.ctypes.data_as(_dp) for m in mats])
    return mats, n, ptrs


def _task_code(task) -> int:
    if task in ("same_vector", PHIKS_SAME_VECTOR):
        return PHIKS_SAME_VECTOR
    if task in ("lincomb", PHIKS_LINCOMB):
        return PHIKS_LINCOMB
    raise ValueError(f"unknown task {task!r}")


def _norms(vnorms):
    if vnorms is None:
        return None, None
    arr = (ctypes.c_double * len(vnorms))(*[float(x) for x in vnorms])
    return arr, ctypes.cast(arr, _dp)


def _host_mats_complex(A: Sequence[np.ndarray]):
    """Complex matrices as row-major (re, im) interleaved float64."""
    mats = [np.ascontiguousarray(np.asarray(a, dtype=np.complex128)) for a in A]
    for m in mats:
        if m.ndim != 2 or m.shape[0] != m.shape[1]:
            raise ValueError("each A_mu must be a square matrix")
    flat = [m.view(np.float64) for m in mats]
    n = (ctypes.c_int64 * len(mats))(*[m.shape[0] for m in mats])
    ptrs = (_dp * len(mats))(*[f.ctypes.data_as(_dp) for f in flat])
    return (mats, flat), n, ptrs


class Plan:
    """Owns a phiks_plan_t (released by close() or garbage collection)."""

    def __init__(self, handle: int, d: int, n, p: int, n_scales: int, task: int,
                 cplx: bool = False):
        self._h = ctypes.c_void_p(handle)
        self.d, self.n, self.p, self.n_scales, self.task = d, list(n), p, n_scales, task
        self.N = int(np.prod(self.n))
        self.cplx = cplx
        self.vlen = 2 * self.N if cplx else self.N   # float64 values per vector

    @property
    def handle(self):
        return self._h

    def info(self):
        s, q, tp, te = (ctypes.c_int() for _ in range(4))
        _check(_lib.phiks_plan_info(self._h, ctypes.byref(s), ctypes.byref(q),
                                    ctypes.byref(tp), ctypes.byref(te)), "phiks_plan_info")
        return {"s": s.value, "q": q.value, "tucker_paper": tp.value, "tucker_exec": te.value}

    def matrix(self, mu: int, kind: int, index: int) -> np.ndarray:
        """One of the plan's small exponentials (phiks_plan_matrix) as a host array:
        kind PHIKS_MATRIX_NODE (node index < q-1) or PHIKS_MATRIX_LEVEL (exp(tau A/2^index))."""
        m = self.n[mu] * (2 if self.cplx else 1)
        buf = DeviceArray(m * m)
        _check(_lib.phiks_plan_matrix(self._h, int(mu), int(kind), int(index), _vp(buf.ptr), None),
               "phiks_plan_matrix")
        return buf.to_numpy().reshape(m, m)

    def workspace_size(self) -> int:
        b = ctypes.c_size_t()
        _check(_lib.phiks_workspace_size(self._h, ctypes.byref(b)), "phiks_workspace_size")
        return b.value

    def close(self):
        if self._h is not None and self._h.value:
            _lib.phiks_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def phiks_plan(A: Sequence[np.ndarray], tau: float, p: int, n_scales: int, tol: float,
               task="same_vector", vnorms: Optional[Sequence[float]] = None,
               precision: int = PHIKS_FP64, stream: int = 0) -> Plan:
    mats, n, ptrs = _host_mats(A)
    keep, vn = _norms(vnorms)
    out = ctypes.c_void_p()
    tc = _task_code(task)
    _check(_lib.phiks_plan(len(mats), n, ptrs, float(tau), int(p), int(n_scales), float(tol),
                           tc, vn, int(precision), ctypes.c_void_p(stream), ctypes.byref(out)),
           "phiks_plan")
    return Plan(out.value, len(mats), list(n), p, n_scales, tc)


def phiks_plan_complex(A: Sequence[np.ndarray], tau: complex, p: int, n_scales: int, tol: float,
                       task="same_vector", vnorms: Optional[Sequence[float]] = None,
                       stream: int = 0) -> Plan:
    """Complex A_mu and step tau; the plan's vectors are complex (DeviceArray.from_numpy
    of a complex array stores it as interleaved float64)."""
    keep, n, ptrs = _host_mats_complex(A)
    karr, vn = _norms(vnorms)
    out = ctypes.c_void_p()
    tc = _task_code(task)
    tau = complex(tau)
    _check(_lib.phiks_plan_complex(len(A), n, ptrs, tau.real, tau.imag, int(p), int(n_scales),
                                   float(tol), tc, vn, ctypes.c_void_p(stream), ctypes.byref(out)),
           "phiks_plan_complex")
    return Plan(out.value, len(A), list(n), p, n_scales, tc, cplx=True)


def phiks_plan_params_complex(A: Sequence[np.ndarray], tau: complex, p: int, n_scales: int,
                              tol: float, task="same_vector", vnorms=None):
    keep, n, ptrs = _host_mats_complex(A)
    karr, vn = _norms(vnorms)
    s, q, tp = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    tau = complex(tau)
    _check(_lib.phiks_plan_params_complex(len(A), n, ptrs, tau.real, tau.imag, int(p),
                                          int(n_scales), float(tol), _task_code(task), vn,
                                          ctypes.byref(s), ctypes.byref(q), ctypes.byref(tp)),
           "phiks_plan_params_complex")
    return s.value, q.value, tp.value


def phiks_apply(plan: Plan, v_ptr: int, out_ptr: int, ws_ptr: int, ws_bytes: int,
                stream: int = 0) -> None:
    _check(_lib.phiks_apply(plan.handle, _vp(v_ptr), _vp(out_ptr), _vp(ws_ptr),
                            ctypes.c_size_t(ws_bytes), _vp(stream)), "phiks_apply")


def phiks_apply_noalloc(plan: Plan, v_ptr: int, out_ptr: int, stream: int = 0) -> None:
    """phiks_apply on the library's fixed per-device scratch (no workspace argument,
    no device allocation); plans needing more than NOALLOC_SCRATCH_BYTES are refused."""
    _check(_lib.phiks_apply_noalloc(plan.handle, _vp(v_ptr), _vp(out_ptr), _vp(stream)),
           "phiks_apply_noalloc")


def phiks_combine(plan: Plan, v_ptrs: Sequence[Optional[int]], out_ptr: int, ws_ptr: int,
                  ws_bytes: int, stream: int = 0) -> None:
    arr = (_vp * len(v_ptrs))(*[None if x is None else _vp(x) for x in v_ptrs])
    _check(_lib.phiks_combine(plan.handle, arr, _vp(out_ptr), _vp(ws_ptr),
                              ctypes.c_size_t(ws_bytes), _vp(stream)), "phiks_combine")


def phiks_tucker(n: Sequence[int], L_ptrs: Sequence[int], v_ptr: int, out_ptr: int,
                 ws_ptr: int, ws_bytes: int, stream: int = 0) -> None:
    nn = (ctypes.c_int64 * len(n))(*[int(x) for x in n])
    lp = (_vp * len(L_ptrs))(*[_vp(x) for x in L_ptrs])
    _check(_lib.phiks_tucker(len(n), nn, lp, _vp(v_ptr), _vp(out_ptr), _vp(ws_ptr),
                             ctypes.c_size_t(ws_bytes), _vp(stream)), "phiks_tucker")


def phiks_plan_params(A: Sequence[np.ndarray], tau: float, p: int, n_scales: int, tol: float,
                      task="same_vector", vnorms: Optional[Sequence[float]] = None):
    """(s, q, T#) the planner chooses (host only, no GPU needed)."""
    mats, n, ptrs = _host_mats(A)
    keep, vn = _norms(vnorms)
    s, q, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_lib.phiks_plan_params(len(mats), n, ptrs, float(tau), int(p), int(n_scales),
                                  float(tol), _task_code(task), vn, ctypes.byref(s),
                                  ctypes.byref(q), ctypes.byref(t)), "phiks_plan_params")
    return s.value, q.value, t.value


def phiks_plan_params_raw(d, n, A_ptrs, tau, p, n_scales, tol, task, vnorms_ptr):
    """Direct pass-through (for argument-validation tests)."""
    s, q, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    return _lib.phiks_plan_params(d, n, A_ptrs, tau, p, n_scales, tol, task, vnorms_ptr,
                                  ctypes.byref(s), ctypes.byref(q), ctypes.byref(t))


def phiks_kernel_timing(enable: bool) -> None:
    _check(_lib.phiks_kernel_timing(1 if enable else 0), "phiks_kernel_timing")


def phiks_kernel_timing_read():
    """(total kernel ms, launches, algorithmic flops) of the mu-mode kernels timed
    since the last read."""
    ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(_lib.phiks_kernel_timing_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl)),
           "phiks_kernel_timing_read")
    return ms.value, n.value, fl.value


def phiks_gll(q: int):
    th = (ctypes.c_double * q)()
    w = (ctypes.c_double * q)()
    _check(_lib.phiks_gll(q, th, w), "phiks_gll")
    return list(th), list(w)


def phiks_rectangle(B: np.ndarray):
    B = np.ascontiguousarray(np.asarray(B, dtype=np.float64))
    xi = (ctypes.c_double * 4)()
    _check(_lib.phiks_rectangle(B.shape[0], B.ctypes.data_as(_dp), xi), "phiks_rectangle")
    return tuple(xi)


def phiks_range_rectangle(B: np.ndarray, rect: int = PHIKS_RECT_BENDIXSON):
    B = np.ascontiguousarray(np.asarray(B, dtype=np.float64))
    xi = (ctypes.c_double * 4)()
    _check(_lib.phiks_range_rectangle(B.shape[0], B.ctypes.data_as(_dp), int(rect), xi),
           "phiks_range_rectangle")
    return tuple(xi)


def planner_options(q_min=None, q_max=None, s_max=None, rect=None):
    """Returns the planner options in force, as (q_min, q_max, s_max, rect); with any
    argument given, replaces those fields (the others kept) and returns the previous
    options."""
    cur = PlannerOptions()
    if q_min is None and q_max is None and s_max is None and rect is None:
        _check(_lib.phiks_planner_options(None, ctypes.byref(cur)), "phiks_planner_options")
        return cur.as_tuple()
    rc = _lib.phiks_planner_options(None, ctypes.byref(cur))
    if rc not in (PHIKS_OK, PHIKS_EINVAL):   # EINVAL: an invalid environment setting
        _check(rc, "phiks_planner_options")
    new = PlannerOptions(cur.q_min if q_min is None else int(q_min),
                         cur.q_max if q_max is None else int(q_max),
                         cur.s_max if s_max is None else int(s_max),
                         cur.rect if rect is None else int(rect))
    _check(_lib.phiks_planner_options(ctypes.byref(new), None), "phiks_planner_options")
    return cur.as_tuple()


def phiks_remainder(q: int, p: int, w: complex):
    err = (ctypes.c_double * p)()
    _check(_lib.phiks_remainder(q, p, float(w.real), float(w.imag), err), "phiks_remainder")
    return list(err)


# ----------------------------------------------------------- device arrays
_lib.phiks_device_count.restype = ctypes.c_int
_lib.phiks_device_count.argtypes = [ctypes.POINTER(ctypes.c_int)]
_lib.phiks_device_alloc.restype = ctypes.c_int
_lib.phiks_device_alloc.argtypes = [ctypes.c_size_t, ctypes.POINTER(_vp)]
_lib.phiks_device_free.restype = ctypes.c_int
_lib.phiks_device_free.argtypes = [_vp]
_lib.phiks_memcpy_htod.restype = ctypes.c_int
_lib.phiks_memcpy_htod.argtypes = [_vp, _vp, ctypes.c_size_t]
_lib.phiks_memcpy_dtoh.restype = ctypes.c_int
_lib.phiks_memcpy_dtoh.argtypes = [_vp, _vp, ctypes.c_size_t]
_lib.phiks_memcpy_dtod.restype = ctypes.c_int
_lib.phiks_memcpy_dtod.argtypes = [_vp, _vp, ctypes.c_size_t, _vp]
_lib.phiks_device_synchronize.restype = ctypes.c_int
_lib.phiks_device_synchronize.argtypes = []


def device_count() -> int:
    n = ctypes.c_int()
    _check(_lib.phiks_device_count(ctypes.byref(n)), "phiks_device_count")
    return n.value


def copy_device(dst: "DeviceArray", src: "DeviceArray", stream: int = 0) -> None:
    n = min(dst.n, src.n) * 8
    _check(_lib.phiks_memcpy_dtod(_vp(dst.ptr), _vp(src.ptr), n, _vp(stream)), "phiks_memcpy_dtod")


def memcpy_dtod(dst_ptr: int, src_ptr: int, nbytes: int, stream: int = 0) -> None:
    """Stream-ordered device-to-device copy of nbytes."""
    _check(_lib.phiks_memcpy_dtod(_vp(dst_ptr), _vp(src_ptr), int(nbytes), _vp(stream)),
           "phiks_memcpy_dtod")


def synchronize() -> None:
    _check(_lib.phiks_device_synchronize(), "phiks_device_synchronize")


for _f, _a in (("phiks_stream_create", [ctypes.POINTER(_vp)]), ("phiks_stream_destroy", [_vp]),
               ("phiks_stream_order", [_vp, _vp]), ("phiks_stream_synchronize", [_vp])):
    getattr(_lib, _f).restype = ctypes.c_int
    getattr(_lib, _f).argtypes = _a


def stream_create() -> int:
    """A new non-blocking stream at the default priority (raw hipStream_t handle)."""
    h = _vp()
    _check(_lib.phiks_stream_create(ctypes.byref(h)), "phiks_stream_create")
    return int(h.value or 0)


def stream_destroy(stream: int) -> None:
    _check(_lib.phiks_stream_destroy(_vp(stream)), "phiks_stream_destroy")


def stream_order(first: int, then: int) -> None:
    """Work enqueued on `then` from now on waits for the work enqueued on `first` so far."""
    _check(_lib.phiks_stream_order(_vp(first), _vp(then)), "phiks_stream_order")


def stream_synchronize(stream: int) -> None:
    _check(_lib.phiks_stream_synchronize(_vp(stream)), "phiks_stream_synchronize")


class DeviceArray:
    """float64 buffer in device memory (allocated through libphiks)."""

    def __init__(self, n: int):
        self.n = int(n)
        p = ctypes.c_void_p()
        _check(_lib.phiks_device_alloc(max(self.n, 1) * 8, ctypes.byref(p)), "phiks_device_alloc")
        self._p = p

    @property
    def ptr(self) -> int:
        return self._p.value

    @property
    def nbytes(self) -> int:
        return self.n * 8

    @classmethod
    def from_numpy(cls, x) -> "DeviceArray":
        """float64 data; complex data is stored as interleaved (re, im) float64."""
        x = np.asarray(x)
        if np.iscomplexobj(x):
            x = np.ascontiguousarray(x.astype(np.complex128)).reshape(-1).view(np.float64)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64)).reshape(-1)
        d = cls(x.size)
        _check(_lib.phiks_memcpy_htod(d._p, x.ctypes.data_as(_vp), x.nbytes), "phiks_memcpy_htod")
        return d

    def to_numpy(self) -> np.ndarray:
        x = np.empty(self.n, dtype=np.float64)
        _check(_lib.phiks_memcpy_dtoh(x.ctypes.data_as(_vp), self._p, x.nbytes), "phiks_memcpy_dtoh")
        return x

    def to_complex(self) -> np.ndarray:
        """The contents read as interleaved (re, im) pairs."""
        return self.to_numpy().view(np.complex128)

    def free(self) -> None:
        if self._p is not None and self._p.value:
            _lib.phiks_device_free(self._p)
        self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def apply_arrays(plan: Plan, v: DeviceArray, out: Optional[DeviceArray] = None,
                 ws: Optional[DeviceArray] = None, stream: int = 0) -> DeviceArray:
    """Same-vector task; out holds n_scales * (p+1) * N values."""
    if plan.task != PHIKS_SAME_VECTOR:
        raise ValueError("plan was made for a linear combination")
    if v.n != plan.vlen:
        raise ValueError("v must hold N values (2N float64 for a complex plan)")
    if out is None:
        out = DeviceArray(plan.n_scales * (plan.p + 1) * plan.vlen)
    if ws is None:
        ws = DeviceArray(plan.workspace_size() // 8 + 1)
    phiks_apply(plan, v.ptr, out.ptr, ws.ptr, ws.nbytes, stream)
    return out


def combine_arrays(plan: Plan, vs, out: Optional[DeviceArray] = None,
                   ws: Optional[DeviceArray] = None, stream: int = 0) -> DeviceArray:
    """Linear-combination task; vs = [v_0, ..., v_p] (None for zero vectors)."""
    if plan.task != PHIKS_LINCOMB:
        raise ValueError("plan was made for the same-vector task")
    if len(vs) != plan.p + 1:
        raise ValueError("need p+1 vectors")
    for x in vs:
        if x is not None and x.n != plan.vlen:
            raise ValueError("vectors must hold N values (2N float64 for a complex plan)")
    if out is None:
        out = DeviceArray(plan.n_scales * plan.vlen)
    if ws is None:
        ws = DeviceArray(plan.workspace_size() // 8 + 1)
    phiks_combine(plan, [None if x is None else x.ptr for x in vs], out.ptr, ws.ptr, ws.nbytes,
                  stream)
    return out


class Batch:
    """Owns a phiks_batch_t (released by close() or garbage collection)."""

    def __init__(self, handle: int, ns_list, p: int, n_scales: int):
        self._h = ctypes.c_void_p(handle)
        self.n = [list(x) for x in ns_list]
        self.N = [int(np.prod(x)) for x in self.n]
        self.count, self.p, self.n_scales = len(self.n), p, n_scales

    @property
    def handle(self):
        return self._h

    def info(self, i: int):
        s, q, tp, te = (ctypes.c_int() for _ in range(4))
        _check(_lib.phiks_batch_info(self._h, int(i), ctypes.byref(s), ctypes.byref(q),
                                     ctypes.byref(tp), ctypes.byref(te)), "phiks_batch_info")
        return {"s": s.value, "q": q.value, "tucker_paper": tp.value, "tucker_exec": te.value}

    def workspace_size(self) -> int:
        b = ctypes.c_size_t()
        _check(_lib.phiks_batch_workspace_size(self._h, ctypes.byref(b)),
               "phiks_batch_workspace_size")
        return b.value

    def close(self):
        if self._h is not None and self._h.value:
            _lib.phiks_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def phiks_batch_plan(As: Sequence[Sequence[np.ndarray]], taus: Sequence[float], p: int,
                     n_scales: int, tol: float, vnorms: Optional[Sequence[float]] = None,
                     precision: int = PHIKS_FP64, stream: int = 0) -> Batch:
    """As[i] = [A_1, ..., A_d] of problem i (host matrices); taus[i] its step."""
    count = len(As)
    if len(taus) != count:
        raise ValueError("one tau per problem")
    keep = [_host_mats(A) for A in As]
    d = (ctypes.c_int * count)(*[len(k[0]) for k in keep])
    n = (_i64p * count)(*[ctypes.cast(k[1], _i64p) for k in keep])
    A = (_dpp * count)(*[ctypes.cast(k[2], _dpp) for k in keep])
    tau = (ctypes.c_double * count)(*[float(t) for t in taus])
    karr, vn = _norms(vnorms)
    out = ctypes.c_void_p()
    _check(_lib.phiks_batch_plan(count, d, n, A, tau, int(p), int(n_scales), float(tol), vn,
                                 int(precision), ctypes.c_void_p(stream), ctypes.byref(out)),
           "phiks_batch_plan")
    return Batch(out.value, [list(k[1]) for k in keep], p, n_scales)


def phiks_batch_apply(batch: Batch, v_ptrs: Sequence[int], out_ptrs: Sequence[int], ws_ptr: int,
                      ws_bytes: int, stream: int = 0) -> None:
    va = (_vp * len(v_ptrs))(*[_vp(x) for x in v_ptrs])
    oa = (_vp * len(out_ptrs))(*[_vp(x) for x in out_ptrs])
    _check(_lib.phiks_batch_apply(batch.handle, va, oa, _vp(ws_ptr), ctypes.c_size_t(ws_bytes),
                                  _vp(stream)), "phiks_batch_apply")


def batch_apply_arrays(batch: Batch, vs: Sequence[DeviceArray], outs=None, ws=None,
                       stream: int = 0):
    """Every problem's outputs, each laid out as apply_arrays' for that problem."""
    if len(vs) != batch.count:
        raise ValueError("one vector per problem")
    for v, N in zip(vs, batch.N):
        if v.n != N:
            raise ValueError("vector i must hold N_i values")
    if outs is None:
        outs = [DeviceArray(batch.n_scales * (batch.p + 1) * N) for N in batch.N]
    if ws is None:
        ws = DeviceArray(batch.workspace_size() // 8 + 1)
    phiks_batch_apply(batch, [v.ptr for v in vs], [o.ptr for o in outs], ws.ptr, ws.nbytes, stream)
    return outs


BATCH_TUNING_FIELDS = ("sq_min", "skinny", "wide_m1", "wide_mk", "wide_lc")


def batch_tuning(values: Optional[dict] = None) -> dict:
    """The batched path's tile-class rules (phiks_batch_tuning); with values, replace them
    first (missing keys keep their current value)."""
    arr = (ctypes.c_int * 5)()
    _check(_lib.phiks_batch_tuning(0, arr), "phiks_batch_tuning")
    if values:
        for k, name in enumerate(BATCH_TUNING_FIELDS):
            if name in values:
                arr[k] = int(values[name])
        _check(_lib.phiks_batch_tuning(1, arr), "phiks_batch_tuning")
    return {name: arr[k] for k, name in enumerate(BATCH_TUNING_FIELDS)}


def batch_dryrun(shapes, plans, p: int, n_scales: int, fork_streams: int = 4):
    """Host-only check of the batched launch schedule (phiks_batch_dryrun): shapes[i] the
    n of problem i, plans[i] its (s, q).  Returns (launches, table bytes, failed checks,
    first failure text)."""
    count = len(shapes)
    d = (ctypes.c_int * count)(*[len(x) for x in shapes])
    ns_arr = [(ctypes.c_int64 * len(x))(*[int(v) for v in x]) for x in shapes]
    n = (_i64p * count)(*[ctypes.cast(a, _i64p) for a in ns_arr])
    s = (ctypes.c_int * count)(*[int(x[0]) for x in plans])
    q = (ctypes.c_int * count)(*[int(x[1]) for x in plans])
    L, T, V = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.phiks_batch_dryrun(count, d, n, s, q, int(p), int(n_scales), int(fork_streams),
                                   ctypes.byref(L), ctypes.byref(T), ctypes.byref(V)),
           "phiks_batch_dryrun")
    return L.value, T.value, V.value, _lib.phiks_last_error().decode() if V.value else ""


def server_lane(n_values: int, lanes: int) -> int:
    """The server's lane for a request of n_values values among `lanes` (host only)."""
    r = _lib.phiks_server_lane(int(n_values), int(lanes))
    if r < 0:
        raise PhiksError(r, "phiks_server_lane")
    return r


def server_clock() -> float:
    """Seconds on the clock of the server's time stamps."""
    return float(_lib.phiks_server_clock())


def server_select_evictions(nbytes: Sequence[int], refs: Sequence[int], last_use: Sequence[int],
                            cache_bytes: int, new_bytes: int, capacity: int):
    """The plan-cache entries the server would evict for a new plan (host only): the
    indices phiks_server_select_evictions picks, in eviction order."""
    n = len(nbytes)
    ba = (ctypes.c_size_t * max(n, 1))(*nbytes)
    ra = (ctypes.c_int * max(n, 1))(*refs)
    la = (ctypes.c_uint64 * max(n, 1))(*last_use)
    victims = (ctypes.c_int * max(n, 1))()
    cnt = ctypes.c_int()
    _check(_lib.phiks_server_select_evictions(n, ba, ra, la, int(cache_bytes), int(new_bytes),
                                              int(capacity), victims, ctypes.byref(cnt)),
           "phiks_server_select_evictions")
    return [victims[i] for i in range(cnt.value)]


def vector_op(op: int, n: int, a: float, x_ptr: int, b: float, y_ptr: Optional[int],
              out_ptr: int, stream: int = 0) -> None:
    """Elementwise device op (PHIKS_VOP_*): see include/phiks.h."""
    _check(_lib.phiks_vector_op(int(op), int(n), float(a), _vp(x_ptr), float(b),
                                None if y_ptr is None else _vp(y_ptr), _vp(out_ptr), _vp(stream)),
           "phiks_vector_op")


class Server:
    """Owns a phiks_server_t: submit() queues one same-vector request, wait() blocks
    until it is done and returns its latency in seconds (wait_times() also its
    completion time on server_clock())."""

    def __init__(self, hbm_budget: int, workspace_bytes: int, max_active: int = 32,
                 lanes: int = 3):
        h = ctypes.c_void_p()
        _check(_lib.phiks_server_create(ctypes.c_size_t(hbm_budget), ctypes.c_size_t(workspace_bytes),
                                        int(max_active), int(lanes), ctypes.byref(h)),
               "phiks_server_create")
        self._h = h

    def register(self, A: Sequence[np.ndarray]) -> int:
        """Registers the operator A_1..A_d; returns its id."""
        mats, n, ptrs = _host_mats(A)
        op = ctypes.c_int64()
        _check(_lib.phiks_server_register(self._h, len(mats), n, ptrs, ctypes.byref(op)),
               "phiks_server_register")
        return op.value

    def submit(self, op: int, tau: float, p: int, n_scales: int, tol: float, v_ptr: int,
               out_ptr: int, precision: int = PHIKS_FP64, timeout: float = 0.0) -> int:
        """Queues one request; `timeout` seconds from now is its deadline (0: none)."""
        t = ctypes.c_int64()
        _check(_lib.phiks_server_submit(self._h, int(op), float(tau), int(p), int(n_scales),
                                        float(tol), int(precision), float(timeout), _vp(v_ptr),
                                        _vp(out_ptr), ctypes.byref(t)),
               "phiks_server_submit")
        return t.value

    def wait_times(self, ticket: int):
        """(latency, completion time) in seconds."""
        lat, done = ctypes.c_double(), ctypes.c_double()
        _check(_lib.phiks_server_wait(self._h, int(ticket), ctypes.byref(lat), ctypes.byref(done)),
               "phiks_server_wait")
        return lat.value, done.value

    def wait(self, ticket: int) -> float:
        return self.wait_times(ticket)[0]

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib.phiks_server_stats(self._h, ctypes.byref(st)), "phiks_server_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            _lib.phiks_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tucker_arrays(n: Sequence[int], Ls: Sequence[DeviceArray], v: DeviceArray,
                  out: Optional[DeviceArray] = None, stream: int = 0) -> DeviceArray:
    N = int(np.prod(n))
    if out is None:
        out = DeviceArray(N)
    ws = DeviceArray(2 * N)
    phiks_tucker(n, [L.ptr for L in Ls], v.ptr, out.ptr, ws.ptr, ws.nbytes, stream)
    ws.free()
    return out
