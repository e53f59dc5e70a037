"""ctypes binding of libshiftsolve.so -- argument marshalling only.

Every function here converts torch tensors to pointers and calls the C ABI
declared in ``include/shiftsolve.h``; all arithmetic happens in the HIP
kernels.  There is no fallback: if the library is missing, or the tensors
are not on the GPU, the call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshiftsolve.so")

SHS_ABI_VERSION = 2
SHS_MODE_FP64 = 0
SHS_MODE_FP32_REFINE = 1
SHS_OUT_X = 1
SHS_OUT_G = 2
SHS_OUT_ETA = 4
SHS_STATUS_OK = 0
SHS_STATUS_SINGULAR = 1
SHS_STATUS_NONFINITE = 2
SHS_STATUS_FALLBACK = 3
SHS_STATUS_NOT_CONVERGED = 4
SHS_MAX_M = 16
SHS_REQ_QUEUED, SHS_REQ_RUNNING, SHS_REQ_DONE, SHS_REQ_FAILED, SHS_REQ_CANCELLED = range(5)
SHS_ERR_CANCELLED = 7
SHS_ERR_STATE = 8
SHS_ERR_SCRATCH = 9
SHS_NOALLOC_SCRATCH_BYTES = 128 << 20

EXPORTED = ("shs_reduce", "shs_solve_workspace", "shs_solve", "shs_apply_q", "shs_get_reduced",
            "shs_info", "shs_set_timing", "shs_last_timings", "shs_destroy", "shs_strerror",
            "shs_abi_version", "shs_server_create", "shs_server_register", "shs_server_submit",
            "shs_server_poll", "shs_server_wait", "shs_server_latency", "shs_server_stats",
            "shs_server_destroy", "shs_server_submit_ex", "shs_server_cancel", "shs_server_pause",
            "shs_server_clock", "shs_reduce_check_plan", "shs_solve_transposed",
            "shs_solve_transposed_workspace", "shs_transfer_norm2", "shs_solve_vec", "shs_solve_vec_workspace",
            "shs_solve_transposed_vec", "shs_solve_transposed_vec_workspace", "shs_project",
            "shs_project_workspace")

_lib = None


class ShsError(RuntimeError):
    def __init__(self, func: str, code: int):
        self.code = code
        msg = _load().shs_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{func} failed with code {code}: {msg}")


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("p", ctypes.c_int64),
                ("reduce_ms", ctypes.c_double), ("resident_bytes", ctypes.c_size_t)]


class _Timings(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in ("sweep_ms", "qstar_ms", "residual_ms", "sweep32_ms",
                                               "sweep32_dense_ms", "other_ms")] + \
               [(f, ctypes.c_int64) for f in ("sweep_calls", "qstar_calls", "residual_calls", "sweep32_calls",
                                              "sweep32_dense_calls", "other_calls", "sweep_shifts",
                                              "sweep32_shifts", "sweep32_dense_shifts", "refine_iterations",
                                              "fallback_shifts")] + \
               [(f, ctypes.c_double) for f in ("sweep_tile_ms", "sweep_update_ms")] + \
               [(f, ctypes.c_int64) for f in ("sweep_tile_calls", "sweep_update_calls")] + \
               [(f, ctypes.c_double) for f in ("sweep_tile_flops", "sweep_update_flops")]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("streams", ctypes.c_int32), ("budget_bytes", ctypes.c_int64),
                ("max_batch", ctypes.c_int32), ("flags", ctypes.c_int32), ("blocked_flops", ctypes.c_double),
                ("reserved", ctypes.c_int64 * 3)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("submitted", "completed", "failed", "cancelled", "queued", "running",
                                              "solves", "batches", "max_batch_systems", "max_batch_requests")] + \
               [(f, ctypes.c_double) for f in ("p50_ms", "p99_ms", "max_ms", "mean_ms", "busy_s")] + \
               [("peak_bytes", ctypes.c_int64)]


class _RequestOpts(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("order_after", ctypes.c_int32), ("after_stream", ctypes.c_void_p),
                ("arrival_s", ctypes.c_double), ("reserved", ctypes.c_int64 * 4)]


class _Config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int64 * 6)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1708_06290_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    i64, vp, dp = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
    lib.shs_reduce.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64, ctypes.POINTER(_Config), vp,
                               ctypes.POINTER(vp)]
    lib.shs_reduce.restype = ctypes.c_int
    lib.shs_solve_workspace.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    lib.shs_solve_workspace.restype = ctypes.c_int
    lib.shs_solve.argtypes = [vp, i64, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                              vp, ctypes.c_size_t, dp, i64, dp, i64, dp, vp, vp]
    lib.shs_solve.restype = ctypes.c_int
    lib.shs_solve_transposed_workspace.argtypes = [vp, i64, i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.shs_solve_transposed_workspace.restype = ctypes.c_int
    lib.shs_solve_transposed.argtypes = [vp, i64, dp, i64, dp, i64, ctypes.c_int, vp, ctypes.c_size_t, dp, i64, dp,
                                         vp, vp]
    lib.shs_solve_transposed.restype = ctypes.c_int
    for nm in ("shs_solve_vec_workspace", "shs_solve_transposed_vec_workspace"):
        getattr(lib, nm).argtypes = [vp, i64, ctypes.POINTER(ctypes.c_size_t)]
        getattr(lib, nm).restype = ctypes.c_int
    for nm in ("shs_solve_vec", "shs_solve_transposed_vec"):
        getattr(lib, nm).argtypes = [vp, i64, dp, dp, i64, ctypes.c_int, vp, ctypes.c_size_t, dp, i64, dp, vp, vp]
        getattr(lib, nm).restype = ctypes.c_int
    lib.shs_solve_noalloc.argtypes = [vp, i64, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      dp, i64, dp, i64, dp, vp, vp]
    lib.shs_solve_noalloc.restype = ctypes.c_int
    lib.shs_project_workspace.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.shs_project_workspace.restype = ctypes.c_int
    lib.shs_project.argtypes = [vp, i64, dp, i64, dp, i64, vp, vp, ctypes.c_size_t, dp, dp, dp, dp, vp, vp]
    lib.shs_project.restype = ctypes.c_int
    lib.shs_transfer_norm2.argtypes = [i64, i64, i64, dp, i64, dp, vp]
    lib.shs_transfer_norm2.restype = ctypes.c_int
    lib.shs_reduce_check_plan.argtypes = [i64, i64, i64, ctypes.POINTER(i64), ctypes.c_char_p, i64]
    lib.shs_reduce_check_plan.restype = ctypes.c_int
    lib.shs_apply_q.argtypes = [vp, i64, dp, i64, dp, i64, vp]
    lib.shs_apply_q.restype = ctypes.c_int
    lib.shs_get_reduced.argtypes = [vp, dp, i64, dp, i64, dp, i64, vp]
    lib.shs_get_reduced.restype = ctypes.c_int
    lib.shs_info.argtypes = [vp, ctypes.POINTER(_Info)]
    lib.shs_info.restype = ctypes.c_int
    lib.shs_set_timing.argtypes = [vp, ctypes.c_int]
    lib.shs_set_timing.restype = ctypes.c_int
    lib.shs_last_timings.argtypes = [vp, ctypes.POINTER(_Timings)]
    lib.shs_last_timings.restype = ctypes.c_int
    lib.shs_server_create.argtypes = [ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)]
    lib.shs_server_create.restype = ctypes.c_int
    lib.shs_server_register.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32)]
    lib.shs_server_register.restype = ctypes.c_int
    lib.shs_server_submit.argtypes = [vp, ctypes.c_int32, i64, dp, ctypes.c_int, ctypes.c_int, dp, i64, dp, i64,
                                      dp, vp, ctypes.POINTER(ctypes.c_int64)]
    lib.shs_server_submit.restype = ctypes.c_int
    lib.shs_server_submit_ex.argtypes = [vp, ctypes.c_int32, i64, dp, ctypes.c_int, ctypes.c_int, dp, i64, dp, i64,
                                         dp, vp, ctypes.POINTER(_RequestOpts), ctypes.POINTER(ctypes.c_int64)]
    lib.shs_server_submit_ex.restype = ctypes.c_int
    lib.shs_server_cancel.argtypes = [vp, i64]
    lib.shs_server_cancel.restype = ctypes.c_int
    lib.shs_server_pause.argtypes = [vp, ctypes.c_int]
    lib.shs_server_pause.restype = ctypes.c_int
    lib.shs_server_clock.argtypes = []
    lib.shs_server_clock.restype = ctypes.c_double
    lib.shs_server_poll.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_int)]
    lib.shs_server_poll.restype = ctypes.c_int
    lib.shs_server_wait.argtypes = [vp, i64, ctypes.c_double]
    lib.shs_server_wait.restype = ctypes.c_int
    lib.shs_server_latency.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double)]
    lib.shs_server_latency.restype = ctypes.c_int
    lib.shs_server_stats.argtypes = [vp, ctypes.POINTER(_ServerStats)]
    lib.shs_server_stats.restype = ctypes.c_int
    lib.shs_server_destroy.argtypes = [vp]
    lib.shs_server_destroy.restype = None
    lib.shs_destroy.argtypes = [vp]
    lib.shs_destroy.restype = None
    lib.shs_strerror.argtypes = [ctypes.c_int]
    lib.shs_strerror.restype = ctypes.c_char_p
    lib.shs_abi_version.argtypes = []
    lib.shs_abi_version.restype = ctypes.c_int
    if lib.shs_abi_version() != SHS_ABI_VERSION:
        raise RuntimeError("libshiftsolve ABI version mismatch")
    _lib = lib
    return lib


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _load()


def _check(func: str, rc: int):
    if rc != 0:
        raise ShsError(func, rc)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _colmajor(t):
    """Column-major copy of a 2-D tensor: returns (storage tensor, ld)."""
    if t.dim() == 1:
        t = t[:, None]
    cm = t.t().contiguous()          # row-major of t^T == column-major of t
    return cm, t.shape[0]


def shs_reduce(A, B, C, stream=None):
    """Controller-Hessenberg reduction of (A, B, C) (float64 CUDA tensors); returns a handle."""
    import torch
    lib = _load()
    for name, t in (("A", A), ("B", B), ("C", C)):
        if not (t.is_cuda and t.dtype == torch.float64):
            raise TypeError(f"{name} must be a float64 CUDA tensor")
    if B.dim() == 1:
        B = B[:, None]
    if C.dim() == 1:
        C = C[None, :]
    n, m = B.shape
    p = C.shape[0]
    Ac, lda = _colmajor(A)
    Bc, ldb = _colmajor(B)
    Cc, ldc = _colmajor(C) if p > 0 else (None, 1)
    cfg = _Config(abi_version=SHS_ABI_VERSION)
    h = ctypes.c_void_p()
    rc = lib.shs_reduce(n, m, p, _ptr(Ac), lda, _ptr(Bc), ldb, _ptr(Cc), max(1, ldc), ctypes.byref(cfg),
                        _stream(stream), ctypes.byref(h))
    _check("shs_reduce", rc)
    return h


def shs_solve_workspace(h, s, mode, outputs):
    lib = _load()
    b = ctypes.c_size_t()
    _check("shs_solve_workspace", lib.shs_solve_workspace(h, s, mode, outputs, ctypes.byref(b)))
    return b.value


def shs_solve(h, shifts, X, G, eta, status, mode=SHS_MODE_FP64, outputs=SHS_OUT_X | SHS_OUT_G,
              tol=1e-13, max_iter=5, work=None, stream=None):
    """Raw solve: every array is a caller-allocated CUDA tensor (see shiftsolve.h).

    ``X`` is a (s*m, n) complex128 tensor (column-major n x (s*m)), ``G`` a
    (s*m, p) complex128 tensor, ``eta`` (s,) float64, ``status`` (s,) int32,
    ``shifts`` (s,) complex128.
    """
    lib = _load()
    s = shifts.numel()
    ldx = X.shape[1] if X is not None else 1
    ldg = G.shape[1] if G is not None else 1
    wptr, wbytes = (_ptr(work), work.numel() * work.element_size()) if work is not None else (None, 0)
    rc = lib.shs_solve(h, s, _ptr(shifts), mode, outputs, tol, max_iter, wptr, wbytes,
                       _ptr(X), ldx, _ptr(G), ldg, _ptr(eta), _ptr(status), _stream(stream))
    _check("shs_solve", rc)


def shs_solve_noalloc(h, shifts, X, G, eta, status, mode=SHS_MODE_FP64, outputs=SHS_OUT_X | SHS_OUT_G,
                      tol=1e-13, max_iter=5, stream=None):
    """As :func:`shs_solve` with the library's static scratch as workspace
    (no device allocation); returns the library's code (0 or an error)."""
    s = shifts.numel()
    ldx = X.shape[1] if X is not None else 1
    ldg = G.shape[1] if G is not None else 1
    return _load().shs_solve_noalloc(h, s, _ptr(shifts), mode, outputs, tol, max_iter, _ptr(X), ldx, _ptr(G), ldg,
                                     _ptr(eta), _ptr(status), _stream(stream))


def shs_solve_transposed_workspace(h, s, r):
    b = ctypes.c_size_t()
    _check("shs_solve_transposed_workspace", _load().shs_solve_transposed_workspace(h, s, r, ctypes.byref(b)))
    return b.value


def shs_solve_transposed(h, shifts, r, D, X, eta, status, outputs=SHS_OUT_X | SHS_OUT_ETA, work=None, stream=None):
    """(H - sigma_j I)^T Y_j = D_j; ``D`` and ``X`` are (s*r, n) complex128
    tensors (column-major n x (s*r)), ``eta`` (s,) float64, ``status`` (s,) int32."""
    lib = _load()
    s = shifts.numel()
    wptr, wbytes = (_ptr(work), work.numel() * work.element_size()) if work is not None else (None, 0)
    ldx = X.shape[1] if X is not None else 1
    rc = lib.shs_solve_transposed(h, s, _ptr(shifts), r, _ptr(D), D.shape[1], outputs, wptr, wbytes, _ptr(X), ldx,
                                  _ptr(eta), _ptr(status), _stream(stream))
    _check("shs_solve_transposed", rc)


def shs_solve_vec_workspace(h, s):
    b = ctypes.c_size_t()
    _check("shs_solve_vec_workspace", _load().shs_solve_vec_workspace(h, s, ctypes.byref(b)))
    return b.value


def shs_solve_transposed_vec_workspace(h, s):
    b = ctypes.c_size_t()
    _check("shs_solve_transposed_vec_workspace", _load().shs_solve_transposed_vec_workspace(h, s, ctypes.byref(b)))
    return b.value


def _vec_call(name, h, shifts, dirs, X, eta, status, outputs, work, stream):
    s = shifts.numel()
    wptr, wbytes = (_ptr(work), work.numel() * work.element_size()) if work is not None else (None, 0)
    ldd = dirs.shape[1] if dirs is not None else 1
    rc = getattr(_load(), name)(h, s, _ptr(shifts), _ptr(dirs), max(1, ldd), outputs, wptr, wbytes, _ptr(X),
                                X.shape[1] if X is not None else 1, _ptr(eta), _ptr(status), _stream(stream))
    _check(name, rc)


def shs_solve_vec(h, shifts, bhat, X, eta, status, outputs=SHS_OUT_X | SHS_OUT_ETA, work=None, stream=None):
    """(H - sigma_j I) x_j = R b_j: ``bhat`` is an (s, m) complex128 tensor
    (column-major m x s), ``X`` (s, n) (column-major n x s)."""
    _vec_call("shs_solve_vec", h, shifts, bhat, X, eta, status, outputs, work, stream)


def shs_solve_transposed_vec(h, shifts, chat, X, eta, status, outputs=SHS_OUT_X | SHS_OUT_ETA, work=None,
                             stream=None):
    """(H - sigma_j I)^T w_j = Ct^T c_j: ``chat`` is an (s, p) complex128
    tensor (column-major p x s) or None when p = 0, ``X`` (s, n)."""
    _vec_call("shs_solve_transposed_vec", h, shifts, chat, X, eta, status, outputs, work, stream)


def shs_project(h, V, W, sel, Ar, Er, Br, Cr, rank_def, work=None, stream=None):
    """Projection onto the real bases of V, W ((r, n) complex128 tensors,
    column-major n x r); ``sel`` (r,) int32; outputs are (r, r), (r, r),
    (m, r), (r, p) float64 tensors (column-major r x r, r x r, r x m, p x r)
    and ``rank_def`` (1,) int32."""
    r = V.shape[0]
    wptr, wbytes = (_ptr(work), work.numel() * work.element_size()) if work is not None else (None, 0)
    rc = _load().shs_project(h, r, _ptr(V), V.shape[1], _ptr(W), W.shape[1], _ptr(sel), wptr, wbytes, _ptr(Ar),
                             _ptr(Er), _ptr(Br), _ptr(Cr), _ptr(rank_def), _stream(stream))
    _check("shs_project", rc)


def shs_transfer_norm2(G, m, norms, stream=None):
    """||G_j||_2 of every p x m block of G, a (s*m, p) complex128 tensor
    (column-major p x (s*m)), into ``norms`` ((s,) float64)."""
    s = G.shape[0] // m
    p = G.shape[1]
    _check("shs_transfer_norm2", _load().shs_transfer_norm2(s, p, m, _ptr(G), max(1, p), _ptr(norms),
                                                            _stream(stream)))


def shs_reduce_check_plan(n, m, p):
    """Host-only dry run of the reduction's launch plan: (violations, launches, first message)."""
    launches = ctypes.c_int64()
    msg = ctypes.create_string_buffer(256)
    rc = _load().shs_reduce_check_plan(n, m, p, ctypes.byref(launches), msg, 256)
    return rc, launches.value, msg.value.decode()


def shs_apply_q(h, Xred, Xorig, stream=None):
    """Xorig = Q Xred for (ncols, n) complex128 tensors (column-major n x ncols)."""
    lib = _load()
    ncols, n = Xred.shape
    _check("shs_apply_q", lib.shs_apply_q(h, ncols, _ptr(Xred), n, _ptr(Xorig), Xorig.shape[1],
                                          _stream(stream)))


def shs_get_reduced(h, H, R, Ct, stream=None):
    """Copy H (n, n), R (m, n), Ct (n, p) -- transposed storage of column-major arrays."""
    lib = _load()
    _check("shs_get_reduced", lib.shs_get_reduced(h, _ptr(H), H.shape[1] if H is not None else 1,
                                                  _ptr(R), R.shape[1] if R is not None else 1,
                                                  _ptr(Ct), Ct.shape[1] if Ct is not None else 1,
                                                  _stream(stream)))


def shs_info(h):
    lib = _load()
    info = _Info()
    _check("shs_info", lib.shs_info(h, ctypes.byref(info)))
    return {"n": info.n, "m": info.m, "p": info.p, "reduce_ms": info.reduce_ms,
            "resident_bytes": info.resident_bytes}


def shs_set_timing(h, enable: bool):
    _check("shs_set_timing", _load().shs_set_timing(h, 1 if enable else 0))


def shs_last_timings(h):
    """Per-phase device time (ms) and counters of the last solve on the handle."""
    t = _Timings()
    _check("shs_last_timings", _load().shs_last_timings(h, ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in _Timings._fields_}


def shs_destroy(h):
    _load().shs_destroy(h)


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

def shs_server_create(streams=4, budget_bytes=64 << 30, max_batch=64, blocked_flops=0.0):
    lib = _load()
    cfg = _ServerConfig(abi_version=SHS_ABI_VERSION, streams=streams, budget_bytes=budget_bytes,
                        max_batch=max_batch, blocked_flops=blocked_flops)
    srv = ctypes.c_void_p()
    _check("shs_server_create", lib.shs_server_create(ctypes.byref(cfg), ctypes.byref(srv)))
    return srv


def shs_server_register(srv, h):
    sid = ctypes.c_int32()
    _check("shs_server_register", _load().shs_server_register(srv, h, ctypes.byref(sid)))
    return sid.value


def shs_server_submit(srv, sys_id, shifts_host, X, G, eta, status, mode=SHS_MODE_FP64,
                      outputs=SHS_OUT_X | SHS_OUT_G):
    """Queue a request; shifts_host is a 1-D complex128 NumPy array (copied)."""
    import numpy as np
    sh = np.ascontiguousarray(np.asarray(shifts_host, dtype=np.complex128).reshape(-1))
    rid = ctypes.c_int64()
    ldx = X.shape[1] if X is not None else 1
    ldg = G.shape[1] if G is not None else 1
    rc = _load().shs_server_submit(srv, sys_id, sh.size, sh.ctypes.data_as(ctypes.c_void_p), mode, outputs,
                                   _ptr(X), ldx, _ptr(G), ldg, _ptr(eta), _ptr(status), ctypes.byref(rid))
    _check("shs_server_submit", rc)
    return rid.value


def shs_server_submit_ex(srv, sys_id, shifts_host, X, G, eta, status, mode=SHS_MODE_FP64,
                         outputs=SHS_OUT_X | SHS_OUT_G, after_stream=None, order_after=True, arrival_s=0.0):
    """Queue a request whose work is ordered after ``after_stream`` (a torch
    stream; None = the current stream) and whose latency runs from
    ``arrival_s`` on the :func:`shs_server_clock` clock (0 = now)."""
    import numpy as np
    sh = np.ascontiguousarray(np.asarray(shifts_host, dtype=np.complex128).reshape(-1))
    opts = _RequestOpts(abi_version=SHS_ABI_VERSION, order_after=1 if order_after else 0,
                        after_stream=_stream(after_stream) if order_after else None, arrival_s=float(arrival_s))
    rid = ctypes.c_int64()
    ldx = X.shape[1] if X is not None else 1
    ldg = G.shape[1] if G is not None else 1
    rc = _load().shs_server_submit_ex(srv, sys_id, sh.size, sh.ctypes.data_as(ctypes.c_void_p), mode, outputs,
                                      _ptr(X), ldx, _ptr(G), ldg, _ptr(eta), _ptr(status), ctypes.byref(opts),
                                      ctypes.byref(rid))
    _check("shs_server_submit_ex", rc)
    return rid.value


def shs_server_cancel(srv, req_id):
    _check("shs_server_cancel", _load().shs_server_cancel(srv, req_id))


def shs_server_pause(srv, paused: bool):
    _check("shs_server_pause", _load().shs_server_pause(srv, 1 if paused else 0))


def shs_server_clock() -> float:
    """The server's steady clock in seconds (for request arrival times)."""
    return float(_load().shs_server_clock())


def shs_server_poll(srv, req_id):
    st = ctypes.c_int()
    _check("shs_server_poll", _load().shs_server_poll(srv, req_id, ctypes.byref(st)))
    return st.value


def shs_server_wait(srv, req_id, timeout_ms=-1.0):
    _check("shs_server_wait", _load().shs_server_wait(srv, req_id, float(timeout_ms)))


def shs_server_latency(srv, req_id):
    ms = ctypes.c_double()
    _check("shs_server_latency", _load().shs_server_latency(srv, req_id, ctypes.byref(ms)))
    return ms.value


def shs_server_stats(srv):
    st = _ServerStats()
    _check("shs_server_stats", _load().shs_server_stats(srv, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in _ServerStats._fields_}


def shs_server_destroy(srv):
    _load().shs_server_destroy(srv)
