"""Thin ctypes binding of liblupp (the C ABI declared in include/lupp.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of liblupp.so. Tensors are passed by device pointer
(``tensor.data_ptr()``) and streams by handle
(``torch.cuda.current_stream().cuda_stream``). PyTorch is used for device
memory and streams only.

The library must have been built (``python -m paper_2609_15217_amd.build``);
importing this module without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime the library then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblupp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_15217_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

LUPP_AOS, LUPP_SOA = 0, 1
LUPP_KEEP_A = 1
LUPP_FMA = 4
LUPP_RAGGED_PER_SIZE = 2
LUPP_VARIANT_AUTO, LUPP_VARIANT_THREAD, LUPP_VARIANT_LANES = 0, 1, 2
LUPP_LAW_NORTON7, LUPP_LAW_NORTON_AF13 = 7, 13
LUPP_E_UNSUPPORTED, LUPP_E_NOMEM, LUPP_E_TOO_LARGE, LUPP_E_HIP_BASE = -900, -901, -902, -1000
LUPP_NOALLOC_MAX_BATCH = 4194304

_P = ctypes.c_void_p
_i64 = ctypes.c_int64


class lupp_law(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("E", ctypes.c_double), ("nu", ctypes.c_double),
                ("A", ctypes.c_double), ("m", ctypes.c_double), ("C", ctypes.c_double),
                ("D", ctypes.c_double), ("dt", ctypes.c_double)]


class lupp_group(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("batch", ctypes.c_int64), ("A", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("strideA", ctypes.c_int64), ("b", ctypes.c_void_p),
                ("strideB", ctypes.c_int64), ("ipiv", ctypes.c_void_p), ("info", ctypes.c_void_p)]


class lupp_points(ctypes.Structure):
    _fields_ = [("count", _i64), ("ld", _i64), ("deps", _P), ("state", _P), ("sig", _P),
                ("iters", _P), ("status", _P), ("tangent", _P)]


class lupp_kernel_info(ctypes.Structure):
    _fields_ = [("vgprs", ctypes.c_int), ("agprs", ctypes.c_int), ("sgprs", ctypes.c_int),
                ("scratch_bytes", ctypes.c_int), ("lds_bytes", ctypes.c_int),
                ("max_threads", ctypes.c_int)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_lupp_create = _sig("lupp_create", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int])
_lupp_destroy = _sig("lupp_destroy", None, [_P])
_lupp_batched_solve = _sig("lupp_batched_solve", ctypes.c_int,
                           [_P, ctypes.c_int, _i64, ctypes.c_int, _P, _i64, _i64, _P, _i64, _P, _P,
                            ctypes.c_uint, _P])
_lupp_batched_solve_ragged = _sig("lupp_batched_solve_ragged", ctypes.c_int,
                                  [_P, _i64, _P, _P, _P, _P, _P, _P, _P, ctypes.c_uint, _P])
_lupp_batched_solve_grouped = _sig("lupp_batched_solve_grouped", ctypes.c_int,
                                   [_P, ctypes.c_int, ctypes.POINTER(lupp_group), ctypes.c_uint, _P])
_lupp_batched_solve_ragged_noalloc = _sig("lupp_batched_solve_ragged_noalloc", ctypes.c_int,
                                          [_P, _i64, _P, _P, _P, _P, _P, _P, _P, ctypes.c_uint, _P])
_lupp_force_variant = _sig("lupp_force_variant", ctypes.c_int,
                           [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int])
_lupp_set_dispatch = _sig("lupp_set_dispatch", ctypes.c_int,
                          [_P, ctypes.c_int, ctypes.c_int, _i64, ctypes.c_int, ctypes.c_int,
                           ctypes.c_int])
_lupp_get_dispatch = _sig("lupp_get_dispatch", ctypes.c_int,
                          [_P, ctypes.c_int, ctypes.c_int, _i64, ctypes.POINTER(ctypes.c_int),
                           ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)])
_lupp_variant_info = _sig("lupp_variant_info", ctypes.c_int,
                          [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                           ctypes.POINTER(lupp_kernel_info)])
_constitutive_update = _sig("constitutive_update", ctypes.c_int,
                            [_P, ctypes.POINTER(lupp_points), ctypes.POINTER(lupp_law),
                             ctypes.c_double, ctypes.c_int, _P])
_lupp_error_string = _sig("lupp_error_string", ctypes.c_char_p, [ctypes.c_int])
_lupp_autotune = _sig("lupp_autotune", ctypes.c_int,
                      [_P, ctypes.c_int, _i64, ctypes.c_int, _P, _i64, _i64, _P, _i64, ctypes.c_int,
                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float), _P])
_lupp_ragged_lanes_supported = _sig("lupp_ragged_lanes_supported", ctypes.c_int,
                                    [ctypes.c_int, ctypes.c_int])
_lupp_set_ragged_lanes = _sig("lupp_set_ragged_lanes", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int])
_lupp_get_ragged_lanes = _sig("lupp_get_ragged_lanes", ctypes.c_int, [_P, ctypes.c_int])
_lupp_autotune_ragged = _sig("lupp_autotune_ragged", ctypes.c_int,
                             [_P, ctypes.c_int, _i64, _P, _P, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float), _P])
_lupp_check_solve_args = _sig("lupp_check_solve_args", ctypes.c_int,
                              [ctypes.c_int, _i64, ctypes.c_int, _P, _i64, _i64, _P, _i64, _P, _P,
                               ctypes.c_uint])

class lupp_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", _i64), ("max_inflight", ctypes.c_int), ("streams", ctypes.c_int),
                ("mode", ctypes.c_int)]


class lupp_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n", ctypes.c_int), ("batch", _i64), ("A", _P), ("b", _P),
                ("x", _P), ("ipiv", _P), ("info", _P), ("lu", _P), ("set_id", _i64),
                ("count", _i64), ("law", ctypes.POINTER(lupp_law)), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("deps", _P), ("sig", _P), ("iters", _P), ("status", _P),
                ("tangent", _P)]


class lupp_server_stats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("rejected", _i64), ("failed", _i64),
                ("queued", _i64), ("inflight", ctypes.c_int), ("peak_inflight", ctypes.c_int),
                ("peak_bytes", _i64), ("budget_bytes", _i64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("elapsed_s", ctypes.c_double), ("passes", _i64), ("launches", _i64)]


_lupp_get_device = _sig("lupp_get_device", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int)])
_lupp_server_create = _sig("lupp_server_create", ctypes.c_int,
                           [_P, ctypes.POINTER(lupp_server_config), ctypes.POINTER(_P)])
_lupp_server_destroy = _sig("lupp_server_destroy", None, [_P])
_lupp_server_add_points = _sig("lupp_server_add_points", ctypes.c_int,
                               [_P, ctypes.c_int, _i64, _P, ctypes.POINTER(_i64)])
_lupp_server_read_points = _sig("lupp_server_read_points", ctypes.c_int, [_P, _i64, _P])
_lupp_server_submit = _sig("lupp_server_submit", _i64, [_P, ctypes.POINTER(lupp_request)])
_lupp_server_poll = _sig("lupp_server_poll", ctypes.c_int, [_P, _i64])
_lupp_server_wait = _sig("lupp_server_wait", ctypes.c_int, [_P, _i64, ctypes.POINTER(ctypes.c_double)])
_lupp_server_get_stats = _sig("lupp_server_get_stats", ctypes.c_int,
                              [_P, ctypes.POINTER(lupp_server_stats)])
_lupp_server_reset_stats = _sig("lupp_server_reset_stats", ctypes.c_int, [_P])

EXPORTED = ["lupp_create", "lupp_destroy", "lupp_batched_solve", "lupp_batched_solve_ragged",
            "lupp_force_variant", "lupp_set_dispatch", "lupp_get_dispatch", "lupp_variant_info",
            "constitutive_update", "lupp_error_string", "lupp_check_solve_args",
            "lupp_autotune", "lupp_get_device", "lupp_server_create", "lupp_server_destroy",
            "lupp_server_add_points", "lupp_server_read_points", "lupp_server_submit",
            "lupp_server_poll", "lupp_server_wait", "lupp_server_get_stats",
            "lupp_server_reset_stats", "lupp_sweep_create", "lupp_sweep_launch",
            "lupp_sweep_destroy", "constitutive_update_batched", "lupp_set_newton_variant",
            "lupp_get_newton_variant", "lupp_set_pivoting", "lupp_get_pivoting",
            "lupp_ragged_lanes_supported", "lupp_set_ragged_lanes", "lupp_get_ragged_lanes",
            "lupp_autotune_ragged", "lupp_batched_solve_ragged_noalloc",
            "lupp_batched_solve_grouped"]


class LuppError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {lupp_error_string(code)} (code {code})")
        self.code = code


def _check(rc: int, what: str) -> int:
    if rc != 0:
        raise LuppError(rc, what)
    return rc


def _ptr(x) -> _P:
    """Device or host address of a torch tensor, numpy array or raw int."""
    if x is None:
        return _P(0)
    if isinstance(x, int):
        return _P(x)
    if hasattr(x, "data_ptr"):
        return _P(x.data_ptr())
    return _P(x.ctypes.data)


def _stream(stream) -> _P:
    if stream is None:
        return _P(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _P(stream)
    return _P(stream.cuda_stream)


def lupp_error_string(code: int) -> str:
    return _lupp_error_string(code).decode()


class Context:
    """Owns a lupp_ctx (dispatch table, device workspace) for one device."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        h = _P()
        _check(_lupp_create(ctypes.byref(h), device), "lupp_create")
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _lupp_destroy(self.handle)
            self.handle = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lupp_create(device: int | None = None) -> Context:
    return Context(device)


def lupp_destroy(ctx: Context):
    ctx.close()


def lupp_batched_solve(ctx: Context, n: int, batch: int, layout: int, A, lda: int, strideA: int,
                       b, strideB: int, ipiv, info, flags: int = 0, stream=None) -> int:
    """Raw C-ABI call: returns the library's code (0, -k, LUPP_E_*)."""
    return _lupp_batched_solve(ctx.handle, n, batch, layout, _ptr(A), lda, strideA, _ptr(b),
                               strideB, _ptr(ipiv), _ptr(info), flags, _stream(stream))


def lupp_batched_solve_ragged(ctx: Context, batch: int, n, offA, offB, A, b, ipiv, info,
                              flags: int = 0, stream=None) -> int:
    return _lupp_batched_solve_ragged(ctx.handle, batch, _ptr(n), _ptr(offA), _ptr(offB), _ptr(A),
                                      _ptr(b), _ptr(ipiv), _ptr(info), flags, _stream(stream))


def group(n: int, batch: int, A, b, ipiv, info, lda: int | None = None,
          strideA: int | None = None, strideB: int | None = None) -> lupp_group:
    """One AoS group descriptor (packed strides by default)."""
    lda = n if lda is None else lda
    return lupp_group(n, batch, _ptr(A).value, lda, lda * n if strideA is None else strideA,
                      _ptr(b).value, n if strideB is None else strideB, _ptr(ipiv).value,
                      _ptr(info).value)


def lupp_batched_solve_grouped(ctx: Context, groups, flags: int = 0, stream=None) -> int:
    """groups: a sequence of lupp_group (or None with ngroups 0)."""
    n = len(groups) if groups is not None else 0
    arr = (lupp_group * max(n, 1))(*groups) if n else None
    return _lupp_batched_solve_grouped(ctx.handle, n, arr, flags, _stream(stream))


def lupp_batched_solve_ragged_noalloc(ctx: Context, batch: int, n, offA, offB, A, b, ipiv, info,
                                      flags: int = 0, stream=None) -> int:
    return _lupp_batched_solve_ragged_noalloc(ctx.handle, batch, _ptr(n), _ptr(offA), _ptr(offB),
                                              _ptr(A), _ptr(b), _ptr(ipiv), _ptr(info), flags,
                                              _stream(stream))


def lupp_check_solve_args(n: int, batch: int, layout: int, A, lda: int, strideA: int, b,
                          strideB: int, ipiv, info, flags: int = 0) -> int:
    return _lupp_check_solve_args(n, batch, layout, _ptr(A), lda, strideA, _ptr(b), strideB,
                                  _ptr(ipiv), _ptr(info), flags)


def lupp_autotune(ctx: Context, n: int, batch: int, layout: int, A, lda: int, strideA: int, b,
                  strideB: int, reps: int = 5, stream=None):
    """Returns (rc, variant, lanes, wpb, ms)."""
    v, l, w, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    rc = _lupp_autotune(ctx.handle, n, batch, layout, _ptr(A), lda, strideA, _ptr(b), strideB, reps,
                        ctypes.byref(v), ctypes.byref(l), ctypes.byref(w), ctypes.byref(ms),
                        _stream(stream))
    return rc, v.value, l.value, w.value, ms.value


def lupp_ragged_lanes_supported(n: int, lanes: int) -> int:
    return _lupp_ragged_lanes_supported(n, lanes)


def lupp_set_ragged_lanes(ctx: Context, n: int, lanes: int) -> int:
    return _lupp_set_ragged_lanes(ctx.handle, n, lanes)


def lupp_get_ragged_lanes(ctx: Context, n: int) -> int:
    return _lupp_get_ragged_lanes(ctx.handle, n)


def lupp_autotune_ragged(ctx: Context, n: int, batch: int, A, b, reps: int = 5, stream=None):
    """Returns (rc, lanes, ms)."""
    l, ms = ctypes.c_int(), ctypes.c_float()
    rc = _lupp_autotune_ragged(ctx.handle, n, batch, _ptr(A), _ptr(b), reps, ctypes.byref(l),
                               ctypes.byref(ms), _stream(stream))
    return rc, l.value, ms.value


def lupp_force_variant(ctx: Context, variant: int, lanes: int = 0, wpb: int = 0) -> int:
    return _lupp_force_variant(ctx.handle, variant, lanes, wpb)


def lupp_set_dispatch(ctx: Context, n: int, layout: int, batch: int, variant: int, lanes: int,
                      wpb: int) -> int:
    return _lupp_set_dispatch(ctx.handle, n, layout, batch, variant, lanes, wpb)


def lupp_get_dispatch(ctx: Context, n: int, layout: int, batch: int = 1 << 20):
    v, l, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_lupp_get_dispatch(ctx.handle, n, layout, batch, ctypes.byref(v), ctypes.byref(l),
                              ctypes.byref(w)), "lupp_get_dispatch")
    return v.value, l.value, w.value


def lupp_variant_info(n: int, layout: int, variant: int, lanes: int = 0, keep_a: int = 0):
    out = lupp_kernel_info()
    rc = _lupp_variant_info(n, layout, variant, lanes, keep_a, ctypes.byref(out))
    if rc != 0:
        return None
    return {f: getattr(out, f) for f, _ in lupp_kernel_info._fields_}


def constitutive_update(ctx: Context, pts: lupp_points, law: lupp_law, tol: float, maxit: int,
                        stream=None) -> int:
    return _constitutive_update(ctx.handle, ctypes.byref(pts), ctypes.byref(law), tol, maxit,
                                _stream(stream))


_lupp_set_pivoting = _sig("lupp_set_pivoting", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double])
_lupp_get_pivoting = _sig("lupp_get_pivoting", ctypes.c_int,
                          [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)])


def lupp_set_pivoting(ctx: Context, tile: int, threshold: float = 1e-10) -> int:
    return _lupp_set_pivoting(ctx.handle, tile, threshold)


def lupp_get_pivoting(ctx: Context):
    t, th = ctypes.c_int(0), ctypes.c_double(0.0)
    rc = _lupp_get_pivoting(ctx.handle, ctypes.byref(t), ctypes.byref(th))
    return rc, t.value, th.value


_lupp_set_newton_variant = _sig("lupp_set_newton_variant", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int])
_lupp_get_newton_variant = _sig("lupp_get_newton_variant", ctypes.c_int,
                                [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)])


def lupp_set_newton_variant(ctx: Context, kind: int, lanes: int) -> int:
    return _lupp_set_newton_variant(ctx.handle, kind, lanes)


def lupp_get_newton_variant(ctx: Context, kind: int):
    v = ctypes.c_int(0)
    rc = _lupp_get_newton_variant(ctx.handle, kind, ctypes.byref(v))
    return rc, v.value


LUPP_BATCHED_GRAPH = 1
_constitutive_update_batched = _sig("constitutive_update_batched", ctypes.c_int,
                                    [_P, ctypes.POINTER(lupp_points), ctypes.POINTER(lupp_law),
                                     ctypes.c_double, ctypes.c_int, ctypes.c_uint, _P,
                                     ctypes.POINTER(ctypes.c_int)])


def constitutive_update_batched(ctx: Context, pts: lupp_points, law: lupp_law, tol: float,
                                maxit: int, flags: int = 0, stream=None):
    """Returns (rc, host-driven iterations)."""
    k = ctypes.c_int(0)
    rc = _constitutive_update_batched(ctx.handle, ctypes.byref(pts), ctypes.byref(law), tol, maxit,
                                      flags, _stream(stream), ctypes.byref(k))
    return rc, k.value


# --------------------------------------------------------------------------
# Time-step sweeps captured in a HIP graph
# --------------------------------------------------------------------------
_lupp_sweep_create = _sig("lupp_sweep_create", ctypes.c_int,
                          [_P, ctypes.POINTER(lupp_points), ctypes.POINTER(lupp_law),
                           ctypes.c_double, ctypes.c_int, ctypes.c_int, _i64, ctypes.POINTER(_P)])
_lupp_sweep_launch = _sig("lupp_sweep_launch", ctypes.c_int, [_P, _P])
_lupp_sweep_destroy = _sig("lupp_sweep_destroy", None, [_P])


class Sweep:
    """Owns a lupp_sweep (an instantiated HIP graph of `steps` updates)."""

    def __init__(self, ctx: Context, pts: lupp_points, law: lupp_law, tol: float, maxit: int,
                 steps: int, deps_step: int):
        h = _P()
        _check(_lupp_sweep_create(ctx.handle, ctypes.byref(pts), ctypes.byref(law), tol, maxit,
                                  steps, deps_step, ctypes.byref(h)), "lupp_sweep_create")
        self.handle = h

    def launch(self, stream=None) -> int:
        return _lupp_sweep_launch(self.handle, _stream(stream))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _lupp_sweep_destroy(self.handle)
            self.handle = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lupp_sweep_create(ctx: Context, pts: lupp_points, law: lupp_law, tol: float, maxit: int,
                      steps: int, deps_step: int) -> Sweep:
    return Sweep(ctx, pts, law, tol, maxit, steps, deps_step)


def lupp_sweep_launch(sweep: Sweep, stream=None) -> int:
    return sweep.launch(stream)


def lupp_sweep_destroy(sweep: Sweep):
    sweep.close()


# --------------------------------------------------------------------------
# Tensor-level helpers (marshalling only)
# --------------------------------------------------------------------------
def batched_solve(ctx: Context, A: torch.Tensor, b: torch.Tensor, layout: int = LUPP_AOS,
                  keep_a: bool = False, ipiv: torch.Tensor | None = None,
                  info: torch.Tensor | None = None, stream=None):
    """In-place batched solve of device tensors.
    AoS: A (batch, n, n) read [s][j][i] (column-major per system), b (batch, n).
    SoA: A (n, n, batch) read [j][i][s], b (n, batch).
    Returns (ipiv, info) int32 device tensors in the matching layout."""
    assert A.is_cuda and A.dtype == torch.float64 and A.is_contiguous()
    assert b.is_cuda and b.dtype == torch.float64 and b.is_contiguous()
    if layout == LUPP_AOS:
        batch, n = A.shape[0], A.shape[1]
        sA, sB = n * n, n
        pshape = (batch, n)
    else:
        n, batch = A.shape[0], A.shape[2]
        sA, sB = batch, batch
        pshape = (n, batch)
    if ipiv is None:
        ipiv = torch.empty(pshape, dtype=torch.int32, device=A.device)
    if info is None:
        info = torch.empty(batch, dtype=torch.int32, device=A.device)
    rc = lupp_batched_solve(ctx, n, batch, layout, A, n, sA, b, sB, ipiv, info,
                            LUPP_KEEP_A if keep_a else 0, stream)
    _check(rc, "lupp_batched_solve")
    return ipiv, info


def make_law(kind: int = 7, E=200e3, nu=0.3, A=1e-8, m=5.0, C=1e4, D=100.0, dt=1e-2) -> lupp_law:
    return lupp_law(kind, E, nu, A, m, C, D, dt)


def points(deps: torch.Tensor, state: torch.Tensor, sig: torch.Tensor, iters: torch.Tensor,
           status: torch.Tensor, tangent: torch.Tensor | None = None) -> lupp_points:
    """SoA point buffers: deps (6, ld), state (kind, ld), sig (6, ld),
    iters/status (count,) int32, optional tangent (36, ld)."""
    count = iters.shape[0]
    ld = deps.shape[1]
    bufs = (deps, state, sig) if tangent is None else (deps, state, sig, tangent)
    for t in bufs:
        assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.shape[1] == ld
    return lupp_points(count, ld, deps.data_ptr(), state.data_ptr(), sig.data_ptr(),
                       iters.data_ptr(), status.data_ptr(),
                       None if tangent is None else tangent.data_ptr())


# --------------------------------------------------------------------------
# Serving loop
# --------------------------------------------------------------------------
LUPP_REQ_SOLVE, LUPP_REQ_UPDATE = 1, 2
LUPP_SERVE_MERGED, LUPP_SERVE_PER_REQUEST = 0, 1


def lupp_get_device(ctx: Context) -> int:
    d = ctypes.c_int()
    _check(_lupp_get_device(ctx.handle, ctypes.byref(d)), "lupp_get_device")
    return d.value


class Server:
    """Owns a lupp_server (device arena, streams, scheduler thread)."""

    def __init__(self, ctx: Context, budget_bytes: int = 0, max_inflight: int = 8, streams: int = 4,
                 mode: int = 0):
        cfg = lupp_server_config(budget_bytes, max_inflight, streams, mode)
        h = _P()
        _check(_lupp_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)), "lupp_server_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _lupp_server_destroy(self.handle)
            self.handle = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lupp_server_create(ctx: Context, budget_bytes: int = 0, max_inflight: int = 8,
                       streams: int = 4, mode: int = 0) -> Server:
    return Server(ctx, budget_bytes, max_inflight, streams, mode)


def lupp_server_destroy(server: Server):
    server.close()


def lupp_server_add_points(server: Server, kind: int, count: int, state=None) -> int:
    sid = _i64()
    _check(_lupp_server_add_points(server.handle, kind, count, _ptr(state), ctypes.byref(sid)),
           "lupp_server_add_points")
    return sid.value


def lupp_server_read_points(server: Server, set_id: int, out) -> int:
    return _lupp_server_read_points(server.handle, set_id, _ptr(out))


def solve_request(n: int, batch: int, A, b, x, ipiv=None, info=None, lu=None) -> lupp_request:
    r = lupp_request()
    r.kind, r.n, r.batch = LUPP_REQ_SOLVE, n, batch
    r.A, r.b, r.x = _ptr(A), _ptr(b), _ptr(x)
    r.ipiv, r.info, r.lu = _ptr(ipiv), _ptr(info), _ptr(lu)
    return r


def update_request(set_id: int, count: int, law: lupp_law, deps, sig=None, iters=None, status=None,
                   tol: float = 1e-12, maxit: int = 20, tangent=None) -> lupp_request:
    r = lupp_request()
    r.kind, r.set_id, r.count = LUPP_REQ_UPDATE, set_id, count
    r.law = ctypes.pointer(law)
    r.tol, r.maxit = tol, maxit
    r.deps, r.sig, r.iters, r.status = _ptr(deps), _ptr(sig), _ptr(iters), _ptr(status)
    r.tangent = _ptr(tangent)
    return r


def lupp_server_submit(server: Server, req: lupp_request) -> int:
    return _lupp_server_submit(server.handle, ctypes.byref(req))


def lupp_server_poll(server: Server, ticket: int) -> int:
    return _lupp_server_poll(server.handle, ticket)


def lupp_server_wait(server: Server, ticket: int):
    lat = ctypes.c_double()
    rc = _lupp_server_wait(server.handle, ticket, ctypes.byref(lat))
    return rc, lat.value


def lupp_server_get_stats(server: Server) -> dict:
    st = lupp_server_stats()
    _check(_lupp_server_get_stats(server.handle, ctypes.byref(st)), "lupp_server_get_stats")
    return {f: getattr(st, f) for f, _ in lupp_server_stats._fields_}


def lupp_server_reset_stats(server: Server) -> int:
    return _lupp_server_reset_stats(server.handle)
