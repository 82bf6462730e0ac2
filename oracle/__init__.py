"""CPU oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct FP64 implementation of what the HIP path
computes: textbook LU with partial pivoting and triangular solves (Section 2.2
of the paper) and the per-point Newton constitutive update (Section 2.1,
Algorithm 2), in C (``lupp_oracle.c``), wrapped here with ctypes.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. It shares no code with the HIP path and never
imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
# A different build of the same source (the mutation tests load planted-mistake
# copies through this variable).
_SO_OVERRIDE = os.environ.get("ORACLE_SO")
_SRC = os.path.join(_HERE, "lupp_oracle.c")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build() -> str:
    """Compile liboracle.so with gcc (no FMA contraction, no fast-math)."""
    tmp = _SO + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm", "-lpthread"], check=True)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _SO_OVERRIDE:
            L = ctypes.CDLL(_SO_OVERRIDE)
        else:
            if not os.path.exists(_SO):
                build()
            L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.oracle_getrf.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P]
        L.oracle_getrf.restype = ctypes.c_int
        L.oracle_getrs.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P]
        L.oracle_getrs.restype = None
        L.oracle_gesv.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, P]
        L.oracle_gesv.restype = ctypes.c_int
        L.oracle_gesv_batch.argtypes = [ctypes.c_int, i64, P, ctypes.c_int, i64, P, i64, P, P, P,
                                        ctypes.c_int]
        L.oracle_gesv_batch.restype = None
        L.oracle_gesv_batch_mode.argtypes = [ctypes.c_int, i64, P, ctypes.c_int, i64, P, i64, P,
                                             P, ctypes.c_int, ctypes.c_double, ctypes.c_int, P,
                                             ctypes.c_int]
        L.oracle_gesv_batch_mode.restype = None
        L.oracle_gesv_ragged.argtypes = [i64, P, P, P, P, P, P, P, ctypes.c_int]
        L.oracle_gesv_ragged.restype = None
        L.oracle_law_eval.argtypes = [P, P, P, P, P, P, P]
        L.oracle_law_eval.restype = None
        L.oracle_constitutive_update.argtypes = [P, i64, P, P, P, P, P, P, P, P,
                                                 ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.oracle_constitutive_update.restype = None
        _ = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------------------
# LU with partial pivoting
# --------------------------------------------------------------------------
def getrf(A: np.ndarray):
    """Factor one matrix given as an (n, n) array read [j][i] (column-major).
    Returns (LU in the same layout, ipiv (1-based int32), info, pivot gap)."""
    a = _f64(A).copy()
    n = a.shape[0]
    ipiv = np.zeros(n, dtype=np.int32)
    gap = np.zeros(1)
    info = lib().oracle_getrf(n, _p(a), n, _p(ipiv), _p(gap))
    return a, ipiv, int(info), float(gap[0])


def getrs(LU: np.ndarray, ipiv: np.ndarray, b: np.ndarray) -> np.ndarray:
    lu = _f64(LU)
    x = _f64(b).copy()
    iv = np.ascontiguousarray(ipiv, dtype=np.int32)
    lib().oracle_getrs(lu.shape[0], _p(lu), lu.shape[0], _p(iv), _p(x))
    return x


def gesv_batch(A: np.ndarray, b: np.ndarray, threads: int | None = None, want_gap=False):
    """Solve a batch in AoS layout: A (batch, n, n) [s][j][i], b (batch, n).
    Returns dict(LU, x, ipiv, info[, gap]); inputs are not modified."""
    a = _f64(A).copy()
    x = _f64(b).copy()
    batch, n = a.shape[0], a.shape[1]
    ipiv = np.zeros((batch, n), dtype=np.int32)
    info = np.zeros(batch, dtype=np.int32)
    gap = np.zeros(batch) if want_gap else None
    lib().oracle_gesv_batch(n, batch, _p(a), n, n * n, _p(x), n, _p(ipiv), _p(info), _p(gap),
                            threads or default_threads())
    out = {"LU": a, "x": x, "ipiv": ipiv, "info": info}
    if want_gap:
        out["gap"] = gap
    return out


def gesv_batch_mode(A: np.ndarray, b: np.ndarray, tile: int = 0, thresh: float = 1e-10,
                    fma: bool = False, threads: int | None = None):
    """Batched dgesv under a pivoting rule (tile 0: textbook; else tile-local
    with acceptance threshold `thresh`) and arithmetic mode (fma: every
    multiply-subtract fused). Returns dict(LU, x, ipiv, info, out_of_tile)."""
    a = _f64(A).copy()
    x = _f64(b).copy()
    batch, n = a.shape[0], a.shape[1]
    ipiv = np.zeros((batch, n), dtype=np.int32)
    info = np.zeros(batch, dtype=np.int32)
    oot = np.zeros(batch, dtype=np.int32)
    lib().oracle_gesv_batch_mode(n, batch, _p(a), n, n * n, _p(x), n, _p(ipiv), _p(info), tile,
                                 thresh if tile else 0.0, 1 if fma else 0, _p(oot),
                                 threads or default_threads())
    return {"LU": a, "x": x, "ipiv": ipiv, "info": info, "out_of_tile": oot}


def gesv_batch_tiled(A: np.ndarray, b: np.ndarray, tile: int, thresh: float = 1e-10,
                     threads: int | None = None):
    """Batched dgesv with tile-local pivoting (strict arithmetic)."""
    return gesv_batch_mode(A, b, tile, thresh, False, threads)


def gesv_ragged(n: np.ndarray, offA: np.ndarray, offB: np.ndarray, A: np.ndarray,
                b: np.ndarray, threads: int | None = None):
    a = _f64(A).copy()
    x = _f64(b).copy()
    nn = np.ascontiguousarray(n, dtype=np.int32)
    oa = np.ascontiguousarray(offA, dtype=np.int64)
    ob = np.ascontiguousarray(offB, dtype=np.int64)
    ipiv = np.zeros(x.size, dtype=np.int32)
    info = np.zeros(nn.size, dtype=np.int32)
    lib().oracle_gesv_ragged(nn.size, _p(nn), _p(oa), _p(ob), _p(a), _p(x), _p(ipiv), _p(info),
                             threads or default_threads())
    return {"LU": a, "x": x, "ipiv": ipiv, "info": info}


# --------------------------------------------------------------------------
# Constitutive update
# --------------------------------------------------------------------------
class _CLaw(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("E", ctypes.c_double), ("nu", ctypes.c_double),
                ("A", ctypes.c_double), ("m", ctypes.c_double), ("C", ctypes.c_double),
                ("D", ctypes.c_double), ("dt", ctypes.c_double)]


@dataclass
class Law:
    """Norton (kind 7) or Norton + Armstrong-Frederick (kind 13) parameters."""
    kind: int = 7
    E: float = 200e3
    nu: float = 0.3
    A: float = 1e-8
    m: float = 5.0
    C: float = 1e4
    D: float = 100.0
    dt: float = 1e-2

    def c(self) -> _CLaw:
        return _CLaw(self.kind, self.E, self.nu, self.A, self.m, self.C, self.D, self.dt)


def law_eval(law: Law, deps, state_t, y):
    nunk = law.kind
    F = np.zeros(nunk)
    J = np.zeros(nunk * nunk)
    sig = np.zeros(6)
    cl = law.c()
    lib().oracle_law_eval(ctypes.byref(cl), _p(_f64(deps)), _p(_f64(state_t)), _p(_f64(y)),
                          _p(F), _p(J), _p(sig))
    return F, J.reshape(nunk, nunk).T.copy(), sig  # J returned as J[r, c]


def constitutive_update(law: Law, deps: np.ndarray, state: np.ndarray | None = None,
                        tol: float = 1e-12, maxit: int = 20, threads: int | None = None,
                        tangent: bool = False, want_y: bool = False):
    """Newton update of every point. deps (count, 6); state (count, kind) or None
    for the virgin state. Returns dict(sig, state, iters, status, resid), plus
    tangent (count, 6, 6) = dsig/d(deps) at converged points (NaN elsewhere)
    when tangent=True, and y (count, kind) = the unknowns of the returned
    iterate when want_y=True (with tol = 0 every point stops after exactly
    maxit solves, unless a zero pivot or a non-finite residual stops it
    earlier)."""
    d = _f64(deps)
    count = d.shape[0]
    st = np.zeros((count, law.kind)) if state is None else _f64(state).copy()
    sig = np.zeros((count, 6))
    iters = np.zeros(count, dtype=np.int32)
    status = np.zeros(count, dtype=np.int32)
    resid = np.zeros(count)
    tan = np.full((count, 6, 6), np.nan) if tangent else None
    y = np.full((count, law.kind), np.nan) if want_y else None
    cl = law.c()
    lib().oracle_constitutive_update(ctypes.byref(cl), count, _p(d), _p(st), _p(sig), _p(iters),
                                     _p(status), _p(resid), _p(tan) if tangent else None,
                                     _p(y) if want_y else None, tol, maxit,
                                     threads or default_threads())
    out = {"sig": sig, "state": st, "iters": iters, "status": status, "resid": resid}
    if tangent:
        out["tangent"] = tan
    if want_y:
        out["y"] = y
    return out
