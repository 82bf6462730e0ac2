"""Seeded input generators.

Layout conventions (per system, column-major, matching LAPACK):

* AoS arrays have shape ``(batch, n, n)`` and are read as ``A[s][j][i]`` so the
  flat offset of element (i, j) of system s is ``s*n*n + i + j*n``.
* SoA (interleaved) arrays have shape ``(n, n, batch)`` read as ``A[j][i][s]``,
  flat offset ``(i + j*n)*batch + s``; right-hand sides ``(n, batch)``.

Every generator is deterministic for a given seed, independent of how many
threads draw it: the batch is cut into fixed chunks of ``CHUNK`` systems and
chunk c draws from child c of ``numpy.random.SeedSequence(seed)``.

Random matrices follow the workloads of the paper's pure-LUpp experiments
(Section 4.2, dense general matrices with no structure), with entries N(0, 1)
as the benchmark configurations ask; the right-hand side is built from a known
solution so that forward errors can be measured.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 65536


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _cond2(a: np.ndarray) -> np.ndarray:
    """Spectral condition number sigma_max / sigma_min of each matrix."""
    s = np.linalg.svd(a, compute_uv=False)
    with np.errstate(divide="ignore"):
        return s[:, 0] / s[:, -1]


def _draw(rng: np.random.Generator, n: int, m: int, kappa_max):
    """Draw m systems of size n: A ~ N(0,1) (resampled while cond2 > kappa_max),
    x_true ~ U(-1, 1). Resamples come from the same stream, after x_true."""
    a = rng.standard_normal((m, n, n))
    x = rng.uniform(-1.0, 1.0, (m, n))
    if kappa_max is not None and m > 0:
        bad = np.flatnonzero(~(_cond2(a) <= kappa_max))
        while bad.size:
            a[bad] = rng.standard_normal((bad.size, n, n))
            bad = bad[~(_cond2(a[bad]) <= kappa_max)]
    return a, x


def _rhs(a: np.ndarray, x: np.ndarray) -> np.ndarray:
    # b_i = sum_j A[s][j][i] * x_j  (column-major A times x)
    return np.matmul(x[:, None, :], a)[:, 0, :]


def systems(n: int, batch: int, seed: int, kappa_max: float | None = None,
            threads: int | None = None):
    """Return (A, b, x_true) in AoS layout for `batch` systems of size n."""
    if not (1 <= n <= 64) or batch < 0:
        raise ValueError("bad n/batch")
    A = np.empty((batch, n, n), dtype=np.float64)
    b = np.empty((batch, n), dtype=np.float64)
    x = np.empty((batch, n), dtype=np.float64)
    nchunks = max(1, math.ceil(batch / CHUNK))
    seqs = np.random.SeedSequence(seed).spawn(nchunks)

    def work(c):
        lo, hi = c * CHUNK, min(batch, (c + 1) * CHUNK)
        rng = np.random.Generator(np.random.PCG64(seqs[c]))
        a, xx = _draw(rng, n, hi - lo, kappa_max)
        A[lo:hi] = a
        x[lo:hi] = xx
        b[lo:hi] = _rhs(a, xx)

    with ThreadPoolExecutor(threads or _threads()) as ex:
        list(ex.map(work, range(nchunks)))
    return A, b, x


def mixed_systems(batch: int, seed: int, nmin: int = 2, nmax: int = 32,
                  kappa_max: float | None = 1e4, threads: int | None = None):
    """A ragged batch: n_s ~ U{nmin..nmax}, packed AoS in system order with
    lda = n_s. Returns a dict with int32 ``n``, int64 ``offA`` / ``offB``
    (exclusive scans of n^2 and n) and flat float64 ``A``, ``b``, ``x_true``."""
    seqs = np.random.SeedSequence(seed).spawn(1 + max(1, math.ceil(batch / CHUNK)))
    ns = np.random.Generator(np.random.PCG64(seqs[0])).integers(
        nmin, nmax + 1, size=batch).astype(np.int32)
    n64 = ns.astype(np.int64)
    offA = np.zeros(batch, dtype=np.int64)
    offB = np.zeros(batch, dtype=np.int64)
    if batch:
        np.cumsum(n64[:-1] * n64[:-1], out=offA[1:])
        np.cumsum(n64[:-1], out=offB[1:])
    totA = int((n64 * n64).sum())
    totB = int(n64.sum())
    A = np.empty(totA, dtype=np.float64)
    b = np.empty(totB, dtype=np.float64)
    x = np.empty(totB, dtype=np.float64)
    nchunks = max(1, math.ceil(batch / CHUNK))

    def work(c):
        lo, hi = c * CHUNK, min(batch, (c + 1) * CHUNK)
        if hi <= lo:
            return
        rng = np.random.Generator(np.random.PCG64(seqs[1 + c]))
        sub = ns[lo:hi]
        for n in np.unique(sub):
            idx = lo + np.flatnonzero(sub == n)
            a, xx = _draw(rng, int(n), idx.size, kappa_max)
            bb = _rhs(a, xx)
            n = int(n)
            ia = offA[idx][:, None] + np.arange(n * n)[None, :]
            ib = offB[idx][:, None] + np.arange(n)[None, :]
            A[ia] = a.reshape(idx.size, n * n)
            x[ib] = xx
            b[ib] = bb

    with ThreadPoolExecutor(threads or _threads()) as ex:
        list(ex.map(work, range(nchunks)))
    return {"n": ns, "offA": offA, "offB": offB, "A": A, "b": b, "x_true": x}


def device_systems(n: int, batch: int, seed: int, device="cuda"):
    """Timing inputs drawn on the device with torch's seeded generator:
    A ~ N(0,1) (batch, n, n) read [s][j][i], b ~ N(0,1) (batch, n). No
    condition filter: pivoting statistics are those of the benchmark
    distribution, which is what launch-configuration timing needs."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    A = torch.randn((batch, n, n), generator=g, dtype=torch.float64, device=device)
    b = torch.randn((batch, n), generator=g, dtype=torch.float64, device=device)
    return A, b


def aos_to_soa(a: np.ndarray) -> np.ndarray:
    """(batch, n, n) -> (n, n, batch), or (batch, n) -> (n, batch)."""
    return np.ascontiguousarray(np.moveaxis(a, 0, -1))


def newton_points(count: int, seed: int, lo: float = -2e-3, hi: float = 2e-3):
    """Kelvin strain increments, i.i.d. U(lo, hi) per component, shape (count, 6)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, (count, 6))


def serving_requests(num: int, seed: int, rate: float = 2000.0,
                     upd_sizes=(1_000, 500_000), solve_sizes=(1_000, 1_000_000),
                     nmin: int = 2, nmax: int = 32, log_uniform: bool = True):
    """A Poisson stream of requests: half constitutive updates (law 7 or 13 at
    50/50), half standalone solves with one n per request."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, num)
    t = np.cumsum(gaps)
    out = []

    def size(lohi):
        lo, hi = lohi
        if log_uniform:
            return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        return int(rng.integers(lo, hi + 1))

    for k in range(num):
        if rng.uniform() < 0.5:
            out.append({"t": float(t[k]), "kind": "update", "size": size(upd_sizes),
                        "law": 7 if rng.uniform() < 0.5 else 13,
                        "seed": int(rng.integers(0, 2**31 - 1))})
        else:
            out.append({"t": float(t[k]), "kind": "solve", "size": size(solve_sizes),
                        "n": int(rng.integers(nmin, nmax + 1)),
                        "seed": int(rng.integers(0, 2**31 - 1))})
    return out


def special_matrices(n: int, seed: int = 0):
    """Named structured inputs (column-major (n, n) arrays read as [j][i])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {}
    out["identity"] = np.eye(n)
    perm = rng.permutation(n)
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 1.0  # [j][i]: column j has its one in row perm[j]
    out["permutation"] = P
    D = rng.uniform(-1.0, 1.0, (n, n))
    for j in range(n):
        D[j, j] = np.sign(D[j, j] or 1.0) * (np.abs(D[j]).sum() + 1.0)
    out["col_diag_dominant"] = D
    U = np.triu(rng.uniform(-1.0, 1.0, (n, n)).T).T  # upper triangle in [j][i]
    for j in range(n):
        U[j, j] = 2.0 + j
    out["upper_triangular"] = U
    Z = rng.standard_normal((n, n))
    Z[min(n - 1, n // 2)] = 0.0
    out["zero_column"] = Z
    if n >= 2:
        R = rng.integers(-3, 4, (n, n)).astype(np.float64)
        R[:, 1] = R[:, 0]  # rows 0 and 1 equal -> exactly singular
        out["duplicate_rows"] = R
        T = rng.integers(-3, 4, (n, n)).astype(np.float64)
        T[0] = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)  # every |candidate| ties
        out["tied_first_column"] = T
    return out
