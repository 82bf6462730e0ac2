"""Pins of the oracle's FMA mode (every multiply-subtract of the elimination
and the substitutions fused; divisions and pivoting unchanged), none of
which re-runs its elimination:

* on integer systems whose elimination is exact (no interchanges, unit
  pivots, integer multipliers) both modes return the known factors and the
  known solution exactly;
* on random systems the pivots equal LAPACK's and the solutions agree with
  LAPACK's to the rounding level; P A = L U; backward error O(n u);
* the mode really changes the arithmetic: results differ from strict mode in
  the last bits for most random systems;
* 2 x 2 systems whose fused and unfused results are known in closed form,
  one for each place a multiply-subtract occurs (the Schur update, the
  forward and the back substitution): with l = 1 - 2^-30 and u = 1 + 2^-30,
  l * u = 1 - 2^-60 exactly, which rounds to 1, so 1 - l*u is 0 in strict
  mode and 2^-60 in FMA mode.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle


def exact_system(n, seed):
    """A = L U with unit-lower L and unit-diagonal U holding entries in
    {-1, 0, 1}: every pivot candidate below the diagonal ties the diagonal,
    the lowest row wins, so no row moves and every quantity is an integer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.tril(rng.integers(-1, 2, (n, n)), -1) + np.eye(n)
    U = np.triu(rng.integers(-1, 2, (n, n)), 1) + np.eye(n)
    A = L @ U
    x = rng.integers(-5, 6, n).astype(float)
    return A, L, U, x


@pytest.mark.parametrize("n", [3, 7, 12, 20, 32])
def test_exact_integer_elimination(n):
    sys = [exact_system(n, 100 + s) for s in range(20)]
    A = np.stack([s[0].T for s in sys])  # column-major per system
    b = np.stack([s[0] @ s[3] for s in sys])
    for fma in (False, True):
        got = oracle.gesv_batch_mode(A, b, fma=fma, threads=2)
        assert np.all(got["ipiv"] == np.arange(1, n + 1))
        for k, (An, L, U, x) in enumerate(sys):
            LU = got["LU"][k].T
            assert np.array_equal(np.tril(LU, -1) + np.eye(n), L)
            assert np.array_equal(np.triu(LU), U)
            assert np.array_equal(got["x"][k], x)


@pytest.mark.parametrize("n", [4, 9, 16, 32])
def test_against_lapack(n):
    rng = np.random.Generator(np.random.PCG64(n))
    A = rng.standard_normal((200, n, n))
    b = rng.standard_normal((200, n))
    got = oracle.gesv_batch_mode(A, b, fma=True, threads=4)
    strict = oracle.gesv_batch(A, b, threads=4)
    differ = 0
    for s in range(200):
        M = A[s].T
        lu, piv = sla.lu_factor(M)
        assert np.array_equal(got["ipiv"][s], piv + 1)
        x = sla.lu_solve((lu, piv), b[s])
        scale = np.abs(x).max()
        assert np.abs(got["x"][s] - x).max() <= 1e-9 * scale
        L = np.tril(got["LU"][s].T, -1) + np.eye(n)
        U = np.triu(got["LU"][s].T)
        P = np.eye(n)
        for k, r in enumerate(got["ipiv"][s] - 1):
            P[[k, r]] = P[[r, k]]
        assert np.abs(P @ M - L @ U).max() <= 1e-13 * n * np.abs(M).max()
        r = np.abs(M @ got["x"][s] - b[s]).max()
        assert r <= 16 * n * 2.2e-16 * (np.abs(M).sum(axis=1).max() * scale + np.abs(b[s]).max())
        differ += not np.array_equal(got["x"][s], strict["x"][s])
    assert differ > 150  # fused arithmetic changes the last bits


E30, E60 = 2.0 ** -30, 2.0 ** -60


def _solve2(rows, rhs, fma):
    """One 2 x 2 system given row-major; returns the oracle's LU (row-major),
    x, ipiv and info."""
    A = np.array(rows, dtype=float).T[None].copy()  # column-major storage
    b = np.array(rhs, dtype=float)[None]
    out = oracle.gesv_batch_mode(A, b, fma=fma, threads=1)
    return out["LU"][0].T, out["x"][0], out["ipiv"][0], int(out["info"][0])


@pytest.mark.parametrize("fma", [False, True])
def test_closed_form_forward_substitution(fma):
    l, y0 = 1.0 - E30, 1.0 + E30
    LU, x, piv, info = _solve2([[1.0, 0.0], [l, 1.0]], [y0, 1.0], fma)
    assert info == 0 and list(piv) == [1, 2]
    assert LU[1, 0] == l and LU[1, 1] == 1.0
    assert x[0] == y0
    assert x[1] == (E60 if fma else 0.0)


@pytest.mark.parametrize("fma", [False, True])
def test_closed_form_back_substitution(fma):
    u, x1 = 1.0 - E30, 1.0 + E30
    LU, x, piv, info = _solve2([[1.0, u], [0.0, 1.0]], [1.0, x1], fma)
    assert info == 0 and list(piv) == [1, 2]
    assert x[1] == x1
    assert x[0] == (E60 if fma else 0.0)


@pytest.mark.parametrize("fma", [False, True])
def test_closed_form_schur_update(fma):
    l, u = 1.0 - E30, 1.0 + E30
    LU, x, piv, info = _solve2([[1.0, u], [l, 1.0]], [1.0, 1.0], fma)
    assert list(piv) == [1, 2] and LU[1, 0] == l
    if fma:
        assert info == 0 and LU[1, 1] == E60
    else:
        assert info == 2 and LU[1, 1] == 0.0
        assert list(x) == [1.0, 1.0]  # b is left unchanged when info > 0
