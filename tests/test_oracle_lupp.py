"""Pins of the CPU oracle's LU with partial pivoting (Section 2.2 of the paper)
against results fixed by mathematics or by an independent library, never by
the oracle itself.

* Cramer's rule in exact rational arithmetic (n <= 4).
* Exact-rational Gaussian elimination with partial pivoting (pivot sequence).
* LAPACK dgetrf through scipy (pivot vector and factors).
* PA = LU reconstruction and the |l_ij| <= 1 partial-pivoting invariant.
* Structured matrices with known pivots / info / solution.
* Exact power-of-two scaling invariance.
* Backward and forward error bounds on b = A x_true systems.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
from workloads import special_matrices, systems

U = 2.0 ** -53


def colmajor_to_rows(a):
    """(n, n) array read [j][i] -> ordinary row-major matrix M[i][j]."""
    return np.asarray(a).T


def det_frac(M):
    n = len(M)
    if n == 1:
        return M[0][0]
    total = Fraction(0)
    for perm in itertools.permutations(range(n)):
        sgn = 1
        for i in range(n):
            for j in range(i + 1, n):
                if perm[i] > perm[j]:
                    sgn = -sgn
        prod = Fraction(1)
        for i in range(n):
            prod *= M[i][perm[i]]
        total += sgn * prod
    return total


def cramer(M, b):
    n = len(M)
    d = det_frac(M)
    xs = []
    for j in range(n):
        Mj = [[(b[i] if c == j else M[i][c]) for c in range(n)] for i in range(n)]
        xs.append(det_frac(Mj) / d)
    return xs, d


def inv_inf_norm_frac(M):
    """||M^-1||_inf exactly (via adjugate / Cramer on unit vectors)."""
    n = len(M)
    cols = []
    for j in range(n):
        e = [Fraction(int(i == j)) for i in range(n)]
        cols.append(cramer(M, e)[0])
    return max(sum(abs(cols[j][i]) for j in range(n)) for i in range(n))


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_cramer_exact_rationals(n):
    rng = np.random.Generator(np.random.PCG64(100 + n))
    checked = 0
    while checked < 60:
        Mi = rng.integers(-6, 7, (n, n))
        bi = rng.integers(-9, 10, n)
        M = [[Fraction(int(v)) for v in row] for row in Mi]
        if det_frac(M) == 0:
            continue
        xs, _ = cramer(M, [Fraction(int(v)) for v in bi])
        A = Mi.T.astype(np.float64)  # column-major storage [j][i]
        out = oracle.gesv_batch(A[None], bi[None].astype(np.float64), threads=1)
        assert out["info"][0] == 0
        x = out["x"][0]
        kappa = float(max(sum(abs(v) for v in row) for row in M) * inv_inf_norm_frac(M))
        xinf = float(max(abs(v) for v in xs))
        err = max(abs(Fraction(float(x[i])) - xs[i]) for i in range(n))
        # First-order bound for a backward-stable solve: c * n * u * kappa * ||x||.
        assert float(err) <= 8 * n * U * kappa * xinf + 1e-300
        if n == 1:
            # one correctly rounded division
            assert x[0] == float(xs[0])
        checked += 1


def exact_pivots(Mi):
    """Pivot rows (1-based, LAPACK interchange form) of Gaussian elimination
    with partial pivoting in exact rational arithmetic, lowest row on ties,
    plus the minimum relative gap between best and second-best candidates."""
    n = len(Mi)
    a = [[Fraction(int(v)) for v in row] for row in Mi]
    piv, gap = [], 1.0
    for k in range(n):
        mags = [abs(a[i][k]) for i in range(k, n)]
        best = max(mags)
        p = k + mags.index(best)
        if len(mags) > 1:
            rest = sorted(mags, reverse=True)[1]
            gap = min(gap, float((best - rest) / best) if best else 0.0)
        piv.append(p + 1)
        if best == 0:
            continue
        a[k], a[p] = a[p], a[k]
        for i in range(k + 1, n):
            l = a[i][k] / a[k][k]
            a[i][k] = l
            for j in range(k + 1, n):
                a[i][j] -= l * a[k][j]
    return piv, gap


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_pivots_match_exact_elimination(n):
    rng = np.random.Generator(np.random.PCG64(200 + n))
    compared = 0
    for _ in range(300):
        Mi = rng.integers(-20, 21, (n, n))
        piv, gap = exact_pivots(Mi)
        if gap < 1e-6:  # floating point may legitimately break a near-tie
            continue
        _, ipiv, info, _ = oracle.getrf(Mi.T.astype(np.float64))
        assert list(ipiv) == piv, (Mi, piv, ipiv)
        compared += 1
    assert compared > 100


@pytest.mark.parametrize("n", [2, 5, 8, 13, 16, 24, 32])
def test_pivots_and_factors_match_lapack(n):
    A, b, _ = systems(n, 200, seed=300 + n)
    out = oracle.gesv_batch(A, b, threads=4, want_gap=True)
    for s in range(A.shape[0]):
        M = colmajor_to_rows(A[s])
        lu, piv = scipy.linalg.lu_factor(M)
        assert np.array_equal(out["ipiv"][s], piv + 1), s
        LU = colmajor_to_rows(out["LU"][s])
        scale = np.abs(lu).max()
        assert np.max(np.abs(LU - lu)) <= 1e-11 * scale
        x_ref = scipy.linalg.lu_solve((lu, piv), b[s])
        assert np.allclose(out["x"][s], x_ref, rtol=1e-9, atol=1e-12 * np.abs(x_ref).max())


def unpack(LU):
    n = LU.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    Uu = np.triu(LU)
    return L, Uu


def perm_from_ipiv(ipiv):
    n = len(ipiv)
    p = list(range(n))
    for k in range(n):
        r = ipiv[k] - 1
        p[k], p[r] = p[r], p[k]
    return p


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 12, 16, 24, 31, 32])
def test_reconstruction_and_multiplier_bound(n):
    A, b, _ = systems(n, 100, seed=400 + n)
    out = oracle.gesv_batch(A, b, threads=4)
    for s in range(A.shape[0]):
        M = colmajor_to_rows(A[s])
        L, Uu = unpack(colmajor_to_rows(out["LU"][s]))
        assert np.all(np.abs(np.tril(L, -1)) <= 1.0)
        p = perm_from_ipiv(out["ipiv"][s])
        assert all(out["ipiv"][s][k] >= k + 1 for k in range(n))
        R = M[p] - L @ Uu
        bound = 4 * n * U * np.abs(np.abs(L) @ np.abs(Uu)).max()
        assert np.abs(R).max() <= bound + 1e-300


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_first_column_multipliers_are_correctly_rounded_quotients(n):
    """Section 2.2's multiplier l_i0 = a_i0 / a_p0 is a true division: after
    the first interchange, every stored multiplier of column 0 is the
    correctly rounded quotient of two input entries (exact rationals,
    rounded once), moved by the later interchanges like the rest of its row.
    A reciprocal multiply a_i0 * (1 / a_p0) rounds twice and misses it on a
    sizeable share of entries."""
    A, b, _ = systems(n, 400, seed=450 + n)
    out = oracle.gesv_batch(A, b, threads=4)
    mism = 0
    for s in range(A.shape[0]):
        col = [Fraction(float(v)) for v in A[s][0]]  # column 0, rows 0..n-1
        ipiv = out["ipiv"][s]
        p0 = ipiv[0] - 1
        rows = list(range(n))
        rows[0], rows[p0] = rows[p0], rows[0]
        mult = [float(col[rows[i]] / col[p0]) for i in range(n)]  # Fraction -> float rounds once
        for k in range(1, n):
            r = ipiv[k] - 1
            mult[k], mult[r] = mult[r], mult[k]
        got = out["LU"][s][0][1:]
        assert np.array_equal(got, np.array(mult[1:])), s
        recip = 1.0 / float(col[p0])
        mism += sum(float(col[rows[i]]) * recip != float(col[rows[i]] / col[p0]) for i in range(1, n))
    assert mism > 0  # the reciprocal form really differs on these inputs


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32])
def test_special_matrices(n):
    sm = special_matrices(n, seed=n)
    rng = np.random.Generator(np.random.PCG64(n))
    b = rng.uniform(-1, 1, n)
    ident = list(range(1, n + 1))

    lu, ipiv, info, _ = oracle.getrf(sm["identity"])
    assert info == 0 and list(ipiv) == ident and np.array_equal(lu, np.eye(n))
    assert np.array_equal(oracle.getrs(lu, ipiv, b), b)

    P = sm["permutation"]  # column j has its one in row perm[j]
    lu, ipiv, info, _ = oracle.getrf(P)
    assert info == 0
    x = oracle.getrs(lu, ipiv, b)
    perm = np.argmax(P, axis=1)
    assert np.array_equal(x, b[perm])  # A x = b  with  A[perm[j], j] = 1

    for name in ("col_diag_dominant", "upper_triangular"):
        lu, ipiv, info, _ = oracle.getrf(sm[name])
        assert info == 0 and list(ipiv) == ident, name
    lu, ipiv, info, _ = oracle.getrf(sm["upper_triangular"])
    assert np.array_equal(lu, sm["upper_triangular"])  # zero multipliers change nothing

    zc = min(n - 1, n // 2)
    _, _, info, _ = oracle.getrf(sm["zero_column"])
    assert info == zc + 1

    if n >= 2:
        _, _, info, _ = oracle.getrf(sm["duplicate_rows"])
        assert info > 0
        A = sm["duplicate_rows"]
        out = oracle.gesv_batch(A[None], b[None], threads=1)
        assert out["info"][0] > 0 and np.array_equal(out["x"][0], b)  # b untouched
        _, ipiv, _, gap = oracle.getrf(sm["tied_first_column"])
        assert ipiv[0] == 1 and gap == 0.0


@pytest.mark.parametrize("s", [-31, -7, 5, 40])
@pytest.mark.parametrize("n", [3, 8, 17, 32])
def test_power_of_two_scaling_is_exact(n, s):
    A, b, _ = systems(n, 50, seed=500 + n)
    o1 = oracle.gesv_batch(A, b, threads=2)
    o2 = oracle.gesv_batch(np.ldexp(A, s), np.ldexp(b, s), threads=2)
    assert np.array_equal(o1["ipiv"], o2["ipiv"])
    assert np.array_equal(o1["x"], o2["x"])
    L1 = np.tril(o1["LU"].transpose(0, 2, 1), -1)
    L2 = np.tril(o2["LU"].transpose(0, 2, 1), -1)
    assert np.array_equal(L1, L2)
    U1 = np.triu(o1["LU"].transpose(0, 2, 1))
    U2 = np.triu(o2["LU"].transpose(0, 2, 1))
    assert np.array_equal(np.ldexp(U1, s), U2)


@pytest.mark.parametrize("n", [4, 8, 12, 16, 24, 32])
def test_backward_and_forward_error(n):
    A, b, xt = systems(n, 400, seed=2000 + n, kappa_max=1e4)
    out = oracle.gesv_batch(A, b, threads=4)
    assert np.all(out["info"] == 0)
    M = A.transpose(0, 2, 1)
    r = b - np.einsum("sij,sj->si", M, out["x"])
    nA = np.abs(M).sum(axis=2).max(axis=1)
    be = np.abs(r).max(axis=1) / (nA * np.abs(out["x"]).max(axis=1) + np.abs(b).max(axis=1))
    # Normwise backward error of a backward-stable LUpp solve is O(n u); the
    # paper reports medians of order 1e-15 for textbook pivoting.
    assert be.max() <= 4 * n * U * 8
    assert np.median(be) < 1e-15
    fe = np.abs(out["x"] - xt).max(axis=1) / np.abs(xt).max(axis=1)
    assert fe.max() <= 1e4 * n * U * 64


def test_ragged_equals_per_size():
    from workloads import mixed_systems
    mx = mixed_systems(3000, seed=33)
    out = oracle.gesv_ragged(mx["n"], mx["offA"], mx["offB"], mx["A"], mx["b"], threads=4)
    for s in range(0, 3000, 97):
        n = int(mx["n"][s])
        a = mx["A"][mx["offA"][s]:mx["offA"][s] + n * n].reshape(n, n)
        bb = mx["b"][mx["offB"][s]:mx["offB"][s] + n]
        o = oracle.gesv_batch(a[None], bb[None], threads=1)
        assert np.array_equal(o["x"][0], out["x"][mx["offB"][s]:mx["offB"][s] + n])
        assert np.array_equal(o["ipiv"][0], out["ipiv"][mx["offB"][s]:mx["offB"][s] + n])
