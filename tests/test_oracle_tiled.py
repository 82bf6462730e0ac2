"""Pins of the oracle's tile-local pivoting (the Tiled solvers' rule, Section
3.2.2; statistics of Section 4.2), none of which re-runs the oracle's
elimination:

* special cases that reduce to other routines: a tile covering the matrix,
  or an infinite acceptance threshold, is textbook partial pivoting (itself
  pinned to LAPACK elsewhere); tile size 1 with threshold 0 is elimination
  without interchanges;
* the first pivot, decided on the untouched first column, follows the rule;
* P A = L U for whatever pivots were chosen;
* the paper's statements: no out-of-tile pivot under the default
  distribution U(-0.5, 0.5), frequent ones under the stress distribution
  U(-5e-10, 5e-10) with the 1e-10 threshold, and its worst-case backward
  error orders (median 1e-15 / max 1e-9 default, median 1e-16 / max 1e-13
  stress, over n in [2, 32]).
"""
import numpy as np
import pytest

import oracle

THRESH = 1e-10


def draw(n, batch, seed, scale):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.uniform(-scale, scale, (batch, n, n))
    b = rng.uniform(-scale, scale, (batch, n))
    return A, b


def perm_of(ipiv):
    n = ipiv.shape[0]
    p = np.arange(n)
    for k in range(n):
        r = ipiv[k] - 1
        p[k], p[r] = p[r], p[k]
    return p


def unpack(LU):
    L = np.tril(LU, -1) + np.eye(LU.shape[0])
    return L, np.triu(LU)


def backward_error(A, x, b):
    r = np.abs(np.einsum("sji,sj->si", A, x) - b).max(axis=1)
    nA = np.abs(A).sum(axis=1).max(axis=1)  # infinity norm of column-major A[s][j][i]
    return r / (nA * np.abs(x).max(axis=1) + np.abs(b).max(axis=1))


@pytest.mark.parametrize("n", [5, 12, 17])
def test_reduces_to_textbook(n):
    A, b = draw(n, 200, 1 + n, 0.5)
    ref = oracle.gesv_batch(A, b, threads=4)
    for ts, th in ((n, THRESH), (n + 3, THRESH), (1, np.inf), (3, np.inf)):
        got = oracle.gesv_batch_tiled(A, b, ts, th, threads=4)
        for k in ("LU", "x", "ipiv", "info"):
            assert np.array_equal(got[k], ref[k]), (ts, th, k)


def test_tile_one_threshold_zero_is_no_pivoting():
    n = 9
    A, b = draw(n, 100, 7, 0.5)
    A += 4 * np.eye(n)  # no zero pivots without interchanges
    got = oracle.gesv_batch_tiled(A, b, 1, 0.0, threads=2)
    assert np.all(got["ipiv"] == np.arange(1, n + 1))
    for s in range(100):
        L, U = unpack(got["LU"][s].T)
        assert np.allclose(L @ U, A[s].T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("ts", [2, 3, 4, 5, 6])
def test_first_pivot_follows_the_rule(ts):
    n = 16
    for scale, seed in ((0.5, 10), (5e-10, 11)):
        A, b = draw(n, 400, seed + ts, scale)
        got = oracle.gesv_batch_tiled(A, b, ts, THRESH, threads=4)
        col = np.abs(A[:, 0, :])
        in_tile = np.argmax(col[:, :ts], axis=1)
        ok = col[np.arange(400), in_tile] >= THRESH
        expect = np.where(ok, in_tile, np.argmax(col, axis=1)) + 1
        assert np.array_equal(got["ipiv"][:, 0], expect)


@pytest.mark.parametrize("ts", [2, 4, 5])
def test_factorisation_reconstructs(ts):
    n = 14
    for scale in (0.5, 5e-10):
        A, b = draw(n, 50, 20 + ts, scale)
        got = oracle.gesv_batch_tiled(A, b, ts, THRESH, threads=2)
        for s in range(50):
            L, U = unpack(got["LU"][s].T)
            P = np.eye(n)[perm_of(got["ipiv"][s])]
            assert np.abs(P @ A[s].T - L @ U).max() <= 1e-12 * scale * n


def test_out_of_tile_frequency_and_backward_error_orders():
    """The paper's statistics, worst case over n in [2, 32] and the tile sizes
    it uses (2..6), at 3000 systems per point."""
    worst = {"default": [0, 0.0], "stress": [0, 0.0]}
    triggered, per_trigger = [], []
    for n in range(2, 33, 3):
        for ts in range(2, 7):
            if ts >= n:
                continue
            for name, scale in (("default", 0.5), ("stress", 5e-10)):
                A, b = draw(n, 3000, 1000 * n + ts, scale)
                got = oracle.gesv_batch_tiled(A, b, ts, THRESH, threads=8)
                assert np.all(got["info"] == 0)
                be = backward_error(A, got["x"], b)
                worst[name][0] = max(worst[name][0], np.median(be))
                worst[name][1] = max(worst[name][1], be.max())
                oot = got["out_of_tile"]
                if name == "default":
                    assert oot.sum() == 0  # no out-of-tile pivot on the default distribution
                else:
                    triggered.append((oot > 0).mean())
                    if (oot > 0).any():
                        per_trigger.append(oot[oot > 0].mean())
    assert worst["default"][0] <= 1e-14 and worst["default"][1] <= 1e-8
    assert worst["stress"][0] <= 1e-15 and worst["stress"][1] <= 1e-12
    # stress: out-of-tile pivots are frequent (the paper: about half the
    # systems, 1.5 per triggering system, depending on the tile size)
    assert 0.2 <= np.median(triggered) <= 1.0
    assert 1.0 <= np.median(per_trigger) <= 4.0
