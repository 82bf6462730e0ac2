"""GPU parity of tile-local pivoting (the Tiled solvers' rule, Section 3.2.2)
against the oracle's tiled mode: bit-exact factors, pivots, info and
solutions for every kernel variant and both layouts, under the paper's
default U(-0.5, 0.5) and stress U(-5e-10, 5e-10) distributions (the latter
forces out-of-tile pivots)."""
import numpy as np
import pytest

import oracle
from test_gpu_lupp import assert_same, gpu_solve, variants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_2609_15217_amd.lupp as L
    return L


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


def draw(n, batch, seed, scale):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, (batch, n, n)), rng.uniform(-scale, scale, (batch, n))


@pytest.mark.parametrize("n", [3, 8, 12, 13, 16, 24, 32])
def test_tile_local_pivoting_bitwise(L, ctx, n):
    try:
        for tile in (2, 4, 5):
            assert L.lupp_set_pivoting(ctx, tile, 1e-10) == 0
            for scale, seed in ((0.5, 1), (5e-10, 2)):
                A, b = draw(n, 260, 100 * n + 10 * tile + seed, scale)
                ref = oracle.gesv_batch_tiled(A, b, tile, 1e-10, threads=8)
                if scale < 1e-3 and tile < n:
                    assert ref["out_of_tile"].sum() > 0  # the fallback is exercised
                for variant, lanes in variants(n):
                    for layout in (L.LUPP_AOS, L.LUPP_SOA):
                        LU, x, pv, io, _ = gpu_solve(L, ctx, A, b, layout, variant, lanes)
                        assert_same(ref, LU, x, pv, io, b=b)
    finally:
        L.lupp_set_pivoting(ctx, 0, 0.0)


def test_pivoting_settings(L, ctx):
    assert L.lupp_get_pivoting(ctx) == (0, 0, 0.0)
    assert L.lupp_set_pivoting(ctx, 33, 1e-10) == -2
    assert L.lupp_set_pivoting(ctx, 4, -1.0) == -3
    assert L.lupp_set_pivoting(ctx, 4, float("nan")) == -3
    # a tile covering the matrix is textbook pivoting
    A, b = draw(10, 300, 5, 0.5)
    ref = oracle.gesv_batch(A, b, threads=4)
    assert L.lupp_set_pivoting(ctx, 16, 1e-10) == 0
    try:
        for layout in (L.LUPP_AOS, L.LUPP_SOA):
            assert_same(ref, *gpu_solve(L, ctx, A, b, layout)[:4], b=b)
    finally:
        L.lupp_set_pivoting(ctx, 0, 0.0)
    assert L.lupp_get_pivoting(ctx) == (0, 0, 0.0)
