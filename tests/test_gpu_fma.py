"""GPU parity of the FMA arithmetic mode (LUPP_FMA) against the oracle's FMA
mode: bit-exact factors, pivots, info and solutions for every kernel variant
and both layouts, also with LUPP_KEEP_A, special matrices and the stress
distribution."""
import numpy as np
import pytest

import oracle
from test_gpu_lupp import assert_same, gpu_solve, variants
from workloads import special_matrices, systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_2609_15217_amd.lupp as L
    return L


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


@pytest.mark.parametrize("n", [1, 3, 8, 12, 13, 16, 24, 32])
def test_fma_mode_bitwise(L, ctx, n):
    A, b, _ = systems(n, 290, seed=8000 + n)
    ref = oracle.gesv_batch_mode(A, b, fma=True, threads=8)
    strict = oracle.gesv_batch(A, b, threads=8)
    if n >= 8:
        assert not np.array_equal(ref["x"], strict["x"])  # the modes really differ
    for variant, lanes in variants(n):
        for layout in (L.LUPP_AOS, L.LUPP_SOA):
            LU, x, pv, io, pad_ok = gpu_solve(L, ctx, A, b, layout, variant, lanes, fma=True)
            assert pad_ok
            assert_same(ref, LU, x, pv, io, b=b)
            LU, x, pv, io, _ = gpu_solve(L, ctx, A, b, layout, variant, lanes, fma=True,
                                         keep_a=True)
            assert_same(ref, LU, x, pv, io, keep_a=True, A=A)


@pytest.mark.parametrize("n", [7, 16, 31])
def test_fma_with_special_and_stress_matrices(L, ctx, n):
    sm = special_matrices(n, seed=n)
    A = np.stack([sm[k] for k in sorted(sm)] * 4)
    b = np.random.Generator(np.random.PCG64(n)).uniform(-1, 1, (A.shape[0], n))
    ref = oracle.gesv_batch_mode(A, b, fma=True, threads=2)
    for layout in (L.LUPP_AOS, L.LUPP_SOA):
        assert_same(ref, *gpu_solve(L, ctx, A, b, layout, fma=True)[:4], b=b)
    # the stress distribution in FMA mode; FMA with tile-local pivoting is
    # not a compiled combination
    rng = np.random.Generator(np.random.PCG64(50 + n))
    A = rng.uniform(-5e-10, 5e-10, (300, n, n))
    b = rng.uniform(-5e-10, 5e-10, (300, n))
    ref = oracle.gesv_batch_mode(A, b, fma=True, threads=8)
    for variant, lanes in variants(n):
        for layout in (L.LUPP_AOS, L.LUPP_SOA):
            assert_same(ref, *gpu_solve(L, ctx, A, b, layout, variant, lanes, fma=True)[:4], b=b)
    assert L.lupp_set_pivoting(ctx, 4, 1e-10) == 0
    try:
        with pytest.raises(AssertionError):
            gpu_solve(L, ctx, A, b, L.LUPP_AOS, fma=True)  # rc == LUPP_E_UNSUPPORTED
    finally:
        L.lupp_set_pivoting(ctx, 0, 0.0)
