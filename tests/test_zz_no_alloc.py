"""The allocation-free ragged solve (lupp_batched_solve_ragged_noalloc) against
the allocating one (lupp_batched_solve_ragged): bitwise the same factors,
solutions, pivots and info, on two calls in a row (the second smaller, so it
runs over a workspace that still holds the first call's plan), plus its
argument checks and the size limit."""
import numpy as np
import pytest
import torch

from workloads import mixed_systems

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def L():
    import paper_2609_15217_amd.lupp as L
    return L


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


def _run(L, ctx, mx, noalloc, flags=0):
    tn = torch.from_numpy(mx["n"]).to(DEV)
    oa = torch.from_numpy(mx["offA"]).to(DEV)
    ob = torch.from_numpy(mx["offB"]).to(DEV)
    A = torch.from_numpy(mx["A"]).to(DEV)
    b = torch.from_numpy(mx["b"]).to(DEV)
    ip = torch.full((b.numel(),), -7, dtype=torch.int32, device=DEV)
    inf = torch.full((tn.numel(),), -7, dtype=torch.int32, device=DEV)
    f = L.lupp_batched_solve_ragged_noalloc if noalloc else L.lupp_batched_solve_ragged
    rc = f(ctx, tn.numel(), tn, oa, ob, A, b, ip, inf, flags)
    assert rc == 0, L.lupp_error_string(rc)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (A, b, ip, inf)]


def test_noalloc_equals_allocating_path_on_two_calls(L, ctx):
    for count, seed, flags in ((300_001, 501, 0), (40_000, 502, 0), (9_999, 503, 1)):
        mx = mixed_systems(count, seed)
        mx["n"][:3] = (33, 0, 1)  # invalid sizes get info = -1, size 1 is served
        ref = _run(L, ctx, mx, False, flags)
        got = _run(L, ctx, mx, True, flags)
        for a, c in zip(ref, got):
            assert np.array_equal(a, c)
        assert got[3][0] == -1 and got[3][1] == -1 and got[3][2] == 0
        assert np.all(got[3][3:] == 0)


def test_noalloc_arguments_and_limit(L, ctx):
    x = torch.zeros(8, dtype=torch.float64, device=DEV)
    i = torch.zeros(8, dtype=torch.int32, device=DEV)
    o = torch.zeros(8, dtype=torch.int64, device=DEV)
    f = L.lupp_batched_solve_ragged_noalloc
    assert f(ctx, 0, None, None, None, None, None, None, None) == 0
    assert f(ctx, -1, i, o, o, x, x, i, i) == -2
    assert f(ctx, 4, None, o, o, x, x, i, i) == -3
    assert f(ctx, 4, i, o, o, x, x, i, i, L.LUPP_RAGGED_PER_SIZE) == -10
    assert f(ctx, L.LUPP_NOALLOC_MAX_BATCH + 1, i, o, o, x, x, i, i) == L.LUPP_E_TOO_LARGE
