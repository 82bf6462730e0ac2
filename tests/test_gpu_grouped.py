"""GPU parity of lupp_batched_solve_grouped (several uniform AoS batches of
different sizes in one call, Section 4.1's size-aware dispatch): bitwise the
oracle's factors, solutions, pivots and info for every group, with padded
leading dimensions and strides, empty groups, a singular system, more groups
than one launch holds, and every ragged lane count; argument checks."""
import numpy as np
import pytest
import torch

import oracle
from workloads import systems

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def L():
    import paper_2609_15217_amd.lupp as L
    return L


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


def make_group(L, n, batch, seed, lda_pad=0, sa_pad=0, sb_pad=0, singular=False):
    A, b, _ = systems(n, batch, seed=seed) if batch else (np.zeros((0, n, n)), np.zeros((0, n)), None)
    if singular and batch:
        A[0][:, 1] = A[0][:, 0]  # rows 0 and 1 equal (storage [j][i]): an exact zero pivot
    lda = n + lda_pad
    sA = lda * n + sa_pad
    sB = n + sb_pad
    hA = np.full((max(batch, 1), sA), np.nan)
    hb = np.full((max(batch, 1), sB), np.nan)
    for s in range(batch):
        for j in range(n):
            hA[s, j * lda:j * lda + n] = A[s][j]
        hb[s, :n] = b[s]
    tA = torch.from_numpy(hA).to(DEV)
    tb = torch.from_numpy(hb).to(DEV)
    ip = torch.full((max(batch, 1), n), -5, dtype=torch.int32, device=DEV)
    inf = torch.full((max(batch, 1),), -5, dtype=torch.int32, device=DEV)
    g = L.group(n, batch, tA, tb, ip, inf, lda=lda, strideA=sA, strideB=sB)
    return {"g": g, "A": A, "b": b, "tA": tA, "tb": tb, "ip": ip, "inf": inf, "lda": lda}


def check(G, factors=True):
    n, A, b = G["g"].n, G["A"], G["b"]
    batch = A.shape[0]
    if batch == 0:
        assert int(G["inf"][0]) == -5  # untouched
        return
    ref = oracle.gesv_batch(A, b, threads=4)
    lda = G["lda"]
    hA = G["tA"].cpu().numpy()
    hb = G["tb"].cpu().numpy()
    LU = np.stack([np.stack([hA[s, j * lda:j * lda + n] for j in range(n)]) for s in range(batch)])
    assert np.array_equal(G["inf"].cpu().numpy(), ref["info"])
    assert np.array_equal(G["ip"].cpu().numpy(), ref["ipiv"])
    assert np.array_equal(hb[:, :n], ref["x"])
    assert np.array_equal(LU, ref["LU"] if factors else A)
    if lda > n:  # padding rows untouched
        assert np.all(np.isnan(hA[:, n:lda]))


def test_grouped_mixed_sizes_bitwise(L, ctx):
    """Eleven groups of sizes 1..32 (one empty) with padded leading
    dimensions and strides; group 5 (n = 8) holds an exactly singular system."""
    spec = [(32, 700), (2, 1000), (17, 333), (5, 4097), (1, 10), (12, 2048), (24, 95),
            (9, 0), (16, 1500), (3, 257), (31, 64)]
    G = [make_group(L, n, bt, seed=600 + k, lda_pad=k % 3, sa_pad=k % 2, sb_pad=(k + 1) % 2,
                    singular=(k == 5))
         for k, (n, bt) in enumerate(spec)]
    rc = L.lupp_batched_solve_grouped(ctx, [x["g"] for x in G])
    assert rc == 0, L.lupp_error_string(rc)
    torch.cuda.synchronize()
    for x in G:
        check(x)
    assert int(G[5]["inf"][0]) > 0


def test_grouped_more_groups_than_one_launch_and_keep_a(L, ctx):
    G = [make_group(L, 2 + k % 31, 37 + 11 * k, seed=700 + k) for k in range(70)]
    assert L.lupp_batched_solve_grouped(ctx, [x["g"] for x in G], L.LUPP_KEEP_A) == 0
    torch.cuda.synchronize()
    for x in G:
        check(x, factors=False)


@pytest.mark.parametrize("n", [4, 8, 16, 20])
def test_grouped_every_lane_count(L, ctx, n):
    lanes = [t for t in (1, 2, 4, 8, 16) if L.lupp_ragged_lanes_supported(n, t)]
    keep = L.lupp_get_ragged_lanes(ctx, n)
    try:
        for t in lanes:
            assert L.lupp_set_ragged_lanes(ctx, n, t) == 0
            G = [make_group(L, n, 3001, seed=800 + n)]
            assert L.lupp_batched_solve_grouped(ctx, [G[0]["g"]]) == 0
            torch.cuda.synchronize()
            check(G[0])
    finally:
        L.lupp_set_ragged_lanes(ctx, n, keep)


def test_grouped_arguments(L, ctx):
    G = make_group(L, 8, 10, seed=900)
    g = G["g"]
    f = L.lupp_batched_solve_grouped
    assert f(ctx, []) == 0
    for field, val in (("n", 0), ("n", 33), ("batch", -1), ("lda", 7), ("strideA", 63),
                       ("strideB", 7), ("A", 0), ("info", 0)):
        bad = L.lupp_group(g.n, g.batch, g.A, g.lda, g.strideA, g.b, g.strideB, g.ipiv, g.info)
        setattr(bad, field, val)
        assert f(ctx, [g, bad]) == -3, field
    assert f(ctx, [g], flags=L.LUPP_FMA) == -4
    torch.cuda.synchronize()
    assert int(G["inf"][0]) == -5  # nothing ran
