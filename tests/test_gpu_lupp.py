"""GPU parity of the batched LU solve (Section 2.2) against the CPU oracle.

The HIP path must reproduce the oracle's pivots, info, factors and solutions
bit for bit (strict mode: same pivot choices, same rounded operations per
element, no FMA), for every compiled variant, both layouts, ragged batch
tails, strides and degenerate inputs.
"""
import functools

import numpy as np
import pytest
import torch

import oracle
from workloads import aos_to_soa, special_matrices, systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_2609_15217_amd.lupp as L
    return L


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


def thread_ok(n):
    return n <= 13


def lanes_widths(n):
    from paper_2609_15217_amd.build import lanes_widths as lw
    return lw(n) if n >= 2 else []


def variants(n):
    out = []
    if thread_ok(n):
        out.append((1, 0))
    out += [(2, t) for t in lanes_widths(n)]
    return out


def gpu_solve(L, ctx, A, b, layout, variant=0, lanes=0, wpb=0, keep_a=False, lda=None,
              stride_pad=0, fma=False):
    """Run the library on AoS numpy inputs; return AoS numpy outputs."""
    batch, n = A.shape[0], A.shape[1]
    lda = lda or n
    dev = torch.device("cuda:0")
    if layout == L.LUPP_AOS:
        sA = lda * n + stride_pad
        Ab = np.zeros((batch, sA))
        for j in range(n):
            Ab[:, j * lda:j * lda + n] = A[:, j, :]
        sB = n + stride_pad
        bb = np.zeros((batch, sB))
        bb[:, :n] = b
        tA = torch.from_numpy(Ab).to(dev)
        tb = torch.from_numpy(bb).to(dev)
        ipiv = torch.zeros((batch, n), dtype=torch.int32, device=dev)
    else:
        ld = batch + stride_pad
        Ab = np.zeros((n * lda, ld))
        S = aos_to_soa(A).reshape(n, n, batch)
        for j in range(n):
            Ab[j * lda:j * lda + n, :batch] = S[j]
        bb = np.zeros((n, ld))
        bb[:, :batch] = aos_to_soa(b)
        tA = torch.from_numpy(Ab).to(dev)
        tb = torch.from_numpy(bb).to(dev)
        sA = sB = ld
        ipiv = torch.zeros((n, ld), dtype=torch.int32, device=dev)
    info = torch.full((batch,), -7, dtype=torch.int32, device=dev)
    assert L.lupp_force_variant(ctx, variant, lanes, wpb) == 0
    try:
        rc = L.lupp_batched_solve(ctx, n, batch, layout, tA, lda, sA, tb, sB, ipiv, info,
                                  (L.LUPP_KEEP_A if keep_a else 0) | (L.LUPP_FMA if fma else 0))
    finally:
        L.lupp_force_variant(ctx, 0, 0, 0)
    assert rc == 0, L.lupp_error_string(rc)
    torch.cuda.synchronize()
    Ao, bo, po, io = tA.cpu().numpy(), tb.cpu().numpy(), ipiv.cpu().numpy(), info.cpu().numpy()
    if layout == L.LUPP_AOS:
        LU = np.stack([Ao[:, j * lda:j * lda + n] for j in range(n)], axis=1)
        x = bo[:, :n]
        pv = po
        pad_ok = np.all(Ao[:, lda * n:] == 0) and np.all(bo[:, n:] == 0) and \
            all(np.all(Ao[:, j * lda + n:(j + 1) * lda] == 0) for j in range(n))
    else:
        LU = np.stack([Ao[j * lda:j * lda + n, :batch].T for j in range(n)], axis=1)
        x = bo[:, :batch].T
        pv = po[:, :batch].T
        pad_ok = np.all(Ao[:, batch:] == 0) and np.all(bo[:, batch:] == 0) and \
            all(np.all(Ao[j * lda + n:(j + 1) * lda] == 0) for j in range(n))
    return LU, x, pv, io, pad_ok


def assert_same(ref, LU, x, pv, io, keep_a=False, A=None, b=None):
    assert np.array_equal(io, ref["info"])
    assert np.array_equal(pv, ref["ipiv"])
    if keep_a:
        assert np.array_equal(LU, A)
    else:
        assert np.array_equal(LU, ref["LU"])
    ok = ref["info"] == 0
    assert np.array_equal(x[ok], ref["x"][ok])
    if b is not None:
        assert np.array_equal(x[~ok], b[~ok])  # b untouched where info > 0


@pytest.mark.parametrize("n", list(range(1, 33)))
def test_every_size_every_variant_bitwise(L, ctx, n):
    batch = 300  # > one workgroup, ragged tail in every variant
    A, b, _ = systems(n, batch, seed=7000 + n)
    ref = oracle.gesv_batch(A, b, threads=8)
    for variant, lanes in variants(n):
        for layout in (L.LUPP_AOS, L.LUPP_SOA):
            LU, x, pv, io, pad_ok = gpu_solve(L, ctx, A, b, layout, variant, lanes)
            assert pad_ok
            assert_same(ref, LU, x, pv, io, b=b)


@pytest.mark.parametrize("wpb", [1, 2, 4])
@pytest.mark.parametrize("n", [3, 8, 13, 21, 32])
def test_workgroup_sizes(L, ctx, n, wpb):
    A, b, _ = systems(n, 517, seed=7100 + n)
    ref = oracle.gesv_batch(A, b, threads=8)
    for variant, lanes in variants(n):
        LU, x, pv, io, _ = gpu_solve(L, ctx, A, b, L.LUPP_SOA, variant, lanes, wpb)
        assert_same(ref, LU, x, pv, io)


@pytest.mark.parametrize("n", [2, 5, 8, 12, 17, 32])
def test_padded_strides_and_keep_a(L, ctx, n):
    A, b, _ = systems(n, 150, seed=7200 + n)
    ref = oracle.gesv_batch(A, b, threads=8)
    for variant, lanes in variants(n):
        for layout in (L.LUPP_AOS, L.LUPP_SOA):
            LU, x, pv, io, pad_ok = gpu_solve(L, ctx, A, b, layout, variant, lanes, lda=n + 3,
                                              stride_pad=5)
            assert pad_ok, "wrote outside the systems"
            assert_same(ref, LU, x, pv, io)
            LU, x, pv, io, _ = gpu_solve(L, ctx, A, b, layout, variant, lanes, keep_a=True)
            assert_same(ref, LU, x, pv, io, keep_a=True, A=A)


@pytest.mark.parametrize("n", [1, 2, 4, 7, 8, 13, 16, 31, 32])
def test_special_and_singular_matrices(L, ctx, n):
    sm = special_matrices(n, seed=n)
    names = sorted(sm)
    A = np.stack([sm[k] for k in names] * 3)
    b = np.random.Generator(np.random.PCG64(n)).uniform(-1, 1, (A.shape[0], n))
    ref = oracle.gesv_batch(A, b, threads=2)
    for variant, lanes in variants(n):
        for layout in (L.LUPP_AOS, L.LUPP_SOA):
            LU, x, pv, io, _ = gpu_solve(L, ctx, A, b, layout, variant, lanes)
            assert_same(ref, LU, x, pv, io, b=b)


def test_stress_magnitudes_and_scaling(L, ctx):
    """Entries of magnitude 5e-10 (the paper's stress distribution is a pure
    rescaling for textbook pivoting): bitwise equal after exact 2^-31 scaling."""
    for n in (6, 12, 24):
        A, b, _ = systems(n, 200, seed=7300 + n)
        As, bs = np.ldexp(A, -31), np.ldexp(b, -31)
        ref = oracle.gesv_batch(As, bs, threads=4)
        for variant, lanes in variants(n):
            LU, x, pv, io, _ = gpu_solve(L, ctx, As, bs, L.LUPP_SOA, variant, lanes)
            assert_same(ref, LU, x, pv, io)


def test_empty_and_single(L, ctx):
    dev = torch.device("cuda:0")
    e = torch.empty(0, dtype=torch.float64, device=dev)
    ei = torch.empty(0, dtype=torch.int32, device=dev)
    assert L.lupp_batched_solve(ctx, 8, 0, L.LUPP_AOS, e, 8, 64, e, 8, ei, ei) == 0
    assert L.lupp_batched_solve(ctx, 8, 0, L.LUPP_AOS, None, 8, 64, None, 8, None, None) == 0
    for n in (1, 9, 32):
        A, b, _ = systems(n, 1, seed=7400 + n)
        ref = oracle.gesv_batch(A, b, threads=1)
        for variant, lanes in variants(n):
            for layout in (L.LUPP_AOS, L.LUPP_SOA):
                LU, x, pv, io, _ = gpu_solve(L, ctx, A, b, layout, variant, lanes)
                assert_same(ref, LU, x, pv, io)


def test_invalid_arguments(L, ctx):
    dev = torch.device("cuda:0")
    t = torch.zeros(64, dtype=torch.float64, device=dev)
    ti = torch.zeros(8, dtype=torch.int32, device=dev)
    assert L.lupp_batched_solve(ctx, 33, 1, 0, t, 33, 33 * 33, t, 33, ti, ti) == -2
    assert L.lupp_batched_solve(ctx, 8, 1, 0, t, 7, 64, t, 8, ti, ti) == -6
    assert L.lupp_batched_solve(ctx, 8, 1, 0, t, 8, 64, t, 8, ti, ti, flags=8) == -12
    assert L.lupp_force_variant(ctx, 2, 3, 0) == -3
    assert L.lupp_set_dispatch(ctx, 20, 0, 1 << 20, 1, 0, 0) == -6  # no thread kernel for n = 20


def test_repeat_is_deterministic(L, ctx):
    A, b, _ = systems(16, 3000, seed=7500)
    r1 = gpu_solve(L, ctx, A, b, L.LUPP_SOA)
    r2 = gpu_solve(L, ctx, A, b, L.LUPP_SOA)
    for u, v in zip(r1[:4], r2[:4]):
        assert np.array_equal(u, v)


def test_config1_default_dispatch(L, ctx):
    """4096 systems, n = 8, N(0,1) without a condition filter, seed 1."""
    A, b, _ = systems(8, 4096, seed=1)
    ref = oracle.gesv_batch(A, b, threads=8)
    for layout in (L.LUPP_AOS, L.LUPP_SOA):
        LU, x, pv, io, _ = gpu_solve(L, ctx, A, b, layout)
        assert_same(ref, LU, x, pv, io)


def bench_soa_ld():
    """The interleaved ldbatch the benchmark lays its arrays out with."""
    import importlib.util
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_consts", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    return bench.SOA_LD


@functools.lru_cache(maxsize=1)
def full_size_systems(n):
    return systems(n, 1 << 20, seed=2000 + n, kappa_max=1e4)


@pytest.mark.slow
@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("n", [4, 8, 12, 16, 24, 32])
def test_full_size_sweep_sampled(L, ctx, n, layout):
    """2^20 systems per size (kappa_2 <= 1e4), default dispatch, in the
    benchmark's launch configuration (interleaved arrays with its padded
    ldbatch, or packed AoS); 4096 sampled systems compared bitwise."""
    batch = 1 << 20
    A, b, xt = full_size_systems(n)
    dev = torch.device("cuda:0")
    info = torch.full((batch,), -7, dtype=torch.int32, device=dev)
    if layout == "soa":
        ld = bench_soa_ld()
        tA = torch.zeros((n, n, ld), dtype=torch.float64, device=dev)
        tA[:, :, :batch] = torch.from_numpy(aos_to_soa(A)).to(dev)
        tb = torch.zeros((n, ld), dtype=torch.float64, device=dev)
        tb[:, :batch] = torch.from_numpy(aos_to_soa(b)).to(dev)
        ipiv = torch.zeros((n, ld), dtype=torch.int32, device=dev)
        rc = L.lupp_batched_solve(ctx, n, batch, L.LUPP_SOA, tA, n, ld, tb, ld, ipiv, info)
    else:
        tA = torch.from_numpy(A).to(dev)
        tb = torch.from_numpy(b).to(dev)
        ipiv = torch.zeros((batch, n), dtype=torch.int32, device=dev)
        rc = L.lupp_batched_solve(ctx, n, batch, L.LUPP_AOS, tA, n, n * n, tb, n, ipiv, info)
    assert rc == 0, L.lupp_error_string(rc)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(n))
    idx = np.sort(rng.choice(batch, 4096, replace=False))
    idx[-1] = batch - 1
    ref = oracle.gesv_batch(A[idx], b[idx], threads=8)
    if layout == "soa":
        xa = tb[:, :batch].cpu().numpy().T
        LU = tA[:, :, :batch].cpu().numpy()[:, :, idx].transpose(2, 0, 1)
        pv = ipiv[:, :batch].cpu().numpy()[:, idx].T
        assert not tA[:, :, batch:].any() and not tb[:, batch:].any()  # padding untouched
    else:
        xa = tb.cpu().numpy()
        LU = tA.cpu().numpy()[idx]
        pv = ipiv.cpu().numpy()[idx]
    assert np.array_equal(info.cpu().numpy(), np.zeros(batch, dtype=np.int32))
    assert np.array_equal(pv, ref["ipiv"])
    assert np.array_equal(LU, ref["LU"])
    assert np.array_equal(xa[idx], ref["x"])
    # forward error against the known solution (kappa_2 <= 1e4)
    fe = np.abs(xa - xt).max(axis=1) / np.abs(xt).max(axis=1)
    assert fe.max() < 1e-9


def solve_far_apart(L, ctx, A, b, ld, variant, lanes):
    """SoA solve of A, b (AoS numpy) placed in an interleaved array whose
    ldbatch `ld` puts the rows of the batch far apart (beyond 2 GiB); only
    the first batch columns of each row are written and read back."""
    batch, n = A.shape[0], A.shape[1]
    dev = torch.device("cuda:0")
    tA = torch.empty((n * n, ld), dtype=torch.float64, device=dev)
    tb = torch.empty((n, ld), dtype=torch.float64, device=dev)
    ipiv = torch.empty((n, ld), dtype=torch.int32, device=dev)
    info = torch.full((batch,), -7, dtype=torch.int32, device=dev)
    tA[:, :batch] = torch.from_numpy(aos_to_soa(A).reshape(n * n, batch)).to(dev)
    tb[:, :batch] = torch.from_numpy(aos_to_soa(b)).to(dev)
    assert L.lupp_force_variant(ctx, variant, lanes, 0) == 0
    try:
        rc = L.lupp_batched_solve(ctx, n, batch, L.LUPP_SOA, tA, n, ld, tb, ld, ipiv, info)
    finally:
        L.lupp_force_variant(ctx, 0, 0, 0)
    assert rc == 0, L.lupp_error_string(rc)
    torch.cuda.synchronize()
    LU = tA[:, :batch].cpu().numpy().reshape(n, n, batch).transpose(2, 0, 1)
    x = tb[:, :batch].cpu().numpy().T
    pv = ipiv[:, :batch].cpu().numpy().T
    io = info.cpu().numpy()
    del tA, tb, ipiv, info
    torch.cuda.empty_cache()
    return LU, x, pv, io


@pytest.mark.parametrize("n,variant,lanes,ld", [
    (6, 1, 0, 60_000_000),   # thread kernel: (n-1) * ldbatch * 8 > 2 GiB
    (8, 2, 8, 40_000_000),   # staged lanes kernel, 8-lane segments
    (16, 2, 16, 18_000_000),  # staged lanes kernel, 16-lane segments
    (3, 2, 4, 90_000_000),   # beyond the lanes kernel's range: thread kernel
])
def test_interleaved_batches_beyond_2gib(L, ctx, n, variant, lanes, ld):
    """Interleaved batches whose rows lie more than 2^31 bytes apart (up to
    37 GB of address range) solve bitwise as the oracle does."""
    A, b, _ = systems(n, 1000, seed=7600 + n)
    ref = oracle.gesv_batch(A, b, threads=8)
    LU, x, pv, io = solve_far_apart(L, ctx, A, b, ld, variant, lanes)
    assert_same(ref, LU, x, pv, io)


def test_interleaved_batch_out_of_range_is_refused(L, ctx):
    """n = 20 has no thread kernel: an ldbatch beyond the lanes kernel's
    32-bit range is refused on the host, before anything is launched."""
    dev = torch.device("cuda:0")
    t = torch.zeros(64, dtype=torch.float64, device=dev)
    ti = torch.zeros(64, dtype=torch.int32, device=dev)
    rc = L.lupp_batched_solve(ctx, 20, 10, L.LUPP_SOA, t, 20, 90_000_000, t, 90_000_000, ti, ti)
    assert rc == L.LUPP_E_UNSUPPORTED
