"""GPU tests of time-step sweeps captured in a HIP graph (lupp_sweep_*): every
replay equals the same steps launched one by one (bitwise: the same kernels
on the same data), with eager work and synchronisation between replays, and
the steps match successive oracle updates."""
import numpy as np
import pytest
import torch

import oracle
from oracle import Law
from newton_check import check_newton
from workloads import newton_points

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def L():
    import paper_2609_15217_amd.lupp as L
    return L


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


def buffers(kind, count, ld, steps, seed, tangent=False):
    d = torch.zeros((steps, 6, ld), dtype=torch.float64, device=DEV)
    host = []
    for t in range(steps):
        dt = newton_points(count, seed=seed + t, lo=-5e-4, hi=5e-4)
        host.append(dt)
        d[t, :, :count] = torch.from_numpy(dt.T.copy())
    st = torch.zeros((kind, ld), dtype=torch.float64, device=DEV)
    sig = torch.zeros((6, ld), dtype=torch.float64, device=DEV)
    it = torch.zeros(count, dtype=torch.int32, device=DEV)
    ss = torch.zeros(count, dtype=torch.int32, device=DEV)
    tan = torch.zeros((36, ld), dtype=torch.float64, device=DEV) if tangent else None
    return d, host, st, sig, it, ss, tan


def snapshot(*ts):
    return [t.cpu().numpy().copy() for t in ts if t is not None]


@pytest.mark.parametrize("kind,tangent", [(7, False), (13, False), (7, True)])
def test_replays_equal_eager_steps(L, ctx, kind, tangent):
    count, ld, steps = 5000, 5003, 4
    law = L.make_law(kind)
    d, _, st, sig, it, ss, tan = buffers(kind, count, ld, steps, seed=80, tangent=tangent)
    # eager: one constitutive_update per step
    for t in range(steps):
        pts = L.points(d[t], st, sig, it, ss, tan)
        assert L.constitutive_update(ctx, pts, law, 1e-12, 40) == 0
    torch.cuda.synchronize()
    ref = snapshot(st, sig, it, ss, tan)
    # graph: captured once, replayed three times from the initial state
    d2, _, st2, sig2, it2, ss2, tan2 = buffers(kind, count, ld, steps, seed=80, tangent=tangent)
    pts2 = L.points(d2[0], st2, sig2, it2, ss2, tan2)
    sw = L.Sweep(ctx, pts2, law, 1e-12, 40, steps, 6 * ld)
    for rep in range(3):
        st2.zero_()
        sig2.zero_()
        x = torch.randn(1 << 16, device=DEV, dtype=torch.float64)  # eager work in between
        assert float(x.abs().sum().item()) > 0
        torch.cuda.synchronize()
        assert sw.launch() == 0
        torch.cuda.synchronize()
        got = snapshot(st2, sig2, it2, ss2, tan2)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b, equal_nan=True), f"replay {rep}"
    sw.close()


def test_steps_follow_the_oracle(L, ctx):
    """A three-step sweep equals the same steps launched one by one
    (bitwise), and each step, started from the state the GPU committed at the
    previous one, passes the every-point Newton parity against the oracle."""
    kind, count, steps = 13, 2000, 3
    law = L.make_law(kind)
    d, host, st, sig, it, ss, _ = buffers(kind, count, count, steps, seed=90)
    pts = L.points(d[0], st, sig, it, ss)
    sw = L.Sweep(ctx, pts, law, 1e-12, 60, steps, 6 * count)
    assert sw.launch() == 0
    torch.cuda.synchronize()
    final = snapshot(st, sig, it, ss)
    sw.close()
    # the same steps eagerly, checked one at a time
    st.zero_()
    prev = np.zeros((count, kind))
    for t in range(steps):
        assert L.constitutive_update(ctx, L.points(d[t], st, sig, it, ss), law, 1e-12, 60) == 0
        torch.cuda.synchronize()
        g = {"state": st.cpu().numpy().T.copy(), "sig": sig.cpu().numpy().T.copy(),
             "iters": it.cpu().numpy().copy(), "status": ss.cpu().numpy().copy()}
        r = check_newton(Law(kind=kind), host[t], prev, 1e-12, 60, g)
        assert (g["status"] == 0).mean() > 0.98, r
        prev = g["state"]
    for a, b in zip(final, snapshot(st, sig, it, ss)):
        assert np.array_equal(a, b)


def test_same_increment_every_step_and_arguments(L, ctx):
    kind, count = 7, 1000
    law = L.make_law(kind)
    d, _, st, sig, it, ss, _ = buffers(kind, count, count, 1, seed=95)
    pts = L.points(d[0], st, sig, it, ss)
    for _ in range(3):
        assert L.constitutive_update(ctx, pts, law, 1e-12, 40) == 0
    torch.cuda.synchronize()
    ref = snapshot(st, sig, it, ss)
    st.zero_()
    sw = L.Sweep(ctx, pts, law, 1e-12, 40, 3, 0)
    assert sw.launch() == 0
    torch.cuda.synchronize()
    for a, b in zip(ref, snapshot(st, sig, it, ss)):
        assert np.array_equal(a, b)
    sw.close()
    with pytest.raises(L.LuppError) as e:
        L.Sweep(ctx, pts, law, 1e-12, 40, 0, 0)
    assert e.value.code == -6
    with pytest.raises(L.LuppError) as e:
        L.Sweep(ctx, pts, law, 1e-12, 40, 2, 5)
    assert e.value.code == -7
