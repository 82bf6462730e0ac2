"""GPU tests of the serving loop: continuous batching under an HBM budget.

* Every request's result is bitwise the same in a mixed, overlapping stream
  as when it runs alone (solves and Newton updates are computed per system /
  per point, independently of the rest of the batch).
* Admission respects the budget; a request larger than the whole budget is
  rejected; host-pointer requests work.
* Device-resident point state advances across update requests exactly as two
  successive oracle updates do (within the Newton tolerance).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import Law
from workloads import newton_points, systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_2609_15217_amd.lupp as L
    return L


@pytest.fixture(scope="module")
def ctx(L):
    return L.Context(0)


DEV = torch.device("cuda:0")


def make_stream(seed=0):
    """A deterministic mix of solve and update requests (device inputs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for k in range(24):
        if rng.uniform() < 0.6:
            n = int(rng.integers(2, 33))
            batch = int(rng.integers(500, 6000))
            A, b, _ = systems(n, batch, seed=1000 + k)
            reqs.append({"kind": "solve", "n": n, "batch": batch,
                         "A": torch.from_numpy(A).to(DEV), "b": torch.from_numpy(b).to(DEV)})
        else:
            reqs.append({"kind": "update", "set": int(rng.integers(0, 2)),
                         "deps": newton_points(3000, seed=2000 + k)})
    return reqs


def run_stream(L, ctx, reqs, budget, inflight, streams, one_at_a_time=False):
    srv = L.Server(ctx, budget, inflight, streams)
    sets = [L.lupp_server_add_points(srv, 7, 3000), L.lupp_server_add_points(srv, 13, 3000)]
    laws = [L.make_law(7), L.make_law(13)]
    outs, tickets, keep = [], [], []
    for q in reqs:
        if q["kind"] == "solve":
            x = torch.empty_like(q["b"])
            ip = torch.empty((q["batch"], q["n"]), dtype=torch.int32, device=DEV)
            inf = torch.empty(q["batch"], dtype=torch.int32, device=DEV)
            lu = torch.empty_like(q["A"])
            r = L.solve_request(q["n"], q["batch"], q["A"], q["b"], x, ip, inf, lu)
            outs.append((x, ip, inf, lu))
        else:
            d = torch.from_numpy(q["deps"].T.copy()).to(DEV)
            sig = torch.empty((6, 3000), dtype=torch.float64, device=DEV)
            it = torch.empty(3000, dtype=torch.int32, device=DEV)
            st = torch.empty(3000, dtype=torch.int32, device=DEV)
            r = L.update_request(sets[q["set"]], 3000, laws[q["set"]], d, sig, it, st)
            outs.append((sig, it, st))
            keep.append(d)
        t = L.lupp_server_submit(srv, r)
        assert t > 0
        tickets.append(t)
        if one_at_a_time:
            assert L.lupp_server_wait(srv, t)[0] == 0
    for t in tickets:
        if not one_at_a_time:
            rc, lat = L.lupp_server_wait(srv, t)
            assert rc == 0 and lat > 0
    stats = L.lupp_server_get_stats(srv)
    states = []
    for kind, sid in zip((7, 13), sets):
        buf = np.zeros((kind, 3000))
        assert L.lupp_server_read_points(srv, sid, buf) == 0
        states.append(buf)
    srv.close()
    torch.cuda.synchronize()
    return [[t.cpu().numpy() for t in o] for o in outs], states, stats


def test_results_same_alone_and_in_the_mix(L, ctx):
    reqs = make_stream(1)
    mixed, st_mixed, stats = run_stream(L, ctx, reqs, budget=256 << 20, inflight=6, streams=4)
    alone, st_alone, _ = run_stream(L, ctx, reqs, budget=256 << 20, inflight=1, streams=1,
                                    one_at_a_time=True)
    for a, b in zip(mixed, alone):
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
    for u, v in zip(st_mixed, st_alone):
        assert np.array_equal(u, v)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["peak_inflight"] >= 2          # requests really overlapped
    assert stats["peak_bytes"] <= 256 << 20
    # solves match the oracle bit for bit
    for q, o in zip(reqs, mixed):
        if q["kind"] == "solve":
            ref = oracle.gesv_batch(q["A"].cpu().numpy(), q["b"].cpu().numpy(), threads=8)
            assert np.array_equal(o[0], ref["x"]) and np.array_equal(o[1], ref["ipiv"])
            assert np.array_equal(o[3], ref["LU"])


def test_tight_budget_and_rejection(L, ctx):
    reqs = [q for q in make_stream(2) if q["kind"] == "solve"][:8]
    biggest = max(q["batch"] * (q["n"] * q["n"] * 8 + q["n"] * 12 + 4) for q in reqs) + (4 << 10)
    got, _, stats = run_stream(L, ctx, reqs, budget=biggest, inflight=8, streams=4)
    assert stats["completed"] == len(reqs)
    assert stats["peak_bytes"] <= biggest
    srv = L.Server(ctx, 1 << 20, 2, 1)
    A = torch.zeros((4096, 32, 32), dtype=torch.float64, device=DEV)
    b = torch.zeros((4096, 32), dtype=torch.float64, device=DEV)
    assert L.lupp_server_submit(srv, L.solve_request(32, 4096, A, b, b)) == L.LUPP_E_NOMEM
    assert L.lupp_server_get_stats(srv)["rejected"] == 1
    bad = L.solve_request(33, 10, A, b, b)
    assert L.lupp_server_submit(srv, bad) == -2
    srv.close()


def test_host_pointer_requests(L, ctx):
    A, b, _ = systems(12, 3000, seed=77)
    x = np.zeros_like(b)
    ip = np.zeros((3000, 12), dtype=np.int32)
    srv = L.Server(ctx, 64 << 20, 4, 2)
    t = L.lupp_server_submit(srv, L.solve_request(12, 3000, A, b, x, ip))
    assert t > 0 and L.lupp_server_wait(srv, t)[0] == 0
    srv.close()
    ref = oracle.gesv_batch(A, b, threads=4)
    assert np.array_equal(x, ref["x"]) and np.array_equal(ip, ref["ipiv"])


@pytest.mark.parametrize("kind", [7, 13])
def test_device_resident_state_two_steps(L, ctx, kind):
    law = Law(kind=kind)
    d1 = newton_points(2000, seed=81)
    d2 = newton_points(2000, seed=82, lo=-5e-4, hi=5e-4)
    # a second step from a non-virgin state needs more iterations than the
    # benchmark's 20; a larger cap keeps most points away from the stop rule's
    # boundary (a few 13-unknown points do not converge from the zero start)
    o1 = oracle.constitutive_update(law, d1, maxit=60, threads=8)
    o2 = oracle.constitutive_update(law, d2, o1["state"], maxit=60, threads=8)
    assert np.all(o1["status"] == 0) and (o2["status"] == 0).mean() > 0.99
    srv = L.Server(ctx, 64 << 20, 4, 2)
    sid = L.lupp_server_add_points(srv, kind, 2000)
    lw = L.make_law(kind)
    sig = np.zeros((6, 2000))
    st = np.zeros(2000, dtype=np.int32)
    it = np.zeros(2000, dtype=np.int32)
    for d in (d1, d2):
        dT = np.ascontiguousarray(d.T)  # must outlive the request
        t = L.lupp_server_submit(srv, L.update_request(sid, 2000, lw, dT, sig, it, st, maxit=60))
        assert L.lupp_server_wait(srv, t)[0] == 0
        del dT
    state = np.zeros((kind, 2000))
    assert L.lupp_server_read_points(srv, sid, state) == 0
    srv.close()
    assert (st == o2["status"]).mean() >= 0.995
    same = (it == o2["iters"]) & (st == 0) & (o2["status"] == 0)
    assert same.mean() > 0.98
    rel = np.abs(sig.T - o2["sig"]).max(axis=1) / np.abs(o2["sig"]).max(axis=1)
    assert rel[same].max() <= 1e-9
    srel = np.abs(state.T - o2["state"]).max(axis=1) / np.abs(o2["state"]).max(axis=1)
    assert srel[same].max() <= 1e-9
