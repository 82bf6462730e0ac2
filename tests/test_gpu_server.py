"""GPU tests of the serving loop: continuous batching under an HBM budget.

* Every request's result is bitwise the same in a mixed, overlapping stream
  as when it runs alone (solves and Newton updates are computed per system /
  per point, independently of the rest of the batch).
* Admission respects the budget; a request larger than the whole budget is
  rejected; host-pointer requests work.
* Device-resident point state advances across update requests: each step
  passes the every-point Newton parity against the oracle (1e-10), started
  from the state the server committed at the previous one.
"""
import numpy as np
import pytest
import torch

import oracle
from newton_check import check_newton
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


def run_stream(L, ctx, reqs, budget, inflight, streams, one_at_a_time=False, mode=0):
    srv = L.Server(ctx, budget, inflight, streams, mode)
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


@pytest.mark.parametrize("mode", [0, 1])
def test_results_same_alone_and_in_the_mix(L, ctx, mode):
    """Device-resident requests in an overlapping stream (merged passes, or
    one launch per request) against the same requests one at a time: bitwise
    the same; solves bitwise the oracle's; no arena used (everything is on
    the device)."""
    reqs = make_stream(1)
    mixed, st_mixed, stats = run_stream(L, ctx, reqs, budget=256 << 20, inflight=6, streams=4,
                                        mode=mode)
    alone, st_alone, _ = run_stream(L, ctx, reqs, budget=256 << 20, inflight=1, streams=1,
                                    one_at_a_time=True, mode=1)
    for a, b in zip(mixed, alone):
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
    for u, v in zip(st_mixed, st_alone):
        assert np.array_equal(u, v)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["peak_inflight"] >= 2          # requests really overlapped
    assert stats["peak_bytes"] == 0             # device data used in place
    assert stats["passes"] <= len(reqs) and stats["launches"] <= len(reqs)
    # solves match the oracle bit for bit
    for q, o in zip(reqs, mixed):
        if q["kind"] == "solve":
            ref = oracle.gesv_batch(q["A"].cpu().numpy(), q["b"].cpu().numpy(), threads=8)
            assert np.array_equal(o[0], ref["x"]) and np.array_equal(o[1], ref["ipiv"])
            assert np.array_equal(o[3], ref["LU"])


def staging_bytes(n, batch):
    """Arena bytes of a solve request whose buffers are all on the host (or
    NULL): matrix, right-hand sides, pivots, info."""
    r = lambda b: (b + 255) // 256 * 256
    return r(batch * n * n * 8) + r(batch * n * 8) + r(batch * n * 4) + r(batch * 4)


def update_staging_bytes(count):
    r = lambda b: (b + 255) // 256 * 256
    return 2 * r(count * 48) + 2 * r(count * 4)


@pytest.mark.parametrize("mode", [0, 1])
def test_requests_queued_behind_the_budget_run_as_one_pass(L, ctx, mode):
    """A large host-buffer request fills the whole arena; the host-buffer
    requests submitted behind it wait for arena space and are admitted
    together when it completes: in merged mode one pass with one grouped
    solve and one launch per law, otherwise one pass and one launch each.
    Results: solves bitwise the oracle's, updates every-point Newton parity,
    and both modes bitwise equal."""
    n0, b0 = 16, 400_000
    budget = staging_bytes(n0, b0)
    A0, bb0, _ = systems(n0, b0, seed=31)
    small = [(int(n), int(bt)) for n, bt in ((3, 700), (32, 90), (12, 1500), (17, 64), (1, 33),
                                             (8, 2049), (24, 300), (5, 999))]
    assert sum(staging_bytes(n, bt) for n, bt in small) + 4 * update_staging_bytes(2000) <= budget
    srv = L.Server(ctx, budget, 64, 4, mode)
    sets = {(k, i): L.lupp_server_add_points(srv, k, 2000) for k in (7, 13) for i in (0, 1)}
    laws = {7: L.make_law(7), 13: L.make_law(13)}
    x0 = np.zeros_like(bb0)
    tickets = [L.lupp_server_submit(srv, L.solve_request(n0, b0, A0, bb0, x0))]
    solves, updates = [], []
    for k, (n, bt) in enumerate(small):
        A, b, _ = systems(n, bt, seed=40 + k)
        out = (np.zeros_like(b), np.zeros((bt, n), dtype=np.int32), np.zeros(bt, dtype=np.int32),
               np.zeros_like(A))
        solves.append((A, b, out))
        tickets.append(L.lupp_server_submit(srv, L.solve_request(n, bt, A, b, *out)))
    for (kind, i), sid in sets.items():
        d = np.ascontiguousarray(newton_points(2000, seed=60 + kind + i).T)
        out = (np.zeros((6, 2000)), np.zeros(2000, dtype=np.int32), np.zeros(2000, dtype=np.int32))
        updates.append((kind, d, out))
        tickets.append(L.lupp_server_submit(srv, L.update_request(sid, 2000, laws[kind], d, *out)))
    assert all(t > 0 for t in tickets)
    for t in tickets:
        assert L.lupp_server_wait(srv, t)[0] == 0
    stats = L.lupp_server_get_stats(srv)
    states = {}
    for key, sid in sets.items():
        buf = np.zeros((key[0], 2000))
        assert L.lupp_server_read_points(srv, sid, buf) == 0
        states[key] = buf
    srv.close()
    nreq = 1 + len(small) + len(sets)
    assert stats["completed"] == nreq and stats["peak_bytes"] <= budget
    if mode == 0:
        assert stats["passes"] == 2 and stats["launches"] == 1 + 1 + 2, stats
    else:
        assert stats["passes"] == nreq and stats["launches"] == nreq, stats
    ref0 = oracle.gesv_batch(A0[:5000], bb0[:5000], threads=8)
    assert np.array_equal(x0[:5000], ref0["x"])
    for A, b, out in solves:
        ref = oracle.gesv_batch(A, b, threads=4)
        assert np.array_equal(out[0], ref["x"]) and np.array_equal(out[1], ref["ipiv"])
        assert np.array_equal(out[2], ref["info"]) and np.array_equal(out[3], ref["LU"])
    for (kind, i), (k2, d, out) in zip(sets, updates):
        g = {"state": states[(kind, i)].T.copy(), "sig": out[0].T.copy(), "iters": out[1],
             "status": out[2]}
        check_newton(Law(kind=kind), d.T.copy(), None, 1e-12, 20, g)


def test_device_inputs_take_no_arena_and_a_is_only_read(L, ctx):
    """32 MiB of device matrices through a 1 MiB server: nothing is staged
    (every buffer is on the device); with no lu requested the matrices are
    left as they were."""
    A, b, _ = systems(32, 4096, seed=71)
    tA = torch.from_numpy(A).to(DEV)
    tb = torch.from_numpy(b).to(DEV)
    x = torch.empty_like(tb)
    ip = torch.empty((4096, 32), dtype=torch.int32, device=DEV)
    inf = torch.empty(4096, dtype=torch.int32, device=DEV)
    srv = L.Server(ctx, 1 << 20, 2, 1)
    t = L.lupp_server_submit(srv, L.solve_request(32, 4096, tA, tb, x, ip, inf))
    assert t > 0 and L.lupp_server_wait(srv, t)[0] == 0
    assert L.lupp_server_get_stats(srv)["peak_bytes"] == 0
    srv.close()
    ref = oracle.gesv_batch(A, b, threads=8)
    assert np.array_equal(x.cpu().numpy(), ref["x"])
    assert np.array_equal(tA.cpu().numpy(), A) and np.array_equal(tb.cpu().numpy(), b)


def test_tight_budget_and_rejection(L, ctx):
    """Host-buffer requests through an arena that holds only the largest of
    them at a time; a request larger than the arena is rejected."""
    rng = np.random.Generator(np.random.PCG64(2))
    reqs = []
    for k in range(8):
        n, bt = int(rng.integers(2, 33)), int(rng.integers(500, 6000))
        A, b, _ = systems(n, bt, seed=1100 + k)
        reqs.append((n, bt, A, b, np.zeros_like(b), np.zeros((bt, n), dtype=np.int32)))
    biggest = max(staging_bytes(n, bt) for n, bt, *_ in reqs)
    srv = L.Server(ctx, biggest, 8, 4)
    tickets = [L.lupp_server_submit(srv, L.solve_request(n, bt, A, b, x, ip))
               for n, bt, A, b, x, ip in reqs]
    for t in tickets:
        assert t > 0 and L.lupp_server_wait(srv, t)[0] == 0
    stats = L.lupp_server_get_stats(srv)
    assert stats["completed"] == len(reqs) and stats["peak_bytes"] <= biggest
    srv.close()
    for n, bt, A, b, x, ip in reqs:
        ref = oracle.gesv_batch(A, b, threads=4)
        assert np.array_equal(x, ref["x"]) and np.array_equal(ip, ref["ipiv"])
    srv = L.Server(ctx, 1 << 20, 2, 1)
    A = np.zeros((4096, 32, 32))
    b = np.zeros((4096, 32))
    assert L.lupp_server_submit(srv, L.solve_request(32, 4096, A, b, b)) == L.LUPP_E_NOMEM
    assert L.lupp_server_get_stats(srv)["rejected"] == 1
    bad = L.solve_request(33, 10, A, b, b)
    assert L.lupp_server_submit(srv, bad) == -2
    srv.close()


def test_server_uses_the_creating_context_settings(L):
    """A context with tile-local pivoting (tile 4, threshold 1e-10): the
    server's solves follow it (the oracle's tiled mode), not textbook
    pivoting."""
    c2 = L.Context(0)
    assert L.lupp_set_pivoting(c2, 4, 1e-10) == 0
    A, b, _ = systems(8, 3000, seed=73)
    x = np.zeros_like(b)
    ip = np.zeros((3000, 8), dtype=np.int32)
    srv = L.Server(c2, 64 << 20, 4, 2)
    t = L.lupp_server_submit(srv, L.solve_request(8, 3000, A, b, x, ip))
    assert t > 0 and L.lupp_server_wait(srv, t)[0] == 0
    srv.close()
    c2.close()
    ref = oracle.gesv_batch_tiled(A, b, tile=4, thresh=1e-10, threads=4)
    textbook = oracle.gesv_batch(A, b, threads=4)
    assert np.array_equal(ip, ref["ipiv"]) and np.array_equal(x, ref["x"])
    assert not np.array_equal(ip, textbook["ipiv"])


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
    """Two update requests on one registered point set: each step passes the
    every-point Newton parity against the oracle (1e-10), the second started
    from the state the server committed at the first."""
    law = Law(kind=kind)
    d1 = newton_points(2000, seed=81)
    d2 = newton_points(2000, seed=82, lo=-5e-4, hi=5e-4)
    # a second step from a non-virgin state needs more iterations than the
    # benchmark's 20; a larger cap keeps most points away from the stop rule's
    # boundary (a few 13-unknown points do not converge from the zero start)
    srv = L.Server(ctx, 64 << 20, 4, 2)
    sid = L.lupp_server_add_points(srv, kind, 2000)
    lw = L.make_law(kind)
    prev = np.zeros((2000, kind))
    for d in (d1, d2):
        sig = np.zeros((6, 2000))
        st = np.zeros(2000, dtype=np.int32)
        it = np.zeros(2000, dtype=np.int32)
        dT = np.ascontiguousarray(d.T)  # must outlive the request
        t = L.lupp_server_submit(srv, L.update_request(sid, 2000, lw, dT, sig, it, st, maxit=60))
        assert L.lupp_server_wait(srv, t)[0] == 0
        del dT
        state = np.zeros((kind, 2000))
        assert L.lupp_server_read_points(srv, sid, state) == 0
        g = {"state": state.T.copy(), "sig": sig.T.copy(), "iters": it, "status": st}
        check_newton(law, d, prev, 1e-12, 60, g)
        assert (st == 0).mean() > 0.99
        prev = g["state"]
    srv.close()
