"""Benchmark: batched FP64 LU with partial pivoting + substitution for tiny
systems, and the fused Newton constitutive update, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

One step = one pass of the standalone-solve sweep: 2^20 independent systems
for each n in {8, 12, 16, 24, 32} (A ~ N(0,1) resampled while
cond2(A) > 1e4, b = A x_true, x_true ~ U(-1,1)), solved in the interleaved
SoA layout and in the AoS layout (10 launches of lupp_batched_solve). The
solve is in place, so every step starts from inputs restored from a pristine
device copy outside the timed region. `value` is systems solved per second
over the timed steps. n = 4 is timed beside the step (the 4..32 figure).

Also reported: the fused Newton update (2^20 points, Norton 7x7 and
Norton+Armstrong-Frederick 13x13), per-call latency p50/p99 of a 4096-system
n = 8 solve, per-kernel durations and roofline fractions, and the CPU oracle
timed on this host on a bounded sample.

Profiling helpers (for rocprofv3):
    python bench.py --only 32:soa --reps 20     run one (n, layout) kernel only
    python bench.py --only newton:13 --reps 5   run one fused Newton update only
    python bench.py --copy-calibration          a plain 2 GiB device copy
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 systems solved/s (n=8..32) + Newton updates/s; p50/p99 latency"
SIZES = (4, 8, 12, 16, 24, 32)
STEP_SIZES = (8, 12, 16, 24, 32)  # the sizes the metric names; n = 4 is reported beside them
BATCH = 1 << 20
# ldbatch of the interleaved arrays: rows of one matrix element 8 MiB + 1.5 KiB
# apart rather than exactly 8 MiB. With a power-of-two row stride the 1024
# lines one workgroup reads (one per element) fall on few HBM channels;
# measured with N(0,1) matrices: n = 16 1.12 -> 0.98 ms, n = 32 6.84 ->
# 6.53 ms, n = 8 unchanged.
SOA_LD = BATCH + 192
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def bytes_per_system(n: int) -> int:
    """dgesv traffic: read A and b, write L\\U, x, ipiv (int32) and info."""
    return 16 * n * n + 20 * n + 4


def flops_per_system(n: int) -> int:
    """Factorisation sum_{m=1}^{n-1} (m + 2 m^2) plus the two triangular
    solves 2 n^2 - n."""
    return sum(m + 2 * m * m for m in range(1, n)) + 2 * n * n - n


# Operations (add, sub, mul, div, sqrt, pow: one each) of one evaluation of
# the law's residual and exact Jacobian (Section 2.1, eqs. 1-3) as the oracle's
# law routine executes them, counted by compiling that routine against a
# counting number type (oracle/law_flops.py; a test keeps these values equal
# to its output). The oracle forms the Jacobian with full 6 x 6 products by
# the deviatoric projector, so the figure bounds from above what the law
# needs. A point evaluates the law at every iterate: solves + 1 times.
LAW_FLOPS = {7: 869, 13: 1331}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# the sources the standalone-solve kernels are compiled from, the dispatch
# table that picks them and the compile flags: counters taken on other
# sources do not describe the kernels this run launches
KERNEL_SOURCES = ("include/lupp.h", "include/lupp_device.h",
                  "paper_2609_15217_amd/csrc/internal.h",
                  "paper_2609_15217_amd/csrc/kernels_thread.h",
                  "paper_2609_15217_amd/csrc/kernels_lanes.h",
                  "paper_2609_15217_amd/csrc/kernels_lanes_soa.h",
                  "paper_2609_15217_amd/dispatch_gfx950.json")


def kernel_source_hash() -> str:
    from paper_2609_15217_amd.build import CXXFLAGS
    h = hashlib.sha256(" ".join(f for f in CXXFLAGS if not f.startswith("/")).encode())
    for rel in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key: str):
    """HBM traffic per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    rec = data.get(kernel_key)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_baseline(host, sizes, newton=True, runs=10):
    """The CPU oracle as it stands, timed on this host: every core this
    process may use (the pool's share, at most 16) and one core; one warm-up
    then `runs` timed runs, median. Bounded samples: the first systems of the
    sweep's inputs per n, and the first points of the Newton workload."""
    import oracle
    from workloads import newton_points
    cores = min(16, len(os.sched_getaffinity(0)))

    def median_time(fn):
        fn()
        ts = []
        for _ in range(runs):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    def solve_rate(per_n, threads):
        def go():
            for n in sizes:
                A, b = host[n]
                oracle.gesv_batch(A[:per_n], b[:per_n], threads=threads)
        return len(sizes) * per_n / median_time(go)

    S_all, S_one = 1 << 18, 1 << 14
    out = {"value": round(solve_rate(S_all, cores)), "unit": "systems/s", "cores": cores,
           "kind": "oracle", "model": cpu_model(), "nproc": os.cpu_count(),
           "median_of": runs, "warmup": 1,
           "sample": f"first {S_all} systems of each n in {list(sizes)} of the sweep's inputs "
                     f"(AoS; the oracle has one layout), {cores} threads",
           "one_core": {"systems_per_s": round(solve_rate(S_one, 1)),
                        "sample": f"first {S_one} systems of each n, 1 thread"}}
    if newton:
        nt = {}
        for kind in (7, 13):
            for label, P, th in (("all", 1 << 16, cores), ("one_core", 1 << 12, 1)):
                deps = newton_points(P, seed=4)
                dt = median_time(lambda: oracle.constitutive_update(oracle.Law(kind=kind), deps,
                                                                    threads=th))
                nt[f"norton{kind}_updates_per_s" + ("" if label == "all" else "_one_core")] = \
                    round(P / dt)
        nt["sample"] = "first 65536 (all cores) / 4096 (one core) points of the benchmark increments"
        out["newton"] = nt
    return out


class ServingPools:
    """Device-resident request payloads (an upstream GPU producer): seeded
    random matrices, right-hand sides and strain increments, and output rings,
    allocated once for every serving run."""

    MAX_SYS, MAX_PTS, SLOTS = 1_000_000, 500_000, 64

    def __init__(self, torch, dev):
        g = torch.Generator(device=dev)
        g.manual_seed(5)
        M, P, S = self.MAX_SYS, self.MAX_PTS, self.SLOTS
        self.A = torch.randn(M * 32 * 32, generator=g, dtype=torch.float64, device=dev)
        self.b = torch.randn(M * 32, generator=g, dtype=torch.float64, device=dev)
        self.d = (torch.rand(6 * P, generator=g, dtype=torch.float64, device=dev) - 0.5) * 4e-3
        self.x = torch.empty((S, M * 32), dtype=torch.float64, device=dev)
        self.ip = torch.empty((S, M * 32), dtype=torch.int32, device=dev)
        self.sig = torch.empty((S, 6 * P), dtype=torch.float64, device=dev)
        self.its = torch.empty((S, 2 * P), dtype=torch.int32, device=dev)


def run_serving(L, ctx, pools, seconds: float, rate: float, mode: int, seed: int = 5):
    """Poisson stream of requests (half solve batches, n ~ U{2..32}, 1k-1M
    systems; half Newton updates of device-resident point sets, 1k-500k
    points, 7x7 or 13x13 law) submitted to the serving loop at their arrival
    times for `seconds` of wall time. Latency runs from the scheduled arrival
    to completion (queueing behind the client's 64 outstanding requests
    included)."""
    import threading

    from workloads import serving_requests
    reqs = serving_requests(int(rate * seconds) + 1, seed=seed, rate=rate)
    reqs = [q for q in reqs if q["t"] <= seconds]
    srv = L.Server(ctx, 48 << 30, 64, 8, mode)
    rng = np.random.Generator(np.random.PCG64(55))
    sets = {7: [], 13: []}
    for kind in (7, 13):
        for _ in range(16):
            cnt = int(round(np.exp(rng.uniform(np.log(1_000), np.log(pools.MAX_PTS)))))
            sets[kind].append((L.lupp_server_add_points(srv, kind, cnt), cnt))
    laws = {7: L.make_law(7), 13: L.make_law(13)}
    done = []
    lock = threading.Semaphore(pools.SLOTS)
    tickets = []
    cv = threading.Condition()

    def collector():
        k = 0
        while True:
            with cv:
                while k >= len(tickets):
                    cv.wait()
                item = tickets[k]
            if item is None:
                return
            t, arrival, submit_at, q = item
            rc, lat = L.lupp_server_wait(srv, t)
            done.append((rc, lat + 1e3 * (submit_at - arrival), q))
            lock.release()
            k += 1

    th = threading.Thread(target=collector)
    th.start()
    ms_sys = ms_pts = 0
    submitted = 0
    t0 = time.perf_counter()
    for k, q in enumerate(reqs):
        now = time.perf_counter() - t0
        if now > seconds:  # overloaded: stop offering at the end of the window
            break
        if q["t"] > now:
            time.sleep(q["t"] - now)
        lock.acquire()
        slot = k % pools.SLOTS
        if q["kind"] == "solve":
            n, bsz = q["n"], min(q["size"], pools.MAX_SYS)
            r = L.solve_request(n, bsz, pools.A.data_ptr(), pools.b.data_ptr(),
                                pools.x[slot].data_ptr(), None, pools.ip[slot].data_ptr())
            ms_sys += bsz
        else:
            sid, cnt = sets[q["law"]][int(rng.integers(0, 16))]
            r = L.update_request(sid, cnt, laws[q["law"]], pools.d.data_ptr(),
                                 pools.sig[slot].data_ptr(), pools.its[slot].data_ptr(),
                                 pools.its[slot].data_ptr() + 4 * pools.MAX_PTS)
            ms_pts += cnt
        submit_at = time.perf_counter() - t0
        t = L.lupp_server_submit(srv, r)
        if t <= 0:
            raise RuntimeError(f"serving submit: {L.lupp_error_string(t)}")
        submitted += 1
        with cv:
            tickets.append((t, q["t"], submit_at, q))
            cv.notify()
    with cv:
        tickets.append(None)
        cv.notify()
    th.join()
    wall = time.perf_counter() - t0
    stats = L.lupp_server_get_stats(srv)
    srv.close()
    lat = np.array([d[1] for d in done if d[0] == 0])
    failed = sum(1 for d in done if d[0] != 0)
    out = {"rate_offered": rate, "mode": "merged" if mode == 0 else "per_request",
           "seconds": seconds, "requests_offered": len(reqs), "requests": submitted,
           "failed": failed, "wall_s": round(wall, 3),
           "p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "systems_per_s": round(ms_sys / wall), "updates_per_s": round(ms_pts / wall),
           "achieved_req_per_s": round(submitted / wall, 1),
           "passes": stats["passes"], "launches": stats["launches"],
           "peak_inflight": stats["peak_inflight"], "peak_bytes": stats["peak_bytes"]}
    log(f"serving {out['mode']} {rate:.0f} req/s x {seconds:.0f} s: p50 {out['p50_ms']} ms "
        f"p99 {out['p99_ms']} ms, {out['achieved_req_per_s']} req/s, {out['launches']} launches "
        f"for {submitted} requests")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-newton", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-sweep-seconds", type=float, default=5.0)
    ap.add_argument("--only", default=None,
                    help="n:layout (e.g. 32:soa) or newton:kind (7 or 13): run that kernel only")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every system and integration point is independent, "
              "so the path runs on one GPU's share; multi-GPU execution is not implemented.",
              flush=True)
        sys.exit(2)

    import torch

    import paper_2609_15217_amd.lupp as L
    from workloads import aos_to_soa, newton_points, systems

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float64, device=dev).fill_(1.0)  # 2 GiB
        dst = torch.empty_like(src)
        for _ in range(args.reps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": src.numel() * 8,
                          "reps": args.reps}), flush=True)
        return

    ctx = L.Context(0)
    if args.only and args.only.startswith("newton:"):
        # one fused Newton update of 2^20 points, `reps` times (profiling)
        kind = int(args.only.split(":")[1])
        count = 1 << 20
        d = torch.from_numpy(newton_points(count, seed=4).T.copy()).to(dev)
        st = torch.zeros((kind, count), dtype=torch.float64, device=dev)
        sig = torch.empty((6, count), dtype=torch.float64, device=dev)
        it = torch.empty(count, dtype=torch.int32, device=dev)
        stt = torch.empty(count, dtype=torch.int32, device=dev)
        pts = L.points(d, st, sig, it, stt)
        law = L.make_law(kind)
        for r in range(args.reps):
            st.zero_()
            rc = L.constitutive_update(ctx, pts, law, 1e-12, 20, stream)
            if rc != 0:
                raise RuntimeError(L.lupp_error_string(rc))
        torch.cuda.synchronize()
        log(f"--only {args.only}: {args.reps} launches done, mean solves/point "
            f"{it.double().mean().item():.3f}")
        return
    sizes = SIZES
    layouts = ("soa", "aos")
    if args.only:
        n_s, lay = args.only.split(":")
        sizes, layouts = (int(n_s),), (lay,)

    # ---------------------------------------------------------------- inputs
    t0 = time.time()
    pristine, work, host = {}, {}, {}
    for n in sizes:
        A, b, _ = systems(n, BATCH, seed=2000 + n, kappa_max=1e4)
        host[n] = (A, b)
        tA = torch.from_numpy(A).to(dev)
        tb = torch.from_numpy(b).to(dev)
        for lay in layouts:
            if lay == "soa":
                pA = torch.zeros((n, n, SOA_LD), dtype=torch.float64, device=dev)
                pA[:, :, :BATCH] = tA.permute(1, 2, 0)
                pb = torch.zeros((n, SOA_LD), dtype=torch.float64, device=dev)
                pb[:, :BATCH] = tb.t()
            else:
                pA, pb = tA, tb
            pristine[(n, lay)] = (pA, pb)
            wA, wb = torch.empty_like(pA), torch.empty_like(pb)
            pshape = (n, SOA_LD) if lay == "soa" else (BATCH, n)
            ipiv = torch.empty(pshape, dtype=torch.int32, device=dev)
            info = torch.empty(BATCH, dtype=torch.int32, device=dev)
            work[(n, lay)] = (wA, wb, ipiv, info)
        del tA, tb
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f}s")

    def restore():
        for key, (pA, pb) in pristine.items():
            wA, wb, _, _ = work[key]
            wA.copy_(pA)
            wb.copy_(pb)

    def launch(key, flags=0):
        n, lay = key
        wA, wb, ipiv, info = work[key]
        layout = L.LUPP_SOA if lay == "soa" else L.LUPP_AOS
        sA, sB = (SOA_LD, SOA_LD) if lay == "soa" else (n * n, n)
        rc = L.lupp_batched_solve(ctx, n, BATCH, layout, wA, n, sA, wb, sB, ipiv, info, flags,
                                  stream)
        if rc != 0:
            raise RuntimeError(f"lupp_batched_solve n={n} {lay}: {L.lupp_error_string(rc)}")

    keys = [(n, lay) for n in sizes for lay in layouts]

    if args.only:
        for r in range(args.reps):
            restore()
            launch(keys[0])
        torch.cuda.synchronize()
        log(f"--only {args.only}: {args.reps} launches done")
        return

    # ------------------------------------------------------------- sweep
    # the timed step: every (n, layout) of n = 8..32; the n = 4 launches are
    # timed the same way after the steps, outside the step's clock
    step_keys = [k for k in keys if k[0] in STEP_SIZES]
    extra_keys = [k for k in keys if k[0] not in STEP_SIZES]
    ev = {k: [] for k in keys}
    for w in range(args.warmup):
        restore()
        for k in keys:
            launch(k)
        torch.cuda.synchronize()
        log(f"warmup step {w + 1}/{args.warmup} done")
    total = 0.0
    for s in range(args.steps):
        restore()
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in step_keys:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            launch(k)
            e1.record(stream)
            ev[k].append((e0, e1))
        torch.cuda.synchronize()
        total += time.perf_counter() - t_start
        for k in extra_keys:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            launch(k)
            e1.record(stream)
            ev[k].append((e0, e1))
        torch.cuda.synchronize()
        log(f"step {s + 1}/{args.steps} done")
    systems_per_step = len(step_keys) * BATCH
    value = systems_per_step * args.steps / total
    ms_per_step = 1000.0 * total / args.steps

    # correctness guard: every system solved
    for k in keys:
        info = work[k][3]
        bad = int((info != 0).sum().item())
        if bad:
            raise RuntimeError(f"{bad} systems with info != 0 for {k}")

    per_kernel = []
    for k in keys:
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev[k]]))
        n, lay = k
        gbs = bytes_per_system(n) * BATCH / (ms * 1e-3) / 1e9
        tfl = flops_per_system(n) * BATCH / (ms * 1e-3) / 1e12
        v, lanes, wpb = L.lupp_get_dispatch(ctx, n, L.LUPP_SOA if lay == "soa" else L.LUPP_AOS, BATCH)
        per_kernel.append({"n": n, "layout": lay, "ms": round(ms, 4),
                           "systems_per_s": round(BATCH / (ms * 1e-3)),
                           "GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                           "fp64_TFLOPs": round(tfl, 3),
                           "variant": "thread" if v == 1 else f"lanes{lanes}", "wpb": wpb})
    extra_ms = sum(r["ms"] for r in per_kernel if r["n"] not in STEP_SIZES)
    sweep_all = {"sizes": list(sizes), "systems_per_s": round(
        len(keys) * BATCH / ((ms_per_step + extra_ms) * 1e-3)),
        "note": "every (n, layout) of the sweep including n = 4: step time plus the n = 4 "
                "launches' event time"}
    dom = max(per_kernel, key=lambda r: r["ms"])
    dom_key = f"lupp_n{dom['n']}_{dom['layout']}"
    achieved = dom["GBps"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": load_traffic(dom_key), "kernel": dom_key,
                "algorithmic_bytes_per_launch": bytes_per_system(dom["n"]) * BATCH}

    # ------------------------------------------------------------- tile-local pivoting
    # the same kernels under the Tiled solvers' pivoting rule (tile 4,
    # threshold 1e-10): on these inputs no pivot leaves its tile
    tiled = {}
    if not args.only:
        assert L.lupp_set_pivoting(ctx, 4, 1e-10) == 0
        for k in keys:
            if k[0] not in (8, 16, 32):
                continue
            tt = []
            for r in range(args.warmup + min(args.steps, 3)):
                restore()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                launch(k)
                e1.record(stream)
                torch.cuda.synchronize()
                if r >= args.warmup:
                    tt.append(e0.elapsed_time(e1))
            base = next(r for r in per_kernel if (r["n"], r["layout"]) == k)["ms"]
            tiled[f"n{k[0]}_{k[1]}"] = {"ms": round(float(np.mean(tt)), 4), "textbook_ms": base}
        assert L.lupp_set_pivoting(ctx, 0, 0.0) == 0
        log(f"tile-local pivoting: {tiled}")

    # ------------------------------------------------------------- FMA mode
    # the same sweep kernels with every multiply-subtract fused (LUPP_FMA)
    fma_mode = {}
    if not args.only:
        for k in keys:
            tt = []
            for r in range(args.warmup + min(args.steps, 3)):
                restore()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                launch(k, L.LUPP_FMA)
                e1.record(stream)
                torch.cuda.synchronize()
                if r >= args.warmup:
                    tt.append(e0.elapsed_time(e1))
            base = next(r for r in per_kernel if (r["n"], r["layout"]) == k)["ms"]
            fma_mode[f"n{k[0]}_{k[1]}"] = {"ms": round(float(np.mean(tt)), 4), "strict_ms": base}
        fma_total = sum(v["ms"] for kk, v in fma_mode.items() if int(kk[1:].split("_")[0]) in STEP_SIZES)
        fma_mode["sweep_systems_per_s"] = round(len(step_keys) * BATCH / (fma_total * 1e-3))
        log(f"FMA mode: {fma_mode}")

    # ------------------------------------------------------------- ragged
    ragged = {}
    if not args.no_ragged:
        # free the sweep buffers first
        pristine.clear()
        work.clear()
        torch.cuda.empty_cache()
        from workloads import mixed_systems
        t1 = time.time()
        mx = mixed_systems(2_000_000, seed=3)
        log(f"mixed batch generated in {time.time() - t1:.1f}s")
        nb = int(mx["n"].size)
        tn = torch.from_numpy(mx["n"]).to(dev)
        toA = torch.from_numpy(mx["offA"]).to(dev)
        toB = torch.from_numpy(mx["offB"]).to(dev)
        pA = torch.from_numpy(mx["A"]).to(dev)
        pb = torch.from_numpy(mx["b"]).to(dev)
        wA, wb = torch.empty_like(pA), torch.empty_like(pb)
        rip = torch.empty(pb.numel(), dtype=torch.int32, device=dev)
        rin = torch.empty(nb, dtype=torch.int32, device=dev)
        n64 = mx["n"].astype(np.int64)
        alg_bytes = int((16 * n64 * n64 + 20 * n64 + 4).sum()) + nb * (4 + 16)
        alg_flops = int(sum(flops_per_system(n) * int((mx["n"] == n).sum()) for n in range(2, 33)))
        for mode, flags in (("class_launches", 0), ("per_size", L.LUPP_RAGGED_PER_SIZE)):
            times = []
            for r in range(args.warmup + args.steps):
                wA.copy_(pA)
                wb.copy_(pb)
                torch.cuda.synchronize()
                t_s = time.perf_counter()
                rc = L.lupp_batched_solve_ragged(ctx, nb, tn, toA, toB, wA, wb, rip, rin, flags, stream)
                torch.cuda.synchronize()
                if rc != 0:
                    raise RuntimeError(f"ragged {mode}: {L.lupp_error_string(rc)}")
                if r >= args.warmup:
                    times.append(time.perf_counter() - t_s)
            if int((rin != 0).sum().item()):
                raise RuntimeError(f"ragged {mode}: systems with info != 0")
            sec = float(np.median(times))
            ragged[mode] = {"ms": round(sec * 1e3, 3), "systems_per_s": round(nb / sec),
                            "GBps": round(alg_bytes / sec / 1e9, 1),
                            "hbm_frac": round(alg_bytes / sec / 1e9 / HBM_PEAK_GBS, 4),
                            "fp64_TFLOPs": round(alg_flops / sec / 1e12, 3)}
            log(f"ragged {mode}: {sec * 1e3:.2f} ms")
        ragged["workload"] = ("2,000,000 FP64 systems, n ~ U{2..32}, A ~ N(0,1) rejected if "
                              "cond2 > 1e4, AoS packed with int64 offsets, seed 3")
        ragged["algorithmic_bytes"] = alg_bytes
        ragged["lanes_per_size"] = {n: L.lupp_get_ragged_lanes(ctx, n) for n in range(1, 33)}
        ragged["speedup_classes_vs_per_size"] = round(
            ragged["per_size"]["ms"] / ragged["class_launches"]["ms"], 3)
        del tn, toA, toB, pA, pb, wA, wb, rip, rin, mx
        torch.cuda.empty_cache()

    # ------------------------------------------------------------- serving
    serving = {}
    if args.serve_seconds > 0:
        pools = ServingPools(torch, dev)
        main_run = run_serving(L, ctx, pools, args.serve_seconds, 2000.0, 0)
        sweep_runs = [run_serving(L, ctx, pools, args.serve_sweep_seconds, r, 0, seed=6)
                      for r in (1000.0, 4000.0, 8000.0, 16000.0, 32000.0)]
        per_request = [run_serving(L, ctx, pools, args.serve_sweep_seconds, r, 1, seed=6)
                       for r in (2000.0, 8000.0)]
        serving = dict(main_run)
        serving["workload"] = ("Poisson arrivals: 50% solve requests (n ~ U{2..32}, 1k-1M systems, "
                               "log-uniform), 50% Newton updates of device-resident point sets "
                               "(1k-500k points, 7x7/13x13 at 50/50); device-resident payloads")
        serving["rate_sweep"] = sweep_runs
        serving["per_request_mode"] = per_request
        del pools
        torch.cuda.empty_cache()

    # ------------------------------------------------------------- latency
    lat = {}
    A1, b1, _ = systems(8, 4096, seed=1)
    pA1 = torch.from_numpy(A1).to(dev)
    pb1 = torch.from_numpy(b1).to(dev)
    wA1, wb1 = torch.empty_like(pA1), torch.empty_like(pb1)
    ip1 = torch.empty((4096, 8), dtype=torch.int32, device=dev)
    in1 = torch.empty(4096, dtype=torch.int32, device=dev)
    samples = []
    for r in range(220):
        wA1.copy_(pA1)
        wb1.copy_(pb1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rc = L.lupp_batched_solve(ctx, 8, 4096, L.LUPP_AOS, wA1, 8, 64, wb1, 8, ip1, in1, 0, stream)
        e1.record(stream)
        assert rc == 0
        samples.append((e0, e1))
    torch.cuda.synchronize()
    us = np.array([a.elapsed_time(b) * 1000.0 for a, b in samples[20:]])
    lat = {"workload": "4096 systems, n=8, AoS, N(0,1), seed 1", "p50_us": round(float(np.percentile(us, 50)), 2),
           "p99_us": round(float(np.percentile(us, 99)), 2),
           "systems_per_s_at_p50": round(4096 / (np.percentile(us, 50) * 1e-6))}
    log(f"latency p50 {lat['p50_us']} us")

    # ------------------------------------------------------------- Newton
    newton = {}
    if not args.no_newton:
        count = 1 << 20
        deps = newton_points(count, seed=4)
        d = torch.from_numpy(deps.T.copy()).to(dev)
        for kind in (7, 13):
            st = torch.zeros((kind, count), dtype=torch.float64, device=dev)
            sig = torch.empty((6, count), dtype=torch.float64, device=dev)
            it = torch.empty(count, dtype=torch.int32, device=dev)
            stt = torch.empty(count, dtype=torch.int32, device=dev)
            pts = L.points(d, st, sig, it, stt)
            law = L.make_law(kind)
            times = []
            for r in range(args.warmup + args.steps):
                st.zero_()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                rc = L.constitutive_update(ctx, pts, law, 1e-12, 20, stream)
                e1.record(stream)
                assert rc == 0
                torch.cuda.synchronize()
                if r >= args.warmup:
                    times.append(e0.elapsed_time(e1))
            ms = float(np.mean(times))
            its = it.double().sum().item()
            conv = int((stt == 0).sum().item())
            # every mapping of the fused update (one lane or T lanes per point)
            mapping = {}
            _, default_lanes = L.lupp_get_newton_variant(ctx, kind)
            for lanes in ((1, 4, 8) if kind == 7 else (1, 8, 16)):
                assert L.lupp_set_newton_variant(ctx, kind, lanes) == 0
                mt = []
                for r in range(args.warmup + min(args.steps, 3)):
                    st.zero_()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    assert L.constitutive_update(ctx, pts, law, 1e-12, 20, stream) == 0
                    e1.record(stream)
                    torch.cuda.synchronize()
                    if r >= args.warmup:
                        mt.append(e0.elapsed_time(e1))
                mapping[f"lanes{lanes}_ms"] = round(float(np.mean(mt)), 3)
            assert L.lupp_set_newton_variant(ctx, kind, 0) == 0
            # the same update plus the consistent tangent of every converged
            # point (one multi-right-hand-side solve after convergence)
            tan = torch.empty((36, count), dtype=torch.float64, device=dev)
            pts_t = L.points(d, st, sig, it, stt, tan)
            ttimes = []
            for r in range(args.warmup + args.steps):
                st.zero_()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                rc = L.constitutive_update(ctx, pts_t, law, 1e-12, 20, stream)
                e1.record(stream)
                assert rc == 0
                torch.cuda.synchronize()
                if r >= args.warmup:
                    ttimes.append(e0.elapsed_time(e1))
            tms = float(np.mean(ttimes))
            # the CPU-driven batched form (Algorithm 1) of the same update
            bt = {}
            for name, flags in (("batched", 0), ("batched_graph", L.LUPP_BATCHED_GRAPH)):
                times_b = []
                for r in range(args.warmup + min(args.steps, 3)):
                    st.zero_()
                    torch.cuda.synchronize()
                    t_s = time.perf_counter()
                    rc, host_iters = L.constitutive_update_batched(ctx, pts, law, 1e-12, 20, flags,
                                                                   stream)
                    torch.cuda.synchronize()
                    assert rc == 0
                    if r >= args.warmup:
                        times_b.append(time.perf_counter() - t_s)
                bt[name] = (float(np.median(times_b)) * 1e3, host_iters)
            newton[f"norton{kind}"] = {"points": count, "ms": round(ms, 3),
                                       "updates_per_s": round(count / (ms * 1e-3)),
                                       "newton_iterations_per_s": round(its / (ms * 1e-3)),
                                       "mean_solves_per_point": round(its / count, 3),
                                       # FP64 rate of the linear solves alone (dgesv flops of
                                       # an n x n system per Newton iteration; the law's
                                       # residual, Jacobian, pow and sqrt are not counted)
                                       "solve_fp64_TFLOPs": round(
                                           its * flops_per_system(kind) / (ms * 1e-3) / 1e12, 3),
                                       "solve_fp64_frac": round(
                                           its * flops_per_system(kind) / (ms * 1e-3) / 1e12
                                           / FP64_PEAK_TFLOPS, 4),
                                       # the same plus the law at every iterate, counted
                                       # on the oracle's formulation (LAW_FLOPS)
                                       "fp64_TFLOPs_with_law": round(
                                           (its * flops_per_system(kind)
                                            + (its + count) * LAW_FLOPS[kind])
                                           / (ms * 1e-3) / 1e12, 3),
                                       "fp64_frac_with_law": round(
                                           (its * flops_per_system(kind)
                                            + (its + count) * LAW_FLOPS[kind])
                                           / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
                                       "converged": conv,
                                       "default_lanes_per_point": default_lanes,
                                       "mapping": mapping,
                                       "with_tangent_ms": round(tms, 3),
                                       "with_tangent_updates_per_s": round(count / (tms * 1e-3)),
                                       "batched_cpu_driven_ms": round(bt["batched"][0], 3),
                                       "batched_graph_ms": round(bt["batched_graph"][0], 3),
                                       "batched_host_iterations": bt["batched"][1],
                                       "fused_speedup_vs_batched": round(bt["batched"][0] / ms, 2)}
            del tan
            log(f"newton {kind}: {ms:.2f} ms, with tangent {tms:.2f} ms, batched "
                f"{bt['batched'][0]:.2f} ms, batched graph {bt['batched_graph'][0]:.2f} ms")

    # ------------------------------------------------------------- sweeps
    sweep = {}
    if not args.no_newton:
        # a small point set advanced over many time steps: one launch per step
        # versus the steps captured once in a HIP graph and replayed
        count, nsteps = 16384, 100
        dsw = torch.from_numpy(newton_points(count, seed=4, lo=-2e-4, hi=2e-4).T.copy()).to(dev)
        st = torch.zeros((7, count), dtype=torch.float64, device=dev)
        sig = torch.empty((6, count), dtype=torch.float64, device=dev)
        it = torch.empty(count, dtype=torch.int32, device=dev)
        stt = torch.empty(count, dtype=torch.int32, device=dev)
        pts = L.points(dsw, st, sig, it, stt)
        law = L.make_law(7)
        graph = L.Sweep(ctx, pts, law, 1e-12, 20, nsteps, 0)
        res = {}
        for mode in ("eager", "graph"):
            times = []
            for r in range(args.warmup + args.steps):
                st.zero_()
                torch.cuda.synchronize()
                t_s = time.perf_counter()
                if mode == "eager":
                    for _ in range(nsteps):
                        assert L.constitutive_update(ctx, pts, law, 1e-12, 20, stream) == 0
                else:
                    assert graph.launch(stream) == 0
                torch.cuda.synchronize()
                if r >= args.warmup:
                    times.append(time.perf_counter() - t_s)
            res[mode] = float(np.median(times))
        graph.close()
        sweep = {"workload": f"{count} points, Norton 7x7, {nsteps} time steps of the same "
                             "increment (U(-2e-4, 2e-4) per Kelvin component, seed 4)",
                 "eager_ms": round(res["eager"] * 1e3, 3), "graph_ms": round(res["graph"] * 1e3, 3),
                 "graph_updates_per_s": round(count * nsteps / res["graph"]),
                 "speedup_graph_vs_eager": round(res["eager"] / res["graph"], 3)}
        log(f"sweep: eager {sweep['eager_ms']} ms, graph {sweep['graph_ms']} ms")
        del dsw, st, sig, it, stt

    # ------------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle_baseline(host, sizes, newton=not args.no_newton)
        log(f"cpu oracle {cpu['value']} systems/s on {cpu['cores']} threads, "
            f"{cpu['one_core']['systems_per_s']} on one")

    out = {
        "metric": METRIC, "value": round(value), "unit": "systems/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "LUpp sweep: 2^20 FP64 systems for each n in {8,12,16,24,32} "
                               "(n = 4 of the same sweep reported beside it), A ~ N(0,1) rejected "
                               "if cond2 > 1e4, b = A x_true, x_true ~ U(-1,1), SoA and AoS, one RHS",
                   "batch_per_n": BATCH, "n": list(STEP_SIZES), "layouts": list(layouts),
                   "soa_ldbatch": SOA_LD,
                   "mode": "strict (bitwise-reproducible, no FMA, true division)"},
        "sweep_n4_to_32": sweep_all,
        "roofline": roofline,
        "newton": newton,
        "sweep": sweep,
        "tile_local_pivoting": tiled,
        "fma_mode": fma_mode,
        "ragged": ragged,
        "serving": serving,
        "latency": lat,
        "per_kernel": per_kernel,
        "cpu_baseline": cpu,
    }
    # Release the device arrays and the library context before the result
    # line: the process then has next to nothing to tear down (about 100 GB
    # of device memory were held) once its output is complete. (A hard exit
    # right after the line would also skip the exit handlers a profiler
    # writes its results from.)
    pristine.clear()
    work.clear()
    host.clear()
    torch.cuda.synchronize()
    ctx.close()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
