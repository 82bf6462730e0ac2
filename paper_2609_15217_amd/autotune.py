"""Measure the fastest kernel variant for every size n = 1..32, both layouts
and both batch-size classes on this GPU, and the fastest lane count of every
size in the ragged (mixed-size) path, and write dispatch_gfx950.json
(compiled into liblupp as its default tables by the build).

    python -m paper_2609_15217_amd.autotune [--out PATH] [--reps 5] [--what all|solve|ragged]

Each standalone entry is chosen by lupp_autotune (a C-ABI call that times
every compiled variant and workgroup size on a device copy of the batch and
keeps the median-fastest); each ragged entry by lupp_autotune_ragged (the
ragged path, one launch per size class, timed on a batch of one size large enough that the
solve, not the grouping kernels, dominates: 2^20 systems up to n = 16, 2^19
above). With --what, the part not measured is kept from the existing file.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

SMALL, LARGE = 4096, 1 << 20
RAGGED_BATCH = {"small": 1 << 20, "large": 1 << 19}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "dispatch_gfx950.json"))
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--sizes", default="1-32")
    ap.add_argument("--what", choices=("all", "solve", "ragged"), default="all")
    args = ap.parse_args()
    lo, hi = (int(v) for v in args.sizes.split("-"))

    import torch

    import paper_2609_15217_amd.lupp as L
    from workloads import device_systems

    ctx = L.Context(0)
    old = json.load(open(args.out)) if os.path.exists(args.out) else {}
    entries = [] if args.what != "ragged" else old.get("entries", [])
    ragged = [] if args.what != "solve" else old.get("ragged", [])
    t0 = time.time()
    for n in range(lo, hi + 1) if args.what != "ragged" else ():
        for bucket, batch in ((0, SMALL), (1, LARGE if n <= 16 else LARGE // 2)):
            A, b = device_systems(n, batch, seed=9000 + n)
            for lay in ("aos", "soa"):
                if lay == "soa":
                    Al, bl = A.permute(1, 2, 0).contiguous(), b.t().contiguous()
                    layout, sA, sB = L.LUPP_SOA, batch, batch
                else:
                    Al, bl = A, b
                    layout, sA, sB = L.LUPP_AOS, n * n, n
                rc, v, lanes, wpb, ms = L.lupp_autotune(ctx, n, batch, layout, Al, n, sA, bl, sB,
                                                        args.reps)
                if rc != 0:
                    raise RuntimeError(f"autotune n={n} {lay}: {L.lupp_error_string(rc)}")
                entries.append({"n": n, "layout": lay, "bucket": bucket, "batch": batch,
                                "variant": "thread" if v == L.LUPP_VARIANT_THREAD else "lanes",
                                "lanes": lanes, "wpb": wpb, "ms": round(ms, 4),
                                "systems_per_s": round(batch / (ms * 1e-3))})
                print(f"[autotune] n={n:2d} {lay} batch={batch:8d}: "
                      f"{entries[-1]['variant']}{lanes if v == 2 else ''} wpb={wpb} {ms:.3f} ms",
                      flush=True)
                del Al, bl
            del A, b
            torch.cuda.empty_cache()
    for n in range(lo, hi + 1) if args.what != "solve" else ():
        batch = RAGGED_BATCH["small" if n <= 16 else "large"]
        A, b = device_systems(n, batch, seed=9100 + n)
        rc, lanes, ms = L.lupp_autotune_ragged(ctx, n, batch, A, b, args.reps)
        if rc != 0:
            raise RuntimeError(f"ragged autotune n={n}: {L.lupp_error_string(rc)}")
        ragged.append({"n": n, "batch": batch, "lanes": lanes, "ms": round(ms, 4)})
        print(f"[autotune] ragged n={n:2d} batch={batch}: lanes {lanes} {ms:.3f} ms", flush=True)
        del A, b
        torch.cuda.empty_cache()
    out = {"arch": "gfx950", "small_batch": SMALL, "large_batch": LARGE,
           "ragged_batch": RAGGED_BATCH,
           "reps": args.reps if args.what != "ragged" else old.get("reps", args.reps),
           "ragged_reps": args.reps if args.what != "solve" else old.get("ragged_reps"),
           "seconds": round(time.time() - t0, 1), "entries": entries, "ragged": ragged}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"[autotune] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
