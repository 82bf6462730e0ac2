"""Writes the stored expected values under tests/golden/ using only the oracle
and the seeded generators (no HIP code).

    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import Law  # noqa: E402
from workloads import newton_points, systems  # noqa: E402


def main():
    # 4096 systems, n = 8, A ~ N(0,1) without a condition filter, seed 1: the
    # first 16 systems' pivots, info and solution (hex-exact doubles).
    A, b, _ = systems(8, 4096, seed=1)
    out = oracle.gesv_batch(A[:16], b[:16], threads=1)
    with open(os.path.join(HERE, "lupp_n8_seed1_first16.txt"), "w") as f:
        f.write("# system info ipiv[8] x[8] (float.hex)\n")
        for s in range(16):
            f.write(" ".join([str(s), str(int(out["info"][s]))]
                             + [str(int(v)) for v in out["ipiv"][s]]
                             + [float(v).hex() for v in out["x"][s]]) + "\n")
    # Newton update of the first 16 points of the 2^20-point workload (seed 4).
    deps = newton_points(16, seed=4)
    with open(os.path.join(HERE, "newton_seed4_first16.txt"), "w") as f:
        f.write("# law point status iters sig[6] (float.hex)\n")
        for kind in (7, 13):
            o = oracle.constitutive_update(Law(kind=kind), deps, threads=1)
            for s in range(16):
                f.write(" ".join([str(kind), str(s), str(int(o["status"][s])),
                                  str(int(o["iters"][s]))]
                                 + [float(v).hex() for v in o["sig"][s]]) + "\n")


if __name__ == "__main__":
    main()
