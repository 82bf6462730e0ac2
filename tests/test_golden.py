"""The oracle still reproduces its stored outputs (tests/golden/, written by
tests/golden/make_golden.py). A change of the oracle's arithmetic must come
with a regenerated fixture and a reason tied to the paper."""
import os

import numpy as np

import oracle
from oracle import Law
from workloads import newton_points, systems

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_lupp_fixture():
    A, b, _ = systems(8, 4096, seed=1)
    out = oracle.gesv_batch(A[:16], b[:16], threads=1)
    rows = [l.split() for l in open(os.path.join(HERE, "lupp_n8_seed1_first16.txt"))
            if not l.startswith("#")]
    for r in rows:
        s = int(r[0])
        assert int(r[1]) == out["info"][s]
        assert [int(v) for v in r[2:10]] == list(out["ipiv"][s])
        assert [float.fromhex(v) for v in r[10:18]] == list(out["x"][s])


def test_newton_fixture():
    deps = newton_points(16, seed=4)
    rows = [l.split() for l in open(os.path.join(HERE, "newton_seed4_first16.txt"))
            if not l.startswith("#")]
    outs = {k: oracle.constitutive_update(Law(kind=k), deps, threads=1) for k in (7, 13)}
    for r in rows:
        o, s = outs[int(r[0])], int(r[1])
        assert int(r[2]) == o["status"][s] and int(r[3]) == o["iters"][s]
        assert [float.fromhex(v) for v in r[4:10]] == list(o["sig"][s])
