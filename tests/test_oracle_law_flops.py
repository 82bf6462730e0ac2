"""The instrumented operation count of the oracle's law evaluation
(oracle/law_flops.py), pinned against a count by hand of the residual of
Section 2.1 as the oracle writes it, and checked for internal consistency."""
import shutil

import pytest

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def counts():
    from oracle.law_flops import counts as c
    return c()


def test_norton_residual_by_hand(counts):
    """Residual of the 7-unknown law, operation by operation:
    eel = eel_t + y (6 add), tr (2 add), sig = 2 mu eel + lam tr on the
    normal components (12 mul + 3 mul + 6 add), tr(sig) (2 add), deviator
    s = sig - tr/3 (6 sub + 3 div), xi = s - 0 (6 sub: the oracle subtracts
    the backstress term, zero without hardening), xi.xi (6 mul + 6 add),
    seq = sqrt(1.5 xi.xi) (1 mul + 1 sqrt), N = 1.5 xi / seq (6 mul + 6 div),
    F_e = y + dp N - deps (6 mul + 12 add), F_p = dp - (dt A) seq^m (1 mul,
    1 pow, 1 sub)."""
    c = counts["7_residual"]
    assert (c["add"], c["mul"], c["div"], c["sqrt"], c["pow"]) == (47, 35, 9, 1, 1)


def test_hardening_adds_the_backstress_terms(counts):
    """13 unknowns: alpha = alpha_t + d_alpha (6 add), X = (2/3 C) alpha
    (6 mul), and F_a = d_alpha - dp N + D dp alpha (6 x: 3 mul, 2 add)."""
    r7, r13 = counts["7_residual"], counts["13_residual"]
    assert r13["add"] - r7["add"] == 6 + 12
    assert r13["mul"] - r7["mul"] == 6 + 18
    assert (r13["div"], r13["sqrt"], r13["pow"]) == (r7["div"], r7["sqrt"], r7["pow"])


def test_jacobian_costs_more_than_the_residual(counts):
    for k in (7, 13):
        r, j = counts[f"{k}_residual"], counts[f"{k}_residual_jacobian"]
        assert j["flops"] > r["flops"]
        assert j["pow"] == r["pow"] + 1  # d(seq^m)/dseq
        assert j["flops"] == j["add"] + j["mul"] + j["div"] + j["sqrt"] + j["pow"]


def test_benchmark_uses_these_counts(counts):
    import importlib.util
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_consts", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    assert bench.LAW_FLOPS == {k: counts[f"{k}_residual_jacobian"]["flops"] for k in (7, 13)}
