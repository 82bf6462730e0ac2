"""Pins of the CPU oracle's per-point Newton constitutive update (Section 2.1,
Algorithm 2 of the paper) against results that do not come from the oracle:

* the analytic Jacobian against central finite differences of the residual;
* the isotropic Norton law against its scalar radial-return equation solved by
  bisection (any initial elastic strain);
* the Armstrong-Frederick law from the virgin state against its own scalar
  reduction, and with C = D = 0 against the Norton law;
* the elastic limit (A = 0) and zero loading;
* objectivity under rotations (Kelvin 6x6 form);
* the stop rule: maxit exhaustion, non-finite input.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import Law
from workloads import newton_points

S2 = math.sqrt(2.0)


def lame(law):
    lam = law.E * law.nu / ((1 + law.nu) * (1 - 2 * law.nu))
    mu = law.E / (2 * (1 + law.nu))
    return lam, mu


def stiffness(law):
    lam, mu = lame(law)
    one = np.array([1, 1, 1, 0, 0, 0.0])
    return lam * np.outer(one, one) + 2 * mu * np.eye(6)


def kdev(v):
    out = v.copy()
    out[:3] -= v[:3].sum() / 3
    return out


def seq_of(v):
    return math.sqrt(1.5 * float(v @ v))


@pytest.mark.parametrize("kind", [7, 13])
def test_jacobian_matches_finite_differences(kind):
    law = Law(kind=kind)
    rng = np.random.Generator(np.random.PCG64(7 + kind))
    for trial in range(20):
        deps = rng.uniform(-2e-3, 2e-3, 6)
        st = np.zeros(kind)
        st[:6] = rng.uniform(-1e-3, 1e-3, 6)
        st[6] = rng.uniform(0, 1e-2)
        if kind == 13:
            st[7:] = kdev(rng.uniform(-1e-3, 1e-3, 6))
        y = np.zeros(kind)
        y[:6] = rng.uniform(-1e-3, 1e-3, 6)
        y[6] = rng.uniform(0, 2e-3)
        if kind == 13:
            y[7:] = rng.uniform(-1e-3, 1e-3, 6)
        F0, J, _ = oracle.law_eval(law, deps, st, y)
        Jfd = np.zeros_like(J)
        for c in range(kind):
            h = 1e-7 * max(1e-3, abs(y[c]))
            yp, ym = y.copy(), y.copy()
            yp[c] += h
            ym[c] -= h
            Fp, _, _ = oracle.law_eval(law, deps, st, yp)
            Fm, _, _ = oracle.law_eval(law, deps, st, ym)
            Jfd[:, c] = (Fp - Fm) / (2 * h)
        scale = np.abs(J).max()
        assert np.abs(J - Jfd).max() <= 1e-6 * scale, (trial, np.abs(J - Jfd).max(), scale)


def radial_return(law, deps, eel_t):
    """Isotropic Norton: s = s_tr - 2 mu dp N_tr and seq = seq_tr - 3 mu dp, so
    dp solves g(dp) = dp - dt A (seq_tr - 3 mu dp)^m = 0 on [0, seq_tr/(3 mu)],
    g increasing. Bisection to the last representable point."""
    lam, mu = lame(law)
    sig_tr = stiffness(law) @ (eel_t + deps)
    s_tr = kdev(sig_tr)
    q = seq_of(s_tr)
    if q == 0:
        return sig_tr
    lo, hi = 0.0, q / (3 * mu)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        g = mid - law.dt * law.A * (q - 3 * mu * mid) ** law.m
        if g > 0:
            hi = mid
        else:
            lo = mid
    dp = 0.5 * (lo + hi)
    N = 1.5 * s_tr / q
    return sig_tr - 2 * mu * dp * N


def test_norton_matches_radial_return():
    law = Law(kind=7)
    deps = newton_points(200, seed=11)
    rng = np.random.Generator(np.random.PCG64(12))
    st = np.zeros((200, 7))
    st[100:, :6] = rng.uniform(-5e-4, 5e-4, (100, 6))  # non-virgin elastic strain
    st[100:, 6] = rng.uniform(0, 1e-2, 100)
    out = oracle.constitutive_update(law, deps, st, tol=1e-15, maxit=60, threads=4)
    assert np.all(out["status"] == 0)
    for s in range(200):
        ref = radial_return(law, deps[s], st[s, :6])
        assert np.abs(out["sig"][s] - ref).max() <= 1e-10 * np.abs(ref).max(), s
    # benchmark stop rule on the virgin points: still within 1e-7 of the exact return
    out12 = oracle.constitutive_update(law, deps[:100], None, tol=1e-12, maxit=20, threads=4)
    ok = out12["status"] == 0
    assert ok.all()
    for s in range(100):
        ref = radial_return(law, deps[s], st[s, :6])
        assert np.abs(out12["sig"][s] - ref).max() <= 1e-7 * np.abs(ref).max()


def af_virgin_return(law, deps):
    """Armstrong-Frederick from alpha_t = 0: alpha = dp N / (1 + D dp), so
    seq = seq_tr - (3 mu + C / (1 + D dp)) dp and dp solves
    dp - dt A seq(dp)^m = 0; seq is decreasing in dp, so bisection applies."""
    lam, mu = lame(law)
    sig_tr = stiffness(law) @ deps
    s_tr = kdev(sig_tr)
    q = seq_of(s_tr)
    lo, hi = 0.0, q / (3 * mu)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        sq = q - (3 * mu + law.C / (1 + law.D * mid)) * mid
        g = mid - law.dt * law.A * max(sq, 0.0) ** law.m
        if g > 0:
            hi = mid
        else:
            lo = mid
    dp = 0.5 * (lo + hi)
    N = 1.5 * s_tr / q
    return sig_tr - 2 * mu * dp * N, dp * N / (1 + law.D * dp), dp


def test_armstrong_frederick_virgin_scalar_reduction():
    law = Law(kind=13)
    deps = newton_points(200, seed=13)
    out = oracle.constitutive_update(law, deps, None, tol=1e-15, maxit=60, threads=4)
    assert np.all(out["status"] == 0)
    for s in range(200):
        sig, alpha, dp = af_virgin_return(law, deps[s])
        assert np.abs(out["sig"][s] - sig).max() <= 1e-10 * np.abs(sig).max()
        assert abs(out["state"][s, 6] - dp) <= 1e-10 * dp
        assert np.abs(out["state"][s, 7:] - alpha).max() <= 1e-9 * np.abs(alpha).max()


def test_af_without_hardening_reduces_to_norton():
    deps = newton_points(300, seed=14)
    o7 = oracle.constitutive_update(Law(kind=7), deps, tol=1e-14, maxit=40, threads=4)
    o13 = oracle.constitutive_update(Law(kind=13, C=0.0, D=0.0), deps, tol=1e-14, maxit=40,
                                     threads=4)
    assert np.all(o7["status"] == 0) and np.all(o13["status"] == 0)
    rel = np.abs(o7["sig"] - o13["sig"]).max(axis=1) / np.abs(o7["sig"]).max(axis=1)
    assert rel.max() <= 1e-10


def test_elastic_limit_and_zero_loading():
    law = Law(kind=7, A=0.0)
    deps = newton_points(50, seed=15)
    out = oracle.constitutive_update(law, deps, threads=1)
    assert np.all(out["status"] == 0) and np.all(out["iters"] == 1)
    ref = deps @ stiffness(law).T
    assert np.abs(out["sig"] - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.allclose(out["state"][:, :6], deps, rtol=0, atol=1e-18)
    assert np.all(out["state"][:, 6] == 0)
    for kind in (7, 13):
        z = oracle.constitutive_update(Law(kind=kind), np.zeros((5, 6)), threads=1)
        assert np.all(z["iters"] == 0) and np.all(z["status"] == 0)
        assert np.all(z["sig"] == 0) and np.all(z["state"] == 0)


def kelvin_rotation(Q):
    """6x6 matrix R with kelvin(Q e Q^T) = R kelvin(e)."""
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    w = [1, 1, 1, S2, S2, S2]
    R = np.zeros((6, 6))
    for b, (k, l) in enumerate(pairs):
        E = np.zeros((3, 3))
        E[k, l] = E[l, k] = 1.0 / w[b]
        QE = Q @ E @ Q.T
        for a, (i, j) in enumerate(pairs):
            R[a, b] = QE[i, j] * w[a]
    return R


@pytest.mark.parametrize("kind", [7, 13])
def test_objectivity(kind):
    rng = np.random.Generator(np.random.PCG64(16 + kind))
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    R = kelvin_rotation(Q)
    assert np.allclose(R @ R.T, np.eye(6), atol=1e-14)
    deps = newton_points(100, seed=17)
    law = Law(kind=kind)
    o1 = oracle.constitutive_update(law, deps, tol=1e-15, maxit=60, threads=4)
    o2 = oracle.constitutive_update(law, deps @ R.T, tol=1e-15, maxit=60, threads=4)
    assert np.all(o1["status"] == 0) and np.all(o2["status"] == 0)
    rot = o1["sig"] @ R.T
    rel = np.abs(rot - o2["sig"]).max(axis=1) / np.abs(rot).max(axis=1)
    assert rel.max() <= 1e-10


def test_stop_rule_counts_linear_solves():
    """maxit is the number of linear solves (the residual is tested at
    x_0 .. x_maxit). With A = 0 the law is linear and elastic: the first
    Newton step solves it exactly (J = [[I, N], [0, 1]], F(x_1) = 0 in
    floating point), so maxit = 1 converges in one solve while maxit = 0
    stops before any solve."""
    deps = newton_points(50, seed=19)
    law = Law(kind=7, A=0.0)
    one = oracle.constitutive_update(law, deps, maxit=1, threads=2)
    assert np.all(one["status"] == 0) and np.all(one["iters"] == 1)
    assert np.all(one["resid"] == 0.0)
    assert np.array_equal(one["state"][:, :6], deps) and np.all(one["state"][:, 6] == 0)
    zero = oracle.constitutive_update(law, deps, maxit=0, threads=2)
    assert np.all(zero["status"] == 1) and np.all(zero["iters"] == 0)
    assert np.all(zero["state"] == 0)
    # a point that stops on the cap has made exactly maxit solves, and a
    # point that converges under a cap converges identically without it
    deps = newton_points(400, seed=20)
    for kind in (7, 13):
        free = oracle.constitutive_update(Law(kind=kind), deps, maxit=60, threads=4)
        assert np.all(free["status"] == 0)
        for maxit in (1, 2, 5, 12):
            cap = oracle.constitutive_update(Law(kind=kind), deps, maxit=maxit, threads=4)
            hit = cap["status"] == 1
            assert hit.any()
            assert np.all(cap["iters"][hit] == maxit)
            assert np.all(free["iters"][hit] > maxit)
            conv = cap["status"] == 0
            assert np.all(cap["iters"][conv] <= maxit)
            assert np.array_equal(cap["iters"][conv], free["iters"][conv])
            assert np.array_equal(cap["sig"][conv], free["sig"][conv])
            assert np.all(cap["state"][hit] == 0)  # not committed


def test_stop_rule_maxit_and_nonfinite():
    deps = newton_points(200, seed=18)
    out = oracle.constitutive_update(Law(kind=7), deps, maxit=1, threads=2)
    assert np.all(out["iters"] <= 1)
    assert (out["status"] == 1).mean() > 0.9
    st0 = np.zeros((200, 7))
    assert np.array_equal(out["state"][out["status"] == 1], st0[out["status"] == 1])
    bad = deps[:3].copy()
    bad[0, 0] = np.nan
    bad[1, 3] = np.inf
    o = oracle.constitutive_update(Law(kind=13), bad, threads=1)
    assert list(o["status"][:2]) == [3, 3] and o["status"][2] == 0
    assert np.all(o["state"][:2] == 0)


@pytest.mark.parametrize("kind", [7, 13])
def test_iteration_statistics_reported(kind):
    """Not a pin: records the iteration counts of the benchmark workload. The
    paper's application needs about two iterations per point on a real, much
    milder load step; this synthetic step is stiffer."""
    deps = newton_points(4000, seed=4)
    out = oracle.constitutive_update(Law(kind=kind), deps, threads=8)
    assert (out["status"] == 0).mean() > 0.99
    assert 5 < out["iters"].mean() < 20


# --------------------------------------------------------------------------
# Consistent tangent operator dsig/d(deps) at convergence (Section 2.5;
# Section 4.3: one multi-right-hand-side solve after convergence).
# --------------------------------------------------------------------------

def test_tangent_elastic_limit_is_the_stiffness():
    law = Law(kind=7, A=0.0)
    deps = newton_points(20, seed=31)
    out = oracle.constitutive_update(law, deps, threads=1, tangent=True)
    D = stiffness(law)
    assert np.all(out["status"] == 0)
    assert np.abs(out["tangent"] - D).max() <= 1e-12 * np.abs(D).max()


def prior_state(kind, count, seed):
    """A non-virgin state: elastic strain and (AF) a back-strain alpha."""
    rng = np.random.Generator(np.random.PCG64(seed))
    st = np.zeros((count, kind))
    st[:, :6] = rng.uniform(-1e-3, 1e-3, (count, 6))
    if kind == 13:
        st[:, 7:] = rng.uniform(-5e-3, 5e-3, (count, 6))
    return st


@pytest.mark.parametrize("virgin", [True, False])
@pytest.mark.parametrize("kind", [7, 13])
def test_tangent_matches_finite_differences_of_the_update(kind, virgin):
    """Central differences of the converged stress over the strain increment
    (each perturbed update converged to 1e-15) against the tangent. With a
    back-strain the AF tangent is not symmetric, so a transposed tangent
    fails here."""
    law = Law(kind=kind)
    deps = newton_points(12, seed=32 + kind)
    st0 = None if virgin else prior_state(kind, 12, 35 + kind)
    base = oracle.constitutive_update(law, deps, st0, tol=1e-15, maxit=80, threads=4,
                                      tangent=True)
    ok = base["status"] == 0  # (a few AF points do not converge from a loaded state)
    assert ok.sum() >= 8
    assert np.all(base["state"][ok, 6] > (0 if virgin else st0[ok, 6]))  # plastic flow
    h = 1e-8
    fd = np.zeros((12, 6, 6))
    for c in range(6):
        dp, dm = deps.copy(), deps.copy()
        dp[:, c] += h
        dm[:, c] -= h
        sp = oracle.constitutive_update(law, dp, st0, tol=1e-15, maxit=80, threads=4)
        sm = oracle.constitutive_update(law, dm, st0, tol=1e-15, maxit=80, threads=4)
        assert np.all(sp["status"][ok] == 0) and np.all(sm["status"][ok] == 0)
        fd[:, :, c] = (sp["sig"] - sm["sig"]) / (2 * h)
    T, fd = base["tangent"][ok], fd[ok]
    scale = np.abs(T).max(axis=(1, 2))
    err = np.abs(T - fd).max(axis=(1, 2)) / scale
    assert err.max() <= 1e-5, err
    # viscoplastic flow makes the tangent softer than the elastic stiffness
    D = stiffness(law)
    assert np.all(np.abs(T - D).max(axis=(1, 2)) > 1e-3 * np.abs(D).max())


@pytest.mark.parametrize("kind", [7, 13])
def test_tangent_objectivity(kind):
    """Virgin state, isotropic law: T(R deps) = R T(deps) R^T."""
    rng = np.random.Generator(np.random.PCG64(40 + kind))
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    R = kelvin_rotation(Q)
    deps = newton_points(50, seed=41)
    law = Law(kind=kind)
    o1 = oracle.constitutive_update(law, deps, tol=1e-15, maxit=80, threads=4, tangent=True)
    o2 = oracle.constitutive_update(law, deps @ R.T, tol=1e-15, maxit=80, threads=4, tangent=True)
    assert np.all(o1["status"] == 0) and np.all(o2["status"] == 0)
    rot = R @ o1["tangent"] @ R.T
    rel = np.abs(rot - o2["tangent"]).max(axis=(1, 2)) / np.abs(rot).max(axis=(1, 2))
    assert rel.max() <= 1e-9


def test_tangent_only_for_converged_points():
    deps = newton_points(400, seed=42)
    out = oracle.constitutive_update(Law(kind=7), deps, maxit=16, threads=2, tangent=True)
    bad = out["status"] != 0
    assert bad.any() and (~bad).any()
    assert np.all(np.isnan(out["tangent"][bad]))
    assert np.all(np.isfinite(out["tangent"][~bad]))


def test_norton_tangent_is_symmetric():
    """Associative J2 viscoplasticity integrated by backward Euler has a
    symmetric consistent tangent (Kelvin notation), in any state."""
    law = Law(kind=7)
    deps = newton_points(40, seed=43)
    o = oracle.constitutive_update(law, deps, prior_state(7, 40, 44), tol=1e-14, maxit=80,
                                   threads=4, tangent=True)
    T = o["tangent"][o["status"] == 0]
    assert len(T) > 30
    asym = np.abs(T - T.transpose(0, 2, 1)).max(axis=(1, 2)) / np.abs(T).max(axis=(1, 2))
    assert asym.max() <= 1e-12
