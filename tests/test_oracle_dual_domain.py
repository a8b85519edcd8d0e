"""Pins for the oracle's dual domains and objective shift.

Covers the restricted dual domain Y-hat = Y ∩ B of problem (R-min-max) (§3.2: the ball of
eq. (defcalB) and the separable balls of the Remark after it), lambda on the unit simplex (the
kernel-learning min-max form of §5) and the identity part rho I of the objective's Hessian.
Pinned against:
  * the variational inequality that characterises a Euclidean projection, checked on many points
    of the set including its extreme points, and an independent bisection for the simplex
    threshold;
  * closed-form saddle points of restricted problems: with lambda capped at B < lambda*, the
    single-ball QP's saddle point is x = -(Q_0 + B I)^{-1} q_0 with lambda = B; with |v| capped at
    B_v < |v*|, the equality-constrained QP's is x = -Q_0^{-1}(q_0 + v a) with v = sign(v*) B_v;
  * a ball that never binds leaves the trajectory bitwise unchanged;
  * the simplex min-max problem min_x f(x) + max_i g_i(x) against the textbook log-barrier
    method on its epigraph form;
  * rho I against the same identity stored densely in Q_0.
"""
import numpy as np
import pytest

import qcqp_inputs as qi
from tests import pins


def _spd(rng, n, shift=0.5):
    A = rng.standard_normal((n, n))
    return A @ A.T / n + shift * np.eye(n)


def _problem(orc, Q, q, c, lb, ub, A=None, b=None, **kw):
    return orc.Problem(Q=Q, q=q, c=c, lb=lb, ub=ub, A=A, b=b, **kw)


def _simplex_bisection(z):
    """Threshold theta with sum max(z - theta, 0) = 1, by bisection (independent of sorting)."""
    lo, hi = np.min(z) - 1.0, np.max(z)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.sum(np.maximum(z - mid, 0.0)) > 1.0:
            lo = mid
        else:
            hi = mid
    return np.maximum(z - 0.5 * (lo + hi), 0.0)


def _members(rng, kind, p, m, B=0.0, Bv=0.0, Bl=0.0, count=400):
    """Points of Y-hat (random, plus extreme points where the set has them)."""
    pts = []
    for _ in range(count):
        v = rng.standard_normal(p) * rng.uniform(0, 3)
        if kind == "simplex":
            lam = rng.dirichlet(np.full(m, rng.uniform(0.2, 2.0)))
        else:
            lam = np.abs(rng.standard_normal(m)) * rng.uniform(0, 3)
            lam[rng.random(m) < 0.3] = 0.0
        if Bv > 0 and np.linalg.norm(v) > 0:
            v *= rng.uniform(0, 1) * Bv / np.linalg.norm(v)
        if Bl > 0 and np.linalg.norm(lam) > 0:
            lam *= rng.uniform(0, 1) * Bl / np.linalg.norm(lam)
        y = np.concatenate([v, lam])
        if B > 0 and np.linalg.norm(y) > 0:
            y *= rng.uniform(0, 1) * B / np.linalg.norm(y)
        pts.append(y)
    if kind == "simplex":
        for i in range(m):
            e = np.zeros(p + m)
            e[p + i] = 1.0
            pts.append(e)
    return pts


CASES = [
    dict(kind="nonneg"),
    dict(kind="nonneg", ball=1.5),
    dict(kind="nonneg", ball_v=0.7, ball_l=1.2),
    dict(kind="nonneg", ball_l=0.4),
    dict(kind="simplex"),
    dict(kind="simplex", ball_v=0.5),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_projection_variational_inequality(orc, case):
    rng = np.random.default_rng(11)
    p, m, n = 2, 5, 3
    kw = {k: v for k, v in case.items() if k != "kind"}
    P = _problem(orc, np.zeros((m + 1, n, n)), np.zeros((m + 1, n)), np.zeros(m + 1),
                 -np.ones(n), np.ones(n), A=np.ones((p, n)), b=np.zeros(p),
                 lambda_set=case["kind"], **kw)
    members = _members(rng, case["kind"], p, m, B=kw.get("ball", 0.0), Bv=kw.get("ball_v", 0.0),
                       Bl=kw.get("ball_l", 0.0))
    for trial in range(60):
        z = rng.standard_normal(p + m) * rng.choice([0.1, 1.0, 10.0])
        w = orc.project_dual(P, z)
        lam = w[p:]
        assert np.all(lam >= 0.0)
        if case["kind"] == "simplex":
            assert abs(lam.sum() - 1.0) <= 1e-14
        if "ball" in kw:
            assert np.linalg.norm(w) <= kw["ball"] * (1 + 1e-15)
        if "ball_v" in kw:
            assert np.linalg.norm(w[:p]) <= kw["ball_v"] * (1 + 1e-15)
        if "ball_l" in kw:
            assert np.linalg.norm(lam) <= kw["ball_l"] * (1 + 1e-15)
        if "ball" not in kw and "ball_v" not in kw:
            np.testing.assert_array_equal(w[:p], z[:p])       # v is free
        # <z - w, u - w> <= 0 for every u in the set
        worst = max(float((z - w) @ (u - w)) for u in members)
        assert worst <= 1e-12 * (1 + np.linalg.norm(z)) ** 2, (trial, worst)
        if case["kind"] == "simplex" and "ball_v" not in kw:
            np.testing.assert_allclose(lam, _simplex_bisection(z[p:]), atol=1e-13)
        # a projection is idempotent
        np.testing.assert_allclose(orc.project_dual(P, w), w, atol=1e-15)


def _ball_constrained(rng, n):
    """min 1/2 x'Q0 x + q0'x  s.t. 1/2||x||^2 <= rho with the unconstrained minimiser outside."""
    Q0 = _spd(rng, n)
    q0 = rng.standard_normal(n) * 3.0
    rho = 0.5
    Q = np.stack([Q0, np.eye(n)])
    q = np.stack([q0, np.zeros(n)])
    c = np.array([0.0, -rho])
    return Q0, q0, rho, Q, q, c


def test_small_ball_caps_the_multiplier(orc):
    rng = np.random.default_rng(21)
    n = 6
    Q0, q0, rho, Q, q, c = _ball_constrained(rng, n)
    x_star, lam_star = pins.ball_qp_bisection(Q0, q0, rho)
    assert lam_star > 0.5
    B = 0.5 * lam_star
    xB = -np.linalg.solve(Q0 + B * np.eye(n), q0)
    assert 0.5 * xB @ xB - rho > 0                     # the cap binds: lambda = B
    lb, ub = -10 * np.ones(n), 10 * np.ones(n)
    for kw in (dict(ball=B), dict(ball_l=B)):
        P = _problem(orc, Q, q, c, lb, ub, **kw)
        r = orc.solve(P, orc.Options(tau_bar=1.0 / np.linalg.norm(Q0, 2), tol=0.0,
                                     max_iter=6000, restart_every=400))
        np.testing.assert_allclose(r["x"], xB, atol=1e-8)
        assert abs(r["y"][0] - B) <= 1e-9
        g = orc.gap(P, r["x"], r["y"])
        assert abs(g["G"]) <= 1e-12
        # the unrestricted problem's KKT residual stays away from zero
        assert orc.kkt(P, r["x"], r["y"])["rel_kkt"] > 1e-3


def test_small_v_ball_caps_the_equality_multiplier(orc):
    rng = np.random.default_rng(22)
    n = 5
    Q0 = _spd(rng, n)
    q0 = rng.standard_normal(n)
    a = rng.standard_normal(n)
    beta = 2.0
    Qi = np.linalg.inv(Q0)
    v_star = -(beta + a @ Qi @ q0) / (a @ Qi @ a)
    Bv = 0.5 * abs(v_star)
    v = np.sign(v_star) * Bv
    xB = -Qi @ (q0 + v * a)
    P = _problem(orc, Q0[None], q0[None], np.zeros(1), -10 * np.ones(n), 10 * np.ones(n),
                 A=a[None], b=np.array([beta]), ball_v=Bv)
    assert np.all(np.abs(xB) < 10)
    r = orc.solve(P, orc.Options(tau_bar=1.0 / np.linalg.norm(Q0, 2), tol=0.0, max_iter=6000))
    np.testing.assert_allclose(r["x"], xB, atol=1e-8)
    assert abs(r["y"][0] - v) <= 1e-9


@pytest.mark.parametrize("variant", ["yx", "xy"])
def test_ball_that_never_binds_leaves_the_trajectory_unchanged(orc, variant):
    inst = qi.random_qcqp(40, 4, seed=5, shift=0.01, p=1)
    L = np.linalg.norm(inst.Q[0], 2)
    o = (orc.Options.xy if variant == "xy" else orc.Options)(tau_bar=1.0 / L, tol=0.0, max_iter=60)
    base = orc.solve(orc.Problem(inst), o)
    for kw in (dict(ball=1e6), dict(ball_v=1e6, ball_l=1e6)):
        r = orc.solve(orc.Problem(inst, **kw), o)
        np.testing.assert_array_equal(r["x"], base["x"])
        np.testing.assert_array_equal(r["y"], base["y"])
        assert r["info"]["trials"] == base["info"]["trials"]


def test_large_ball_gives_the_unrestricted_solution(orc):
    inst = qi.random_qcqp(30, 3, seed=8, shift=0.01)
    L = np.linalg.norm(inst.Q[0], 2)
    o = orc.Options(tau_bar=1.0 / L, tol=1e-9, max_iter=100000)
    ref = orc.solve(orc.Problem(inst), o)
    assert ref["info"]["status"] == "converged"
    B = 1.5 * np.linalg.norm(ref["y"]) + 0.1
    r = orc.solve(orc.Problem(inst, ball=B), o)
    assert r["info"]["status"] == "converged"
    np.testing.assert_allclose(r["x"], ref["x"], atol=1e-6)
    assert abs(r["info"]["f"] - ref["info"]["f"]) <= 1e-8 * (1 + abs(ref["info"]["f"]))


def _simplex_instance(rng, n, m):
    Q = np.stack([_spd(rng, n, 0.2) for _ in range(m + 1)])
    q = rng.standard_normal((m + 1, n))
    c = rng.uniform(-1, 1, m + 1)
    c[0] = 0.0
    return Q, q, c


@pytest.mark.parametrize("variant", ["yx", "xy"])
def test_simplex_min_max_against_barrier_epigraph(orc, variant):
    """min_x max_{lambda in simplex} f(x) + sum lambda_i g_i(x) = min_{x,t} f(x) + t s.t.
    g_i(x) <= t: the epigraph QCQP in n + 1 variables, solved by the log-barrier method."""
    rng = np.random.default_rng(31)
    n, m = 3, 3
    Q, q, c = _simplex_instance(rng, n, m)
    lb, ub = -4 * np.ones(n), 4 * np.ones(n)
    P = _problem(orc, Q, q, c, lb, ub, lambda_set="simplex")
    o = (orc.Options.xy if variant == "xy" else orc.Options)(
        tau_bar=1.0 / np.linalg.norm(Q[0], 2), tol=1e-10, max_iter=200000)
    r = orc.solve(P, o)
    assert r["info"]["status"] == "converged", r["info"]
    lam = r["y"]
    assert np.all(lam >= 0) and abs(lam.sum() - 1) <= 1e-12
    # epigraph form for the barrier method: variables (x, t), t in [-T, T]
    T = 1e3
    Qe = np.zeros((m + 1, n + 1, n + 1))
    qe = np.zeros((m + 1, n + 1))
    for i in range(m + 1):
        Qe[i, :n, :n] = Q[i]
        qe[i, :n] = q[i]
    qe[0, n] = 1.0
    qe[1:, n] = -1.0
    x0 = np.zeros(n + 1)
    x0[n] = max(c[1:]) + 1.0
    xe, _ = pins.barrier_qcqp(Qe, qe, c, np.append(lb, -T), np.append(ub, T), x0=x0)
    np.testing.assert_allclose(r["x"], xe[:n], atol=2e-6)

    def val(x):
        g = [0.5 * x @ Q[i] @ x + q[i] @ x + c[i] for i in range(1, m + 1)]
        return 0.5 * x @ Q[0] @ x + q[0] @ x + max(g)
    assert abs(val(r["x"]) - val(xe[:n])) <= 1e-9 * (1 + abs(val(xe[:n])))
    # lambda is supported on the maximising pieces
    g = np.array([0.5 * r["x"] @ Q[i] @ r["x"] + q[i] @ r["x"] + c[i] for i in range(1, m + 1)])
    assert np.all(lam[g < g.max() - 1e-4] <= 1e-8)


def test_simplex_kkt_is_the_natural_residual(orc):
    rng = np.random.default_rng(41)
    n, m = 4, 3
    Q, q, c = _simplex_instance(rng, n, m)
    P = _problem(orc, Q, q, c, -np.ones(n), np.ones(n), lambda_set="simplex")
    x = rng.uniform(-1, 1, n)
    lam = rng.dirichlet(np.ones(m))
    kk = orc.kkt(P, x, lam)
    g = np.array([0.5 * x @ Q[i] @ x + q[i] @ x + c[i] for i in range(1, m + 1)])
    r = lam - _simplex_bisection(lam + g)
    assert abs(kk["rel_comp"] - np.linalg.norm(r) / (1 + np.linalg.norm(c[1:]))) <= 1e-12
    assert kk["rel_pri"] == 0.0 and kk["max_violation"] == 0.0


def test_q0_shift_equals_identity_stored_in_q0(orc):
    rng = np.random.default_rng(51)
    n, m, rho = 20, 3, 2.0
    Q, q, c = _simplex_instance(rng, n, m)
    lb, ub = np.zeros(n), np.full(n, np.inf)
    Pd = _problem(orc, Q + rho * np.eye(n)[None] * (np.arange(m + 1) == 0)[:, None, None],
                  q, c, lb, ub, lambda_set="simplex")
    Ps = _problem(orc, Q, q, c, lb, ub, lambda_set="simplex", q0_shift=rho)
    Qz = Q.copy()
    Qz[0] = 0.0
    Pz = _problem(orc, Qz[1:], q, c, lb, ub, has_q0=False, lambda_set="simplex",
                  q0_shift=rho)
    Pzd = _problem(orc, np.concatenate([rho * np.eye(n)[None], Qz[1:]]), q, c, lb, ub,
                   lambda_set="simplex")
    x = rng.uniform(0, 1, n)
    y = rng.dirichlet(np.ones(m))
    for a, b in ((Pd, Ps), (Pzd, Pz)):
        oa, ob = orc.operator(a, x, y), orc.operator(b, x, y)
        for k in ("U", "G", "grad"):
            np.testing.assert_allclose(ob[k], oa[k], rtol=1e-13, atol=1e-13)
        assert abs(ob["f"] - oa["f"]) <= 1e-13 * (1 + abs(oa["f"]))
        ga, gb = orc.gap(a, x, y), orc.gap(b, x, y)
        assert abs(ga["G"] - gb["G"]) <= 1e-10 * (1 + abs(ga["G"]))
    o = orc.Options(tau_bar=0.1, mu=rho, tol=1e-9, max_iter=100000)
    ra, rb = orc.solve(Pzd, o), orc.solve(Pz, o)
    assert rb["info"]["status"] == "converged"
    np.testing.assert_allclose(rb["x"], ra["x"], atol=1e-7)


def test_dual_domain_validation(orc):
    n = 3
    Q = np.stack([np.eye(n), np.eye(n)])
    q = np.zeros((2, n))
    c = np.array([0.0, -1.0])
    lb, ub = -np.ones(n), np.ones(n)
    o = orc.Options(tau_bar=1.0)
    for kw in (dict(ball=1.0, ball_v=1.0), dict(lambda_set="simplex", ball=1.0),
               dict(lambda_set="simplex", ball_l=1.0), dict(q0_shift=-1.0), dict(ball=-1.0)):
        r = orc.solve(_problem(orc, Q, q, c, lb, ub, **kw), o)
        assert r["info"]["status"] == "invalid", kw
    bad_lb = lb.copy()
    bad_lb[0] = np.inf
    assert orc.solve(_problem(orc, Q, q, c, bad_lb, np.full(n, np.inf)), o)["info"]["status"] == "invalid"

