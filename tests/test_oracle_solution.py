"""Solution-level pins for the oracle's rAPDB (Algorithm 2 around APDB-yx / APDB-xy).

Pinned against: hand-derived closed forms (tests/golden), the single-ball QP by 1-D multiplier
bisection, brute-force KKT enumeration (n <= 3, m <= 2), exact box-QP enumeration (m = 0), a
textbook log-barrier interior-point method, the Slater dual bound (Lemma "dual bound", §3.2),
and the optimality conditions themselves (lambda >= 0, complementary slackness, x in X).
"""
import json
import os

import numpy as np
import pytest

import qcqp_inputs as qi
from tests import pins

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _opts(orc, inst=None, **kw):
    base = dict(tau_bar=1.0, gamma0=0.1, tol=1e-10, max_iter=200000)
    if inst is not None and inst.has_q0:
        L = np.linalg.norm(np.asarray(inst.Q[0], dtype=float), 2)
        if L > 0:
            base["tau_bar"] = 1.0 / L
    base.update(kw)
    variant = base.pop("variant", "yx")
    if variant == "xy":
        return orc.Options.xy(**base)
    return orc.Options(**base)


VARIANTS = [dict(variant="yx", c_nm=1, restart="fixed"),
            dict(variant="yx", c_nm=0, restart="fixed", restart_every=800),
            dict(variant="yx", c_nm=1, restart="adaptive", ada_every=200),
            dict(variant="yx", c_nm=1, restart="none"),
            dict(variant="xy", c_nm=1, restart="fixed"),
            dict(variant="xy", c_nm=0, restart="fixed", restart_every=2000)]


@pytest.mark.parametrize("var", VARIANTS, ids=lambda v: "-".join(str(x) for x in v.values()))
def test_golden_closed_forms(orc, var):
    data = json.load(open(GOLD))
    for pb in data["problems"]:
        n, m, p = pb["n"], pb["m"], pb["p"]
        A = np.array(pb["A"], float) if p else None
        b = np.array(pb["b"], float) if p else None
        P = orc.Problem(Q=np.array(pb["Q"], float), q=np.array(pb["q"], float),
                        c=np.array(pb["c"], float), lb=np.array(pb["lb"], float),
                        ub=np.array(pb["ub"], float), A=A, b=b)
        r = orc.solve(P, _opts(orc, **var))
        assert r["info"]["status"] == "converged", (pb["name"], r["info"])
        np.testing.assert_allclose(r["x"], pb["x_star"], atol=1e-7, err_msg=pb["name"])
        assert abs(r["info"]["f"] - pb["f_star"]) <= 1e-7 * (1 + abs(pb["f_star"])), pb["name"]
        lam = r["y"][p:]
        np.testing.assert_allclose(lam, pb["lam_star"], atol=1e-6, err_msg=pb["name"])
        if p:
            np.testing.assert_allclose(r["y"][:p], pb["v_star"], atol=1e-6)


@pytest.mark.parametrize("seed", range(4))
def test_single_ball_constraint_bisection(orc, seed):
    """min 1/2x'Q0x + q0'x s.t. 1/2||x||^2 <= rho with the box inactive (sqrt(2 rho) < 10)."""
    n = 25
    rng = np.random.default_rng(100 + seed)
    M = rng.standard_normal((n, n))
    Q0 = M @ M.T / n + 0.05 * np.eye(n)
    q0 = 3.0 * rng.standard_normal(n)
    x_free = -np.linalg.solve(Q0, q0)
    rho = 0.125 * (x_free @ x_free)          # the ball cuts the unconstrained minimiser
    rho = min(rho, 40.0)
    xs, lam = pins.ball_qp_bisection(Q0, q0, rho)
    assert np.sqrt(2 * rho) < 10
    Q = np.stack([Q0, np.eye(n)])
    P = orc.Problem(Q=Q, q=np.stack([q0, np.zeros(n)]), c=np.array([0.0, -rho]),
                    lb=-10 * np.ones(n), ub=10 * np.ones(n))
    for var in VARIANTS[:3] + VARIANTS[4:5]:
        r = orc.solve(P, _opts(orc, **var))
        assert r["info"]["status"] == "converged"
        err = np.linalg.norm(r["x"] - xs) / (1 + np.linalg.norm(xs))
        assert err < 1e-7, (var, err)
        assert abs(r["y"][0] - lam) < 1e-6 * (1 + lam)


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_kkt_enumeration(orc, seed):
    rng = np.random.default_rng(200 + seed)
    n = 2 + seed % 2
    m = 1 + (seed // 2) % 2
    Q = np.empty((m + 1, n, n))
    for i in range(m + 1):
        M = rng.standard_normal((n, n))
        Q[i] = M @ M.T / n + 0.1 * np.eye(n)
    q = 2.0 * rng.standard_normal((m + 1, n))
    c = np.concatenate([[0.0], rng.uniform(-1, -0.1, m)])
    lb, ub = -np.ones(n) * 0.8, np.ones(n) * 0.8
    best = pins.kkt_enumerate(Q, q, c, lb, ub)
    assert best is not None
    xs, lams, fs = best
    P = orc.Problem(Q=Q, q=q, c=c, lb=lb, ub=ub)
    for var in (VARIANTS[0], VARIANTS[4]):
        r = orc.solve(P, _opts(orc, **var))
        assert r["info"]["status"] == "converged"
        np.testing.assert_allclose(r["x"], xs, atol=2e-7)
        assert abs(r["info"]["f"] - fs) <= 1e-8 * (1 + abs(fs))


@pytest.mark.parametrize("seed", range(3))
def test_m0_reduces_to_box_qp(orc, seed):
    """With m = 0, rAPDB-yx is projected gradient with backtracking on a box QP."""
    n = 4
    rng = np.random.default_rng(300 + seed)
    M = rng.standard_normal((n, n))
    H = M @ M.T / n + 0.2 * np.eye(n)
    h = 4.0 * rng.standard_normal(n)
    lo, hi = -np.ones(n), np.ones(n)
    D, val = pins.box_qp_enumerate(H, h, lo, hi)
    P = orc.Problem(Q=H[None], q=h[None], c=np.zeros(1), lb=lo, ub=hi)
    r = orc.solve(P, _opts(orc, restart="none"))
    assert r["info"]["status"] == "converged"
    np.testing.assert_allclose(r["x"], D, atol=1e-9)


@pytest.mark.parametrize("seed,p", [(0, 0), (1, 2)])
def test_barrier_method_objective(orc, seed, p):
    """f* from an independent log-barrier interior-point solve (stands in for a commercial one)."""
    inst = qi.random_qcqp(30, 6, seed=400 + seed, shift=0.01, p=p)
    xb, fb = pins.barrier_qcqp(inst.Q, inst.q, inst.c, inst.lb, inst.ub, inst.A, inst.b)
    P = orc.Problem(inst)
    for var in VARIANTS:
        r = orc.solve(P, _opts(orc, inst, **var))
        assert r["info"]["status"] == "converged", (var, r["info"])
        assert abs(r["info"]["f"] - fb) <= 1e-7 * (1 + abs(fb)), (var, r["info"]["f"], fb)
        assert np.linalg.norm(r["x"] - xb) / (1 + np.linalg.norm(xb)) < 1e-5


def test_optimality_conditions_and_slater_bound(orc):
    """lambda >= 0, complementary slackness, x in X; ||lambda*|| within the Slater bound
    (f(x~) - q(lambda^))/min_i(-g_i(x~)) with x~ = 0 and q(0) >= c_0 - ||ub * q_0||_1."""
    inst = qi.random_qcqp(100, 10, seed=qi.config_seed(1), shift=0.0)
    P = orc.Problem(inst)
    r = orc.solve(P, _opts(orc, inst, tol=1e-9))
    x, lam = r["x"], r["y"]
    assert np.all(lam >= 0)
    assert np.all(x >= inst.lb) and np.all(x <= inst.ub)
    g = np.array([0.5 * x @ inst.Q[i] @ x + inst.q[i] @ x + inst.c[i] for i in range(1, 11)])
    assert np.max(g) <= 1e-8
    assert np.max(np.abs(lam * g)) <= 1e-7
    f_tilde = inst.c[0]
    q_lower = inst.c[0] - np.sum(np.abs(inst.q[0]) * inst.ub)
    bound = (f_tilde - q_lower) / np.min(-inst.c[1:])
    assert np.linalg.norm(lam) <= bound


def test_restarts_reach_the_same_solution(orc):
    """Forced frequent fixed restarts (from the last iterate and from the average) and the
    adaptive test all reach the same solution."""
    inst = qi.random_qcqp(40, 5, seed=9, shift=0.01)
    P = orc.Problem(inst)
    ref = orc.solve(P, _opts(orc, inst, restart="none"))
    for kw in (dict(restart="fixed", restart_every=7),
               dict(restart="fixed", restart_every=15, restart_from_average=True),
               dict(restart="adaptive", ada_first=5, ada_every=10),
               dict(restart="adaptive", ada_first=5, ada_every=10, restart_from_average=True)):
        r = orc.solve(P, _opts(orc, inst, **kw))
        assert r["info"]["status"] == "converged", kw
        if kw["restart"] == "fixed":
            assert r["info"]["restarts"] >= 1
        np.testing.assert_allclose(r["x"], ref["x"], atol=1e-7)
