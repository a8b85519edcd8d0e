"""Pins for the oracle's step-size logic, smoothed duality gap and KKT residual.

Step sizes: the lemmas of §3.1/§3.2 (monotone and non-monotone settings) fix exact identities
and bounds that any correct implementation satisfies:
  * mu = 0  =>  gamma_k = gamma_0, so sigma_k / tau_k = gamma_0;
  * monotone (c_nm = 0, mu = 0): tau_k non-increasing, tau_k <= tau_bar, and the number of test
    evaluations over K iterations is exactly K + log_{1/eta}(tau_bar / tau_{K-1});
  * non-monotone: tau_{k+1}/tau_k <= phi = (1 + sqrt 5)/2 and the count obeys
    K + log_{1/eta}(tau_bar/tau_{K-1}) + 1/2 sum log_{1/eta}(1 + tau_k/tau_{k-1});
  * mu > 0: gamma_{k+1} = gamma_k (1 + mu tau_k);
  * each accepted trial satisfied the test E_k <= rhs.
Smoothed gap (Definition in §4, Remark in §4.2): G >= 0 on the domain, G ~ 0 at a saddle point,
and the x-/y-parts agree with brute force (face enumeration of the box QP, scipy on y).
"""
import dataclasses

import numpy as np
import pytest

import qcqp_inputs as qi
from tests import pins

PHI = (1 + 5 ** 0.5) / 2


def _inst():
    return qi.random_qcqp(60, 8, seed=21, shift=0.01)


def _run(orc, P, K, **kw):
    o = orc.Options(tau_bar=2.0, gamma0=0.1, restart="none", max_iter=K, tol=0.0, **kw)
    r = orc.solve(P, o, trace_cap=K)
    assert r["info"]["iters"] == K
    return r


@pytest.mark.parametrize("variant", ["yx", "xy"])
def test_monotone_trial_count_identity(orc, variant):
    P = orc.Problem(_inst())
    K = 150
    kw = dict(c_nm=0)
    if variant == "xy":
        kw.update(variant="xy", c_alpha=0.25, c_beta=0.3, delta=0.4)
    r = _run(orc, P, K, **kw)
    tr = r["trace"]
    tau, sig, ntr, E, rhs = tr.T
    assert np.all(tau[1:] <= tau[:-1])
    assert np.all(tau <= 2.0)
    np.testing.assert_allclose(sig / tau, 0.1, rtol=1e-14)
    expect = K + np.log(2.0 / tau[-1]) / np.log(1 / 0.7)
    assert abs(ntr.sum() - expect) < 1e-6
    assert r["info"]["trials"] == int(ntr.sum())
    assert np.all(E <= rhs)


@pytest.mark.parametrize("variant", ["yx", "xy"])
def test_nonmonotone_ratio_and_trial_bound(orc, variant):
    P = orc.Problem(_inst())
    K = 150
    kw = dict(c_nm=1)
    if variant == "xy":
        kw.update(variant="xy", c_alpha=0.25, c_beta=0.3, delta=0.4)
    r = _run(orc, P, K, **kw)
    tau, sig, ntr, E, rhs = r["trace"].T
    assert np.all(tau[1:] / tau[:-1] <= PHI * (1 + 1e-12))
    L = np.log(1 / 0.7)
    ratios = np.concatenate([[tau[0] / 2.0], tau[1:] / tau[:-1]])
    bound = K + np.log(2.0 / tau[-1]) / L + 0.5 * np.sum(np.log(1 + ratios[:-1]) / L)
    assert ntr.sum() <= bound + 1e-9
    assert ntr.sum() <= (1 + np.log(PHI) / L) * K + np.log(2.0 / tau.min()) / L + 1e-9
    assert np.all(E <= rhs)


def test_gamma_growth_with_mu(orc):
    P = orc.Problem(_inst())
    K = 60
    r = _run(orc, P, K, c_nm=1, mu=0.05)
    tau, sig, ntr, E, rhs = r["trace"].T
    gam = sig / tau
    assert abs(gam[0] - 0.1) < 1e-15
    np.testing.assert_allclose(gam[1:], gam[:-1] * (1 + 0.05 * tau[:-1]), rtol=1e-13)


def test_speculative_equivalence_of_backtracking(orc):
    """Trial k re-uses tau_k <- eta tau_k: the accepted tau is tau_k^o * eta^(trials-1)."""
    P = orc.Problem(_inst())
    K = 40
    r = _run(orc, P, K, c_nm=1)
    tau, sig, ntr, E, rhs = r["trace"].T
    tau_o = np.empty(K)
    tau_o[0] = 2.0
    prev = 2.0
    for k in range(1, K):
        tau_o[k] = tau[k - 1] * np.sqrt(1 + tau[k - 1] / prev)
        prev = tau[k - 1]
    np.testing.assert_allclose(tau, tau_o * 0.7 ** (ntr - 1), rtol=1e-13)


def test_gap_nonnegative_and_zero_at_saddle(orc):
    inst = _inst()
    P = orc.Problem(inst)
    rng = np.random.default_rng(0)
    for _ in range(3):
        x = rng.uniform(-1, 1, inst.n)
        y = rng.uniform(0, 1, inst.m)
        g = orc.gap(P, x, y)
        assert g["G"] >= 0 and g["Py"] >= 0 and g["Px"] >= -1e-12
    r = orc.solve(P, orc.Options(tau_bar=1.0, gamma0=0.1, tol=1e-11))
    g = orc.gap(P, r["x"], r["y"])
    assert 0 <= g["G"] <= 1e-9


def test_gap_parts_bruteforce(orc):
    """Tiny instance: Px from exact face enumeration of the box QP, Py by numeric maximisation."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(5)
    n, m, xi = 3, 2, 0.04
    Q = np.empty((m + 1, n, n))
    for i in range(m + 1):
        M = rng.standard_normal((n, n))
        Q[i] = M @ M.T / n
    q = rng.standard_normal((m + 1, n))
    c = np.array([0.0, -0.5, -0.3])
    lb, ub = -np.ones(n), np.ones(n)
    P = orc.Problem(Q=Q, q=q, c=c, lb=lb, ub=ub)
    x = np.array([0.3, -0.9, 0.95])
    lam = np.array([0.4, 0.0])
    g = orc.gap(P, x, lam, xi=xi)
    gx = Q[0] @ x + q[0] + sum(lam[i - 1] * (Q[i] @ x + q[i]) for i in (1, 2))
    H = Q[0] + lam[0] * Q[1] + lam[1] * Q[2] + 2 * xi * np.eye(n)
    D, val = pins.box_qp_enumerate(H, gx, lb - x, ub - x)
    assert abs(g["Px"] - (-val)) < 1e-11
    gvals = np.array([0.5 * x @ Q[i] @ x + q[i] @ x + c[i] for i in (1, 2)])

    def negpy(yp):
        return -(gvals @ (yp - lam) - xi * np.sum((yp - lam) ** 2))
    res = minimize(negpy, lam, bounds=[(0, None)] * m, method="L-BFGS-B",
                   options=dict(ftol=1e-15, gtol=1e-12))
    assert abs(g["Py"] - (-res.fun)) < 1e-9


def test_kkt_residual_at_closed_form_and_off_it(orc):
    """rel-KKT ~ 0 at the single-ball optimum from bisection; each block reacts to its own
    violation: a primal shift raises rel_dual, lambda off the optimum raises rel_comp or
    rel_dual, an infeasible point raises rel_pri."""
    n = 10
    rng = np.random.default_rng(7)
    M = rng.standard_normal((n, n))
    Q0 = M @ M.T / n + 0.1 * np.eye(n)
    q0 = 3 * rng.standard_normal(n)
    rho = 0.5
    xs, lam = pins.ball_qp_bisection(Q0, q0, rho)
    P = orc.Problem(Q=np.stack([Q0, np.eye(n)]), q=np.stack([q0, np.zeros(n)]),
                    c=np.array([0.0, -rho]), lb=-10 * np.ones(n), ub=10 * np.ones(n))
    k0 = orc.kkt(P, xs, np.array([lam]))
    assert k0["rel_kkt"] < 1e-12
    k1 = orc.kkt(P, xs * 1.1, np.array([lam]))
    assert k1["rel_pri"] > 1e-3 and k1["rel_dual"] > 1e-3
    k2 = orc.kkt(P, xs, np.array([lam + 1.0]))
    assert k2["rel_dual"] > 1e-3
    k3 = orc.kkt(P, xs * 0.5, np.array([lam]))
    assert k3["rel_comp"] > 1e-2 and k3["rel_pri"] == 0.0


def test_kkt_residual_worked_example(orc):
    """A one-variable instance worked by hand, with every term of the normalisations nonzero
    and distinct: Q_0 = 2, q_0 = 0, c_0 = 0; Q_1 = 4, q_1 = 1, c_1 = -2; A = 2, b = 0.5;
    X = [-10, 10]; at x = 0.5, v = 0.5, lambda = 3:
      Q_0 x + q_0 = 1,  lambda (Q_1 x + q_1) = 3 * 3 = 9,  A'v = 1,  grad_x Phi = 11,
      r_x = 0.5 - clip(0.5 - 11) = 0.5 + 10 = 10.5,  rel_dual = 10.5 / (1 + 1 + 9 + 1) = 0.875;
      g_1 = 0.5 + 0.5 - 2 = -1,  r_l = |min(3, 1)| = 1,  rel_comp = 1 / (1 + 2) = 1/3;
      Ax - b = 0.5,  rel_pri = 0.5 / (1 + 2 + 0.5) = 1/7;
      f = 0.25;  largest violation 0.5."""
    P = orc.Problem(Q=np.array([[[2.0]], [[4.0]]]), q=np.array([[0.0], [1.0]]), c=np.array([0.0, -2.0]),
                    lb=np.array([-10.0]), ub=np.array([10.0]), A=np.array([[2.0]]), b=np.array([0.5]))
    k = orc.kkt(P, np.array([0.5]), np.array([0.5, 3.0]))
    assert k["rel_dual"] == pytest.approx(0.875, rel=1e-15)
    assert k["rel_comp"] == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert k["rel_pri"] == pytest.approx(1.0 / 7.0, rel=1e-15)
    assert k["rel_kkt"] == pytest.approx(0.875, rel=1e-15)
    assert k["f"] == pytest.approx(0.25, rel=1e-15)
    assert k["max_violation"] == pytest.approx(0.5, rel=1e-15)


def _np_ops(inst, x):
    """U and grad_y Phi = (Ax - b, g(x)) with f(x), computed with numpy, independently of the
    oracle (y = (v, lambda))."""
    U = np.einsum("irj,j->ir", inst.Q, x)
    g = np.array([0.5 * x @ U[i] + inst.q[i] @ x + inst.c[i] for i in range(inst.m + 1)])
    r = inst.A @ x - inst.b if inst.p else np.zeros(0)
    return U, np.concatenate([r, g[1:]]), g[0]


def _np_phi(inst, x, y):
    U, G, f = _np_ops(inst, x)
    return f + y @ G


def _np_gradx(inst, x, y):
    U, _, _ = _np_ops(inst, x)
    gx = U[0] + inst.q[0] + y[inst.p:] @ (U[1:] + inst.q[1:])
    return gx + inst.A.T @ y[:inst.p] if inst.p else gx


def _np_proj(inst, y):
    """onto R^p x R^m_+"""
    return np.concatenate([y[:inst.p], np.maximum(0.0, y[inst.p:])])


@pytest.mark.parametrize("constraints", ["inequalities", "with_equalities"])
@pytest.mark.parametrize("start", ["origin", "positive_multipliers"])
@pytest.mark.parametrize("variant", ["yx", "xy"])
def test_test_function_matches_printed_definition(orc, variant, start, constraints):
    """Re-evaluate E_k from its printed definition (Phi differences for yx, gradient
    differences for xy) for the first iterations and check the oracle's accept/reject
    sequence, its recorded E_k and its next iterate.  From lambda^0 = 0 the first dual step of
    yx stays at 0 on this instance (g(x^0) < 0), so the term of E_0 that carries alpha_0 is
    zero; the start with lambda^0 > 0 makes it count.  The second instance adds two equality
    constraints Ax = b (v free), whose multipliers enter grad_x Phi through A'v."""
    inst = qi.random_qcqp(12, 3, seed=31, shift=0.05)
    if constraints == "with_equalities":
        A = np.random.default_rng(3).standard_normal((2, inst.n))
        inst = dataclasses.replace(inst, p=2, A=A, b=A @ np.full(inst.n, 0.05))
    P = orc.Problem(inst)
    ny = inst.p + inst.m
    y0 = None if start == "origin" else np.concatenate([np.full(inst.p, -0.3), np.full(inst.m, 0.5)])
    eta, tb, g0 = 0.7, 2.0, 0.3
    if variant == "yx":
        ca, cb, dl = 0.4, 0.0, 0.5
    else:
        ca, cb, dl = 0.25, 0.3, 0.4
    K = 4
    runs = []
    for k in range(K + 1):
        o = orc.Options(variant=variant, tau_bar=tb, gamma0=g0, restart="none", max_iter=k,
                        tol=0.0, c_alpha=ca, c_beta=cb, delta=dl, eta=eta)
        runs.append(orc.solve(P, o, y0=y0, trace_cap=K))
    tr = runs[K]["trace"]
    for k in range(K):
        x, yk = runs[k]["x"], runs[k]["y"][:ny]
        xp, yp = (runs[k - 1]["x"], runs[k - 1]["y"][:ny]) if k else (x, yk)
        sig_prev = tr[k - 1, 1] if k else g0 * tb
        tau_prev = tr[k - 1, 0] if k else tb
        tau_pp = (tr[k - 2, 0] if k >= 2 else tb)
        tau0 = tb if k == 0 else tau_prev * np.sqrt(1 + tau_prev / tau_pp)
        alpha_k = ca / sig_prev if variant == "yx" else ca / tau_prev
        beta_k = g0 * cb / sig_prev
        _, G, _ = _np_ops(inst, x)
        _, Gp, _ = _np_ops(inst, xp)
        for j in range(60):
            tau = tau0 * eta ** j
            sig = g0 * tau
            th = sig_prev / sig
            if variant == "yx":
                ly = _np_proj(inst, yk + sig * ((1 + th) * G - th * Gp))
                xn = np.clip(x - tau * _np_gradx(inst, x, ly), inst.lb, inst.ub)
                d = xn - x
                _, Gn, _ = _np_ops(inst, xn)
                E = (_np_phi(inst, xn, ly) - _np_phi(inst, x, ly) - _np_gradx(inst, x, ly) @ d
                     - 0.5 * d @ d / tau + np.sum((Gn - G) ** 2) / (2 * ca / sig)
                     - (1 / sig - th * alpha_k) * 0.5 * np.sum((ly - yk) ** 2))
            else:
                s = (1 + th) * _np_gradx(inst, x, yk) - th * _np_gradx(inst, xp, yp)
                xn = np.clip(x - tau * s, inst.lb, inst.ub)
                d = xn - x
                _, Gn, _ = _np_ops(inst, xn)
                ly = _np_proj(inst, yk + sig * Gn)
                a1, b1 = ca / tau, g0 * cb / sig
                E = (np.sum((_np_gradx(inst, xn, ly) - _np_gradx(inst, xn, yk)) ** 2) / (2 * a1)
                     - 0.5 * np.sum((ly - yk) ** 2) / sig
                     + np.sum((_np_gradx(inst, xn, yk) - _np_gradx(inst, x, yk)) ** 2) / (2 * b1)
                     - (1 / tau - th * (alpha_k + beta_k)) * 0.5 * d @ d)
            rhs = -dl / tau * 0.5 * d @ d - dl / sig * 0.5 * np.sum((ly - yk) ** 2)
            if E <= rhs:
                break
        assert j + 1 == int(tr[k, 2]), (k, j, tr[k])
        assert abs(E - tr[k, 3]) <= 1e-7 * (abs(E) + abs(rhs))
        np.testing.assert_allclose(runs[k + 1]["x"], xn, rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(runs[k + 1]["y"][:ny], ly, rtol=1e-11, atol=1e-12)
