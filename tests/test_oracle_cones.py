"""Pins for the oracle's conic dual domain and its map of stored matrices.

lambda in R^{m0}_+ x Q^{k_1} x ... x Q^{k_r} (second-order cones, self-dual) is the multiplier of
a conic constraint g(x) in -K (the cone setting of §2.1).  Constraints whose Q_i = 0 (affine)
need no stored matrix.  Pinned against:
  * the projection onto K*: the variational inequality on points and extreme rays of the cone,
    and the spectral-decomposition formula of the second-order cone (an independent closed
    form);
  * min 1/2 ||x - a||^2 s.t. x in Q^n, written as g(x) = (-x_1, x_2, ..., x_n) in -Q^n with every
    g_i affine (no stored matrix): the solution is the projection of a onto Q^n;
  * a quadratic second-order-cone constraint rho - 1/2 ||x||^2 >= ||Bx + b|| against scipy's
    SLSQP, and the optimality conditions (lambda in Q, <lambda, g> = 0, small KKT residual);
  * one-dimensional cones Q^1 = R_+ give the R^m_+ trajectory bitwise;
  * a stored zero matrix and an absent one give the same trajectory bitwise.
"""
import numpy as np
import pytest

import qcqp_inputs as qi


def _proj_soc_spectral(z):
    """Pi_Q(z) by the spectral decomposition z = l1 u1 + l2 u2, l = t -+ ||x||."""
    t, x = z[0], z[1:]
    nx = np.linalg.norm(x)
    w = x / nx if nx > 0 else np.zeros_like(x)
    if len(x) and nx == 0:
        w = np.zeros_like(x)
        w[0] = 1.0
    u1 = 0.5 * np.concatenate([[1.0], -w])
    u2 = 0.5 * np.concatenate([[1.0], w])
    l1, l2 = t - nx, t + nx
    return max(l1, 0.0) * u1 + max(l2, 0.0) * u2


def _cone_members(rng, dims, m0, count=300):
    pts = []
    for _ in range(count):
        parts = [np.abs(rng.standard_normal(m0)) * (rng.random(m0) > 0.3)]
        for k in dims:
            u = rng.standard_normal(k - 1)
            r = np.linalg.norm(u) if k > 1 else 0.0
            t = r * rng.choice([1.0, 1.0 + rng.uniform(0, 2)])      # boundary or interior
            parts.append(np.concatenate([[t], u]) * rng.uniform(0, 3))
        pts.append(np.concatenate(parts))
    return pts


def _cone_problem(orc, n, m, dims, **kw):
    return orc.Problem(Q=np.zeros((m + 1, n, n)), q=np.zeros((m + 1, n)), c=np.zeros(m + 1),
                       lb=-np.ones(n), ub=np.ones(n), lambda_set="cones", soc_dims=dims, **kw)


@pytest.mark.parametrize("ball", [0.0, 2.0])
def test_cone_projection_variational_inequality(orc, ball):
    rng = np.random.default_rng(3)
    dims = [3, 1, 4]
    m0 = 2
    m = m0 + sum(dims)
    P = _cone_problem(orc, 2, m, dims, ball=ball)
    members = _cone_members(rng, dims, m0)
    if ball:
        members = [u * min(1.0, rng.uniform(0, 1) * ball / max(np.linalg.norm(u), 1e-300))
                   for u in members]
    for trial in range(80):
        z = rng.standard_normal(m) * rng.choice([0.1, 1.0, 10.0])
        w = orc.project_dual(P, z)
        # feasibility
        assert np.all(w[:m0] >= 0)
        off = m0
        for k in dims:
            assert np.linalg.norm(w[off + 1:off + k]) <= w[off] * (1 + 1e-14) + 1e-300
            off += k
        if ball:
            assert np.linalg.norm(w) <= ball * (1 + 1e-15)
        worst = max(float((z - w) @ (u - w)) for u in members)
        assert worst <= 1e-12 * (1 + np.linalg.norm(z)) ** 2, (trial, worst)
        if not ball:
            ref = np.concatenate([np.maximum(z[:m0], 0)] +
                                 [_proj_soc_spectral(z[o:o + k]) for o, k in
                                  zip(np.cumsum([m0] + dims[:-1]), dims)])
            np.testing.assert_allclose(w, ref, atol=1e-13 * (1 + np.linalg.norm(z)))
        np.testing.assert_allclose(orc.project_dual(P, w), w, atol=1e-14)


@pytest.mark.parametrize("variant", ["yx", "xy"])
def test_affine_soc_constraint_gives_the_cone_projection(orc, variant):
    """min 1/2||x - a||^2 s.t. x_1 >= ||x_{2:n}||: g(x) = (-x_1, x_2, .., x_n) in -Q^n, affine,
    so only Q_0 = I is stored; the answer is Pi_Q(a)."""
    rng = np.random.default_rng(5)
    n = 6
    a = rng.standard_normal(n)
    a[0] = -0.3                                      # a lies outside the cone
    x_ref = _proj_soc_spectral(a)
    q = np.zeros((n + 1, n))
    q[0] = -a
    q[1, 0] = -1.0
    for j in range(1, n):
        q[1 + j, j] = 1.0
    stored = np.zeros(n + 1, dtype=np.int32)
    stored[0] = 1
    P = orc.Problem(Q=np.eye(n)[None], q=q, c=np.zeros(n + 1), lb=-10 * np.ones(n),
                    ub=10 * np.ones(n), lambda_set="cones", soc_dims=[n], q_stored=stored)
    mk = orc.Options.xy if variant == "xy" else orc.Options
    r = orc.solve(P, mk(tau_bar=1.0, gamma0=1.0, tol=1e-11, max_iter=200000))
    assert r["info"]["status"] == "converged", r["info"]
    np.testing.assert_allclose(r["x"], x_ref, atol=1e-8)
    lam = r["y"]
    assert np.linalg.norm(lam[1:]) <= lam[0] * (1 + 1e-12)         # lambda in Q^n (self-dual)
    g = np.concatenate([[-r["x"][0]], r["x"][1:]])
    assert abs(lam @ g) <= 1e-8                                    # complementarity


def test_quadratic_soc_constraint_against_slsqp(orc):
    """rho - 1/2||x||^2 >= ||Bx + b||: g = (1/2||x||^2 - rho, Bx + b) in -Q^{k+1}; convex since
    lambda_1 >= 0 on Q.  Reference: scipy SLSQP on the same problem."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(7)
    n, k, rho = 4, 2, 2.0
    A = rng.standard_normal((n, n))
    Q0 = A @ A.T / n + 0.3 * np.eye(n)
    q0 = rng.standard_normal(n) * 4
    B = rng.standard_normal((k, n))
    b = rng.standard_normal(k) * 0.3
    m = k + 1
    Q = np.stack([Q0, np.eye(n)])
    q = np.zeros((m + 1, n))
    q[0] = q0
    q[2:] = B
    c = np.concatenate([[0.0, -rho], b])
    stored = np.array([1, 1] + [0] * k, dtype=np.int32)
    P = orc.Problem(Q=Q, q=q, c=c, lb=-10 * np.ones(n), ub=10 * np.ones(n), lambda_set="cones",
                    soc_dims=[m], q_stored=stored)
    r = orc.solve(P, orc.Options(tau_bar=1.0 / np.linalg.norm(Q0, 2), gamma0=1.0, tol=1e-10,
                                 max_iter=200000))
    assert r["info"]["status"] == "converged", r["info"]
    fun = lambda x: 0.5 * x @ Q0 @ x + q0 @ x
    con = lambda x: rho - 0.5 * x @ x - np.linalg.norm(B @ x + b)
    # SLSQP may report a line-search stop at this precision; its point is checked directly
    ref = minimize(fun, np.zeros(n), jac=lambda x: Q0 @ x + q0, method="SLSQP",
                   constraints=[{"type": "ineq", "fun": con}], options=dict(ftol=1e-13, maxiter=2000))
    assert con(ref.x) >= -1e-9
    assert con(r["x"]) >= -1e-9
    np.testing.assert_allclose(r["x"], ref.x, atol=1e-5)
    assert fun(r["x"]) <= fun(ref.x) + 1e-8
    lam = r["y"]
    assert np.linalg.norm(lam[1:]) <= lam[0] * (1 + 1e-12)
    x = r["x"]
    g = np.concatenate([[0.5 * x @ x - rho], B @ x + b])
    assert abs(lam @ g) <= 1e-7
    assert orc.kkt(P, x, lam)["rel_kkt"] <= 1e-9


def test_one_dimensional_cones_are_the_nonnegative_orthant(orc):
    inst = qi.random_qcqp(30, 4, seed=9, shift=0.01)
    L = np.linalg.norm(inst.Q[0], 2)
    o = orc.Options(tau_bar=1 / L, tol=0.0, max_iter=80)
    a = orc.solve(orc.Problem(inst), o)
    b = orc.solve(orc.Problem(inst, lambda_set="cones", soc_dims=[1, 1]), o)
    np.testing.assert_array_equal(a["x"], b["x"])
    np.testing.assert_array_equal(a["y"], b["y"])


def test_stored_zero_matrix_equals_absent_matrix(orc):
    inst = qi.random_qcqp(25, 3, seed=10, shift=0.01)
    Q = np.array(inst.Q)
    Q[2] = 0.0
    L = np.linalg.norm(Q[0], 2)
    o = orc.Options(tau_bar=1 / L, tol=0.0, max_iter=60)
    dense = orc.solve(orc.Problem(Q=Q, q=inst.q, c=inst.c, lb=inst.lb, ub=inst.ub), o)
    stored = np.array([1, 1, 0, 1], dtype=np.int32)
    sparse = orc.solve(orc.Problem(Q=Q[[0, 1, 3]], q=inst.q, c=inst.c, lb=inst.lb, ub=inst.ub,
                                   q_stored=stored), o)
    np.testing.assert_array_equal(dense["x"], sparse["x"])
    np.testing.assert_array_equal(dense["y"], sparse["y"])


def test_cone_validation(orc):
    n = 3
    Q = np.stack([np.eye(n), np.eye(n), np.eye(n)])
    q = np.zeros((3, n))
    c = np.array([0.0, -1.0, -1.0])
    lb, ub = -np.ones(n), np.ones(n)
    o = orc.Options(tau_bar=1.0)
    for kw in (dict(soc_dims=[3]), dict(soc_dims=[0]), dict(soc_dims=[])):
        P = orc.Problem(Q=Q, q=q, c=c, lb=lb, ub=ub, lambda_set="cones", **kw)
        assert orc.solve(P, o)["info"]["status"] == "invalid", kw
    bad = np.array([0, 1, 1], dtype=np.int32)       # disagrees with has_q0
    P = orc.Problem(Q=Q[1:], q=q, c=c, lb=lb, ub=ub, q_stored=bad)
    assert orc.solve(P, o)["info"]["status"] == "invalid"


def test_cone_kkt_residual_worked_example(orc):
    """One variable, one scalar constraint in R_+ and one second-order cone of dimension 2,
    all affine (only Q_0 = 2 stored), worked by hand at x = 1, lambda = 0:
      g = (q_i x + c_i) = (0.5, (1, 3));  Pi_{R_+}(0.5) = 0.5;  the cone block (t, u) = (1, 3)
      has |u| > |t|, so Pi_Q = ((1 + 3) / 2) (1, 3 / 3) = (2, 2), of norm 2 sqrt(2);
      dist(g, -K) = ||Pi_K*(g)|| = sqrt(0.25 + 8) and the largest violation is 2 sqrt(2);
      r_l = ||lambda - Pi_K*(lambda + g)|| = sqrt(8.25);  ||c_{1..3}|| = sqrt(10.25);
      grad_x Phi = Q_0 x = 2, r_x = 1 - clip(1 - 2) = 2, rel_dual = 2 / (1 + 2)."""
    q = np.zeros((4, 1))
    c = np.array([0.0, 0.5, 1.0, 3.0])
    stored = np.array([1, 0, 0, 0], dtype=np.int32)
    P = orc.Problem(Q=np.array([[[2.0]]]), q=q, c=c, lb=np.array([-10.0]), ub=np.array([10.0]),
                    lambda_set="cones", soc_dims=[2], q_stored=stored)
    k = orc.kkt(P, np.array([1.0]), np.zeros(3))
    den = 1.0 + np.sqrt(10.25)
    assert k["max_violation"] == pytest.approx(2.0 * np.sqrt(2.0), rel=1e-15)
    assert k["rel_pri"] == pytest.approx(np.sqrt(8.25) / den, rel=1e-15)
    assert k["rel_comp"] == pytest.approx(np.sqrt(8.25) / den, rel=1e-15)
    assert k["rel_dual"] == pytest.approx(2.0 / 3.0, rel=1e-15)
    assert k["rel_kkt"] == pytest.approx(np.sqrt(8.25) / den, rel=1e-15)
    assert k["f"] == pytest.approx(1.0, rel=1e-15)
