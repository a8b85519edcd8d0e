"""Pins for the oracle's restart driver.

rAPDB (Algorithm 2, §4.1) calls the APDB routine again from the restart point, so a restart runs
the routine's first line afresh: tau_{-1} = tau_0 = tau_bar, sigma_{-1} = gamma_0 tau_bar,
gamma = gamma_0, x^{-1} = x^0 (no momentum), the weighted averages emptied.  The restart point is
the weighted average of the epoch's iterates in Algorithm 2 and the last iterate in the
experiments (§5.1); both are options.  The adaptive variant (eq. (ada_restart), §4.2) restarts
when G_xi at the candidate point is at most q times G_xi at the epoch's start, on the schedule of
§5.1: G_xi at k = ada_first gives the first reference without a restart, then the test runs at
every global k > ada_first with k % ada_every == 0, and a successful test makes the candidate's
value the new reference.

The pins check the driver from outside the oracle:
  * the step sizes of every iteration, recomputed in numpy from the trace's trial counts with the
    first line of Algorithm 1 re-entered at every restart (a restart that keeps tau or gamma, or
    a missing restart, changes them);
  * the iterates after a restart equal those of a fresh solve started at the restart point;
  * every adaptive decision equals the one an independent numpy G_xi (closed-form y-part, exact
    box-QP face enumeration, tests/pins.py) makes at the same iterates, and the number of G_xi
    evaluations equals the number of schedule points;
  * the restart point of Algorithm 2 equals sum_k t_k z^{k+1} / sum_k t_k with t_k = sigma_k /
    sigma_0, recomputed from the iterates and the trace.
"""
import numpy as np
import pytest

import qcqp_inputs as qi
from tests import pins


def _opts(orc, variant="yx", **kw):
    if variant == "xy":
        return orc.Options.xy(**kw)
    return orc.Options(**kw)


def _capped(orc, P, variant, base, k, **extra):
    """Solve with max_iter = k: returns the iterate z^k before any restart decision at k."""
    kw = dict(base)
    kw.update(extra)
    kw["max_iter"] = k
    return orc.solve(P, _opts(orc, variant, **kw), trace_cap=max(k, 1))


def _expected_steps(trace, restart_at, tau_bar, gamma0, mu, eta, c_nm):
    """tau_k and sigma_k of every accepted iteration from the trial counts alone: Algorithm 1's
    step-size rule (non-monotone form for c_nm = 1) with its first line re-entered at each k in
    restart_at (and at k = 0)."""
    K = len(trace)
    tau = np.empty(K)
    sig = np.empty(K)
    for k in range(K):
        if k == 0 or k in restart_at:
            nom, prev, gam = tau_bar, tau_bar, gamma0
        t = int(trace[k, 2])
        tau[k] = nom * eta ** (t - 1)
        sig[k] = gam * tau[k]
        gam_next = gam * (1.0 + mu * tau[k])
        nom = tau[k] * np.sqrt(gam / gam_next * (1.0 + c_nm * tau[k] / prev))
        prev = tau[k]
        gam = gam_next
    return tau, sig


FIXED_CASES = [dict(variant="yx", c_nm=1, mu=0.0),
               dict(variant="yx", c_nm=1, mu=0.3),
               dict(variant="yx", c_nm=0, mu=0.3),
               dict(variant="xy", c_nm=1, mu=0.0),
               dict(variant="xy", c_nm=0, mu=0.3)]


@pytest.mark.parametrize("case", FIXED_CASES, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_fixed_restarts_reenter_the_first_line(orc, case):
    """Every K-hat accepted iterations tau, sigma/tau = gamma and the non-monotone ratio start
    afresh; in between they follow Algorithm 1's rule.  mu > 0 makes gamma grow within an epoch,
    so a restart that kept gamma would show in sigma/tau."""
    inst = qi.random_qcqp(20, 4, seed=11, shift=0.01)
    P = orc.Problem(inst)
    Khat = 9
    tau_bar = 1.0 / np.linalg.norm(inst.Q[0], 2)
    variant = case["variant"]
    base = dict(tau_bar=tau_bar, gamma0=0.1, mu=case["mu"], c_nm=case["c_nm"], tol=1e-9,
                max_iter=20000, restart="fixed", restart_every=Khat)
    r = orc.solve(P, _opts(orc, variant, **base), trace_cap=20000)
    info, tr = r["info"], r["trace"]
    assert info["status"] == "converged"
    K = info["iters"]
    assert K > 3 * Khat
    restart_at = set(range(Khat, K, Khat))
    assert info["restarts"] == len(restart_at)
    o = _opts(orc, variant, **base)
    tau, sig = _expected_steps(tr, restart_at, tau_bar, o.gamma0, o.mu, o.eta, o.c_nm)
    np.testing.assert_allclose(tr[:, 0], tau, rtol=1e-12)
    np.testing.assert_allclose(tr[:, 1], sig, rtol=1e-12)
    for k in restart_at:
        assert tr[k, 1] / tr[k, 0] == pytest.approx(o.gamma0, rel=1e-14)
        assert tr[k, 0] == pytest.approx(tau_bar * o.eta ** (tr[k, 2] - 1), rel=1e-13)
    if case["mu"] > 0:   # gamma has grown by the end of every epoch
        assert tr[Khat - 1, 1] / tr[Khat - 1, 0] > 1.01 * o.gamma0


@pytest.mark.parametrize("variant", ["yx", "xy"])
@pytest.mark.parametrize("from_average", [False, True])
def test_restart_continues_as_a_fresh_solve(orc, variant, from_average):
    """After the restart at k = K-hat the trajectory is that of a new solve started at the
    restart point: same step sizes and trial counts, same iterates (no momentum, no carried
    step size, no carried averages)."""
    inst = qi.random_qcqp(20, 4, seed=12, shift=0.01)
    P = orc.Problem(inst)
    Khat = 8
    base = dict(tau_bar=1.0 / np.linalg.norm(inst.Q[0], 2), gamma0=0.1, tol=1e-12,
                restart="fixed", restart_every=Khat, restart_from_average=from_average)
    full = _capped(orc, P, variant, base, 3 * Khat)
    assert full["info"]["restarts"] == 2
    z = _restart_point(orc, P, variant, base, Khat, from_average)
    fresh_kw = dict(base, restart="none")
    fresh = orc.solve(P, _opts(orc, variant, **dict(fresh_kw, max_iter=2 * Khat)),
                      x0=z[0], y0=z[1], trace_cap=2 * Khat)
    a, b = full["trace"][Khat:2 * Khat], fresh["trace"][:Khat]
    np.testing.assert_array_equal(a[:, 2], b[:, 2])
    np.testing.assert_allclose(a[:, :2], b[:, :2], rtol=1e-12)
    np.testing.assert_allclose(a[:, 3:], b[:, 3:], rtol=1e-8, atol=1e-14)
    at2 = _capped(orc, P, variant, base, 2 * Khat)
    ref2 = orc.solve(P, _opts(orc, variant, **dict(fresh_kw, max_iter=Khat)), x0=z[0], y0=z[1])
    np.testing.assert_allclose(at2["x"], ref2["x"], rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(at2["y"], ref2["y"], rtol=1e-11, atol=1e-13)


def _restart_point(orc, P, variant, base, Khat, from_average):
    """The point Algorithm 2 restarts from after the first epoch of K-hat iterations: the last
    iterate z^{K-hat}, or sum_k t_k z^{k+1} / sum_k t_k with t_k = sigma_k / sigma_0."""
    last = _capped(orc, P, variant, base, Khat)
    if not from_average:
        return last["x"], last["y"]
    sig = last["trace"][:Khat, 1]
    t = sig / sig[0]
    xs = np.zeros(P.n)
    ys = np.zeros(P.ny)
    for k in range(Khat):
        zk = _capped(orc, P, variant, base, k + 1)
        xs += t[k] * zk["x"]
        ys += t[k] * zk["y"]
    xa, ya = xs / t.sum(), ys / t.sum()
    # the average must differ from the last iterate, or this case pins nothing
    assert np.linalg.norm(xa - last["x"]) > 1e-3 * (1 + np.linalg.norm(xa))
    return xa, ya


def test_restart_point_is_the_weighted_average(orc):
    """Algorithm 2's restart point: with restart_from_average the first iteration after the
    restart starts from sum t_k z^{k+1} / sum t_k (checked against a fresh solve from the
    numpy average), and not from the last iterate."""
    inst = qi.random_qcqp(15, 3, seed=13, shift=0.01)
    P = orc.Problem(inst)
    Khat = 6
    base = dict(tau_bar=1.0 / np.linalg.norm(inst.Q[0], 2), gamma0=0.1, tol=1e-12,
                restart="fixed", restart_every=Khat, restart_from_average=True)
    after = _capped(orc, P, "yx", base, Khat + 1)
    assert after["info"]["restarts"] == 1
    xa, ya = _restart_point(orc, P, "yx", base, Khat, True)
    one = orc.solve(P, _opts(orc, "yx", **dict(base, restart="none", max_iter=1)), x0=xa, y0=ya)
    np.testing.assert_allclose(after["x"], one["x"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(after["y"], one["y"], rtol=1e-12, atol=1e-14)
    xl, yl = _restart_point(orc, P, "yx", base, Khat, False)
    wrong = orc.solve(P, _opts(orc, "yx", **dict(base, restart="none", max_iter=1)), x0=xl, y0=yl)
    assert np.linalg.norm(wrong["x"] - after["x"]) > 1e-6


ADA_CASES = [dict(variant="yx", seed=0, box=1.0, q=0.15, first=5, every=10),
             dict(variant="yx", seed=2, box=10.0, q=0.15, first=5, every=10),
             dict(variant="yx", seed=4, box=1.0, q=0.5, first=5, every=10),
             dict(variant="xy", seed=0, box=1.0, q=0.3, first=10, every=20)]


@pytest.mark.parametrize("case", ADA_CASES, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_adaptive_decisions_match_an_independent_gap(orc, case):
    """Walk the §5.1 schedule: at every schedule point take the oracle's iterate (a solve capped
    there), evaluate G_xi with the independent numpy routine, decide eq. (ada_restart) with the
    reference rule of §5.1, and compare with what the oracle did there (its restart count one
    iteration later, and a step size that restarted from tau_bar)."""
    inst = qi.random_qcqp(6, 3, seed=case["seed"], shift=0.0, box=case["box"])
    P = orc.Problem(inst)
    xi = 0.04
    variant = case["variant"]
    base = dict(tau_bar=1.0 / np.linalg.norm(inst.Q[0], 2), gamma0=0.1, tol=1e-10,
                max_iter=5000, restart="adaptive", ada_first=case["first"],
                ada_every=case["every"], q_restart=case["q"], xi=xi)
    full = orc.solve(P, _opts(orc, variant, **base), trace_cap=5000)
    K = full["info"]["iters"]
    assert full["info"]["status"] == "converged"
    sched = [case["first"]] + [k for k in range(case["first"] + 1, K) if k % case["every"] == 0]
    assert full["info"]["gap_evals"] == len(sched)
    o = _opts(orc, variant, **base)
    Gref = None
    fired = held = 0
    restart_at = set()
    for s in sched:
        zs = _capped(orc, P, variant, base, s)
        G = pins.smoothed_gap(inst.Q, inst.q, inst.c, inst.lb, inst.ub, zs["x"], zs["y"], xi)
        n_before = zs["info"]["restarts"]
        n_after = _capped(orc, P, variant, base, s + 1)["info"]["restarts"]
        if Gref is None:                        # k = ada_first: reference only
            Gref = G
            assert n_after == n_before
            continue
        assert abs(G - case["q"] * Gref) > 1e-3 * Gref, "decision too close to call"
        if G <= case["q"] * Gref:
            fired += 1
            restart_at.add(s)
            Gref = G
            assert n_after == n_before + 1, (s, G, Gref)
        else:
            held += 1
            assert n_after == n_before, (s, G, Gref)
    assert full["info"]["restarts"] == fired
    assert fired >= 3 and held >= 1
    assert full["info"]["last_gap"] == pytest.approx(G, rel=1e-8, abs=1e-14)
    tau, sig = _expected_steps(full["trace"], restart_at, base["tau_bar"], o.gamma0, o.mu,
                               o.eta, o.c_nm)
    np.testing.assert_allclose(full["trace"][:, 0], tau, rtol=1e-12)
    np.testing.assert_allclose(full["trace"][:, 1], sig, rtol=1e-12)


def test_adaptive_from_average_tests_the_average(orc):
    """With restart_from_average the schedule's candidate is the epoch's weighted average: the
    oracle's G_xi at the first test point equals the numpy G_xi of the average of the iterates
    since the start (no restart before it)."""
    inst = qi.random_qcqp(6, 3, seed=0, shift=0.0, box=1.0)
    P = orc.Problem(inst)
    xi, first, every = 0.04, 5, 10
    base = dict(tau_bar=1.0 / np.linalg.norm(inst.Q[0], 2), gamma0=0.1, tol=1e-10,
                restart="adaptive", ada_first=first, ada_every=every, q_restart=0.15, xi=xi,
                restart_from_average=True)
    s = every
    zs = _capped(orc, P, "yx", base, s + 1)
    assert zs["info"]["gap_evals"] == 2
    xa, ya = _restart_point(orc, P, "yx", dict(base, restart="none"), s, True)
    G = pins.smoothed_gap(inst.Q, inst.q, inst.c, inst.lb, inst.ub, xa, ya, xi)
    assert zs["info"]["last_gap"] == pytest.approx(G, rel=1e-8)
    zl = _capped(orc, P, "yx", dict(base, restart="none"), s)
    G_last = pins.smoothed_gap(inst.Q, inst.q, inst.c, inst.lb, inst.ub, zl["x"], zl["y"], xi)
    assert abs(G_last - G) > 1e-6 * G
