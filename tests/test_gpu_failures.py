"""Failure paths that arise inside a solve: finite data whose iteration overflows.

A constraint matrix scaled to 1e200 is finite, so qcqp_create accepts it, but the first trial
point's constraint value and the ||G(x+) - G(x)||^2 term of the backtracking test overflow to
infinity: no step size passes the test, the step underflows or the trial cap is met, and the
solve must stop with QCQP_E_NUMERICAL rather than loop or return a number.  In a batch the failed
slot is reported finished with that status while a healthy slot beside it still returns the same
bits as alone.  (The kernels only compute with inf/NaN; nothing faults.)
"""
import numpy as np
import pytest

from tests.gpu_common import announce, oracle, qi, tau_bar_of, to_np

pytestmark = pytest.mark.gpu


def _overflowing(n=24, m=2, seed=91):
    inst = qi.random_qcqp(n, m, seed=seed, shift=0.01)
    Q = inst.Q.copy()
    Q[1] *= 1e200
    inst.Q = Q
    return inst


def test_overflow_mid_solve_returns_numerical():
    from paper_2605_29291_amd import QCQPError, Solver, abi
    inst = _overflowing()
    assert np.all(np.isfinite(inst.Q))
    announce("overflow mid-solve, single instance")
    s = Solver(inst, tau_bar=1.0, gamma0=0.1)
    with pytest.raises(QCQPError) as e:
        s.solve()
    assert e.value.code == abi.E_NUMERICAL
    s.close()


def test_failed_slot_leaves_its_batch_neighbour_unchanged():
    from paper_2605_29291_amd import Batch, Solver
    good = qi.random_qcqp(80, 6, seed=92, shift=0.01)
    opts = dict(tau_bar=tau_bar_of(good), gamma0=0.1)
    announce("healthy request alone")
    s = Solver(good, **opts)
    x0, y0, i0 = s.solve()
    s.close()
    announce("healthy request beside an overflowing one")
    b = Batch(max_slots=2)
    bad_slot = b.admit(Solver(_overflowing(), tau_bar=1.0, gamma0=0.1))
    good_slot = b.admit(Solver(good, **opts))
    got = {}
    for _ in range(10000):
        b.step(4)
        for slot in b.poll():
            got[slot] = b.fetch(slot)
        if len(got) == 2:
            break
    b.close()
    assert got[bad_slot][3]["status"] == "numerical", got[bad_slot][3]
    _, xg, yg, ig = got[good_slot]
    assert ig["status"] == "ok"
    np.testing.assert_array_equal(to_np(xg), to_np(x0))
    np.testing.assert_array_equal(to_np(yg), to_np(y0))
    assert (ig["iters"], ig["trials"]) == (i0["iters"], i0["trials"])


def test_create_refuses_asymmetric_or_non_finite_matrices():
    from paper_2605_29291_amd import QCQPError, Solver, abi
    base = qi.random_qcqp(70, 3, seed=93, shift=0.01)
    announce("asymmetric / non-finite Q refused at create")
    for storage in ("float64", "bfloat16"):
        for sym in ((0, 1) if storage == "float64" else (0,)):
            bad = qi.random_qcqp(70, 3, seed=93, shift=0.01)
            Q = bad.Q.copy()
            # one entry off its mirror image, by more than a 16-bit rounding step (the check
            # sees the stored values)
            Q[2, 5, 40] += (1e-6 if storage == "float64" else 1e-2) * np.abs(Q[2]).max()
            bad.Q = Q
            with pytest.raises(QCQPError) as e:
                Solver(bad, tau_bar=1.0, storage=storage, sym_pass=sym)
            assert e.value.code == abi.E_INVALID and "not symmetric" in str(e.value)
            nan = qi.random_qcqp(70, 3, seed=93, shift=0.01)
            Q = nan.Q.copy()
            Q[1, 69, 3] = np.nan
            nan.Q = Q
            with pytest.raises(QCQPError) as e:
                Solver(nan, tau_bar=1.0, storage=storage, sym_pass=sym)
            assert e.value.code == abi.E_INVALID and "non-finite" in str(e.value)
    # an unsymmetrised product A A' / n is symmetric only up to rounding: accepted
    rng = np.random.default_rng(5)
    A = rng.standard_normal((4, 70, 70))
    near = qi.random_qcqp(70, 3, seed=93, shift=0.01)
    near.Q = np.einsum("kij,klj->kil", A, A) / 70
    s = Solver(near, tau_bar=1.0)
    s.close()


def test_infeasible_problem_runs_to_its_cap_like_the_oracle():
    """g_1(x) = 1/2 ||x||^2 + 1 <= 0 has no solution.  The solve stops at max_iter with status
    not_converged and finite iterates, its multiplier of the impossible constraint grows, the
    primal residual stays away from zero, and the trajectory equals the oracle's (same trial
    count, iterates to 1e-10)."""
    import dataclasses
    base = qi.random_qcqp(60, 3, seed=81, shift=0.01)
    Q, q, c = base.Q.copy(), base.q.copy(), base.c.copy()
    Q[1], q[1], c[1] = np.eye(60), 0.0, 1.0
    inst = dataclasses.replace(base, Q=Q, q=q, c=c, name="infeasible")
    tb = 1.0 / np.linalg.norm(Q[0], 2)
    from paper_2605_29291_amd import Solver
    announce("infeasible QCQP to its iteration cap")
    x, y, info = Solver(inst, tau_bar=tb, gamma0=0.1, max_iter=300, tol=1e-6).solve()
    ref = oracle.solve(oracle.Problem(inst), oracle.Options(tau_bar=tb, gamma0=0.1, max_iter=300, tol=1e-6))
    assert info["status"] == "not_converged" and ref["info"]["status"] == "not_converged", (info, ref["info"])
    assert info["iters"] == 300 and info["trials"] == ref["info"]["trials"]
    xs, ys = to_np(x), to_np(y)
    assert np.all(np.isfinite(xs)) and np.all(np.isfinite(ys))
    np.testing.assert_allclose(xs, ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(ys, ref["y"][:3], rtol=1e-10, atol=1e-11)
    assert ys[0] > 10.0
    kk = oracle.kkt(oracle.Problem(inst), xs, ys)
    assert kk["rel_pri"] > 0.1 and abs(info["rel_kkt"] - kk["rel_kkt"]) <= 1e-12 * (1 + kk["rel_kkt"])
