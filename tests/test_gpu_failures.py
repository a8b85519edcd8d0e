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

from tests.gpu_common import announce, qi, tau_bar_of, to_np

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
