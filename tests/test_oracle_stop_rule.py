"""Pin for the oracle's second stop rule: the termination criterion of the experiments of §5.1,
max{ |f(x) - f*| / (1 + |f*|), mean constraint violation } <= tol for a known optimal value f*.
The criterion is re-evaluated from the problem data with numpy at the iterate where the solve
stops and at the iterate before it (obtained by capping the iteration count)."""
import dataclasses

import numpy as np
import pytest

import qcqp_inputs as qi


def _paper_criterion_numpy(Q, q, c, x, f_star, A=None, b=None):
    """max{|f - f*|/(1 + |f*|), mean violation} evaluated from the data with numpy."""
    m = q.shape[0] - 1
    f = 0.5 * x @ Q[0] @ x + q[0] @ x + c[0]
    g = np.array([0.5 * x @ Q[i] @ x + q[i] @ x + c[i] for i in range(1, m + 1)])
    viol = list(np.maximum(g, 0.0))
    if A is not None:
        viol += list(np.abs(A @ x - b))
    return max(abs(f - f_star) / (1 + abs(f_star)), float(np.mean(viol)) if viol else 0.0)


@pytest.mark.parametrize("variant", ["yx", "xy"])
def test_paper_stop_rule_fires_at_the_first_crossing(orc, variant):
    """The criterion of §5.1 stops the solve at the first iterate where it is <= tol: at k-1
    it is above tol and at k below, both evaluated independently from the problem data."""
    inst = qi.paper_random_qcqp(60, 4, seed=3)
    P = orc.Problem(inst)
    L = np.linalg.norm(inst.Q[0], 2)
    mk = orc.Options.xy if variant == "xy" else orc.Options
    ref = orc.solve(P, mk(tau_bar=1 / L, gamma0=1.0, tol=1e-11, max_iter=200000))
    assert ref["info"]["status"] == "converged"
    fs = ref["info"]["f"]
    kw = dict(tau_bar=1 / L, gamma0=1.0, stop_rule="paper", f_star=fs, max_iter=50000)
    r = orc.solve(P, mk(tol=1e-6, **kw))
    assert r["info"]["status"] == "converged"
    k = r["info"]["iters"]
    assert k > 1
    crit_k = _paper_criterion_numpy(inst.Q, inst.q, inst.c, r["x"], fs)
    assert abs(crit_k - r["info"]["stop_value"]) <= 1e-12
    assert crit_k <= 1e-6
    before = orc.solve(P, mk(tol=0.0, **dict(kw, max_iter=k - 1)))
    assert before["info"]["iters"] == k - 1
    assert _paper_criterion_numpy(inst.Q, inst.q, inst.c, before["x"], fs) > 1e-6
    np.testing.assert_allclose(r["x"], orc.solve(P, mk(tol=0.0, **dict(kw, max_iter=k)))["x"],
                               rtol=0, atol=0)


def test_paper_criterion_counts_equality_constraints(orc):
    """With p equality constraints the mean violation of §5.1 runs over the p + m scalar
    constraints: |Ax - b| for each equality, [g_i]_+ for each inequality.  Compared with numpy
    at early iterates of a capped solve, where both parts of the criterion are large."""
    inst = qi.paper_random_qcqp(40, 4, seed=5)
    rng = np.random.default_rng(11)
    A = rng.standard_normal((2, inst.n))
    b = A @ np.full(inst.n, 0.1)
    inst = dataclasses.replace(inst, p=2, A=A, b=b)
    P = orc.Problem(inst)
    L = np.linalg.norm(inst.Q[0], 2)
    fs = -1.0
    for k in (1, 3, 8):
        r = orc.solve(P, orc.Options(tau_bar=1 / L, gamma0=1.0, stop_rule="paper", f_star=fs, tol=0.0,
                                     max_iter=k))
        assert r["info"]["iters"] == k
        ref = _paper_criterion_numpy(inst.Q, inst.q, inst.c, r["x"], fs, A=A, b=b)
        assert abs(r["info"]["stop_value"] - ref) <= 1e-12 * max(1.0, ref), (k, r["info"]["stop_value"], ref)
