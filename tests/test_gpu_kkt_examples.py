"""The relative KKT residual of qcqp_eval_kkt on two one-variable instances worked by hand (the
same instances pin the oracle's residual in test_oracle_steps.py and test_oracle_cones.py):
every normalisation term nonzero and distinct, an equality constraint, a second-order cone and
constraints without a stored matrix.  The GPU's six outputs, the largest violation included,
equal the hand values and the oracle's."""
import numpy as np
import pytest

from tests.gpu_common import announce, oracle, qi

pytestmark = pytest.mark.gpu

KEYS = ("rel_kkt", "rel_dual", "rel_pri", "rel_comp", "f", "max_violation")


def _check(inst, x, y, expected):
    from paper_2605_29291_amd import Solver
    announce(f"KKT worked example {inst.name}")
    s = Solver(inst, tau_bar=1.0)
    got = s.eval_kkt(x, y)
    s.close()
    ref = oracle.kkt(oracle.Problem(inst), x, y)
    for k in KEYS:
        assert got[k] == pytest.approx(expected[k], rel=1e-14, abs=0.0), (k, got[k], expected[k])
        assert got[k] == pytest.approx(ref[k], rel=1e-14, abs=0.0), (k, got[k], ref[k])


def test_orthant_and_equality_worked_example():
    """Q_0 = 2, q_0 = 0; Q_1 = 4, q_1 = 1, c_1 = -2; A = 2, b = 0.5; X = [-10, 10]; at x = 0.5,
    v = 0.5, lambda = 3: rel_dual = 10.5 / 12, rel_comp = 1/3, rel_pri = 1/7, f = 0.25, largest
    violation |Ax - b| = 0.5.  The library needs p < n, so the instance carries a second
    variable whose data are all zero (x_2 = 0): it adds nothing to any norm or residual."""
    Q = np.zeros((2, 2, 2))
    Q[0, 0, 0], Q[1, 0, 0] = 2.0, 4.0
    inst = qi.Instance(2, 1, 1, Q, np.array([[0.0, 0.0], [1.0, 0.0]]), np.array([0.0, -2.0]),
                       np.full(2, -10.0), np.full(2, 10.0), np.array([[2.0, 0.0]]), np.array([0.5]), True,
                       "kkt_orthant_2var")
    _check(inst, np.array([0.5, 0.0]), np.array([0.5, 3.0]),
           dict(rel_kkt=0.875, rel_dual=0.875, rel_pri=1.0 / 7.0, rel_comp=1.0 / 3.0, f=0.25, max_violation=0.5))


def test_cone_worked_example():
    """Only Q_0 = 2 stored; g = (0.5, (1, 3)) in -(R_+ x Q^2) at x = 1, lambda = 0: the cone block
    projects to (2, 2), so dist(g, -K) = sqrt(8.25), the largest violation is 2 sqrt(2),
    rel_pri = rel_comp = sqrt(8.25) / (1 + sqrt(10.25)), rel_dual = 2/3, f = 1."""
    stored = np.array([1, 0, 0, 0], dtype=np.int32)
    inst = qi.Instance(1, 3, 0, np.array([[[2.0]]]), np.zeros((4, 1)), np.array([0.0, 0.5, 1.0, 3.0]),
                       np.array([-10.0]), np.array([10.0]), None, None, True, "kkt_cone_1d",
                       lambda_set="cones", q_stored=stored, soc_dims=[2])
    r = np.sqrt(8.25) / (1.0 + np.sqrt(10.25))
    _check(inst, np.array([1.0]), np.zeros(3),
           dict(rel_kkt=r, rel_dual=2.0 / 3.0, rel_pri=r, rel_comp=r, f=1.0, max_violation=2.0 * np.sqrt(2.0)))
