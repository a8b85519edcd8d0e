"""qcqp_eval_gap_noalloc (the G_xi evaluation whose scratch is a static device array, for
callers that cannot allocate) against qcqp_eval_gap on the same handle and point.

Both run the same kernels on the same inputs, so their results must be bitwise equal; the
allocating call is itself pinned to the oracle's G_xi (test_gpu_solve.py::test_gap_matches_oracle),
and both are checked against the oracle here too.  Two calls in a row share the device array:
the second, on a smaller handle, must not see the first call's contents.  Sizes past
QCQP_NOALLOC_MAX_N are refused.
"""
import numpy as np
import pytest

from tests.gpu_common import announce, oracle, qi

pytestmark = pytest.mark.gpu


def _solver(inst, **kw):
    from paper_2605_29291_amd import Solver
    return Solver(inst, **kw)


def _point(inst, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, inst.n), rng.uniform(0, 0.5, inst.m)


@pytest.mark.parametrize("device", [False, True])
def test_noalloc_gap_equals_allocating_gap(device):
    import torch
    cases = [(qi.random_qcqp(300, 8, seed=71, shift=0.01), 5),
             (qi.random_qcqp(120, 5, seed=72, shift=0.01), 6)]
    for inst, seed in cases:
        announce(f"noalloc gap n={inst.n} m={inst.m} device={device}")
        s = _solver(inst, tau_bar=1.0, device=device)
        x, y = _point(inst, seed)
        if device:
            xa, ya = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
        else:
            xa, ya = x, y
        got = s.eval_gap(xa, ya, xi=0.04, noalloc=True)
        ref = s.eval_gap(xa, ya, xi=0.04)
        again = s.eval_gap(xa, ya, xi=0.04, noalloc=True)
        s.close()
        assert got == ref == again, (got, ref, again)
        r = oracle.gap(oracle.Problem(inst), x, y, xi=0.04)
        assert abs(got["Py"] - r["Py"]) <= 1e-11 * (1 + abs(r["Py"]))
        assert abs(got["Px"] - r["Px"]) <= 1e-9 * (1 + abs(r["Px"]))


def test_noalloc_gap_at_the_size_limit_and_past_it():
    from paper_2605_29291_amd import QCQPError, abi
    nmax = abi.NOALLOC_MAX_N
    inst = qi.random_qcqp(nmax, 2, seed=73, shift=0.01)
    announce(f"noalloc gap n={nmax}")
    s = _solver(inst, tau_bar=1.0)
    x, y = _point(inst, 7)
    got = s.eval_gap(x, y, xi=0.04, noalloc=True)
    ref = s.eval_gap(x, y, xi=0.04)
    s.close()
    assert got == ref
    big = qi.random_qcqp(nmax + 1, 1, seed=74, shift=0.01)
    announce(f"noalloc gap refused at n={nmax + 1}")
    s = _solver(big, tau_bar=1.0)
    x, y = _point(big, 8)
    with pytest.raises(QCQPError) as e:
        s.eval_gap(x, y, xi=0.04, noalloc=True)
    assert e.value.code == abi.E_INVALID
    assert "QCQP_NOALLOC_MAX_N" in str(e.value)
    s.close()
