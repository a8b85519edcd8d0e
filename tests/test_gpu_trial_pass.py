"""Element-wise parity of the trial pass (qcqp_eval_trial_pass) against the FP64 oracle.

The trial pass is the kernel every backtracking trial streams: it is launched here exactly as the
solve launches it (same kernel, grid, tiles and candidate count B) on given points.

* 32/16-bit storage, incremental mode (the solve's default there): W_b = [Q_i d_b] for the steps
  d_b = x_b - x.  The kernel rounds d_b to FP32 once, each lane accumulates its share of a row
  with FP32 fused multiply-adds (at most k = ceil(n/8) + 8 products: a row is split over at least
  8 lanes, each reading whole 16-byte vectors), and the lanes' partial sums are combined in FP64.
  The stored values are exact in FP32, so with u = 2^-24 and gamma_k = k u / (1 - k u):
      |W_ir - (Q_i d)_r| <= (u + gamma_k + 2^-46) * S_ir,   S_ir = sum_j |Q_ij| |d_j|,
  whatever order the sums take (the last term covers the FP64 combine).  The oracle's (Q_i d)_r
  is the same sum in FP64 over the same stored values.
* FP64 storage, direct mode: [Q_i x_b] accumulated in FP64, checked at 1e-12 of S_ir; and FP64
  storage in incremental mode, W_b in FP64 at the same bar.
* The packed symmetric pass (sym_pass) with B = 1..4 candidates at n = 1100 (nine tile rows,
  so the per-row reduction of the column results runs over more than one group of eight).
* A candidate equal to the iterate gives W = 0 exactly.
"""
import math

import numpy as np
import pytest

from tests.gpu_common import abs_products, announce, oracle, qi, to_np

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _points(n, B, seed, lb=-10.0, ub=10.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.5 * lb, 0.5 * ub, n)
    xc = np.empty((B, n))
    for b in range(B):
        # steps of decreasing length, as the candidates tau eta^b give them
        xc[b] = np.clip(x + 0.7 ** b * 0.05 * rng.standard_normal(n), lb, ub)
    return x, xc


def _fp32_bound(n):
    k = math.ceil(n / 8) + 8
    return U32 + k * U32 / (1.0 - k * U32) + 2.0 ** -46


@pytest.mark.parametrize("storage", ["float32", "bfloat16", "float16"])
@pytest.mark.parametrize("n", [333, 4000])
def test_fp32_accumulated_trial_pass(storage, n):
    from paper_2605_29291_amd import Solver
    m = 3 if n == 4000 else 6
    B = 3
    inst = qi.round_instance(qi.random_qcqp(n, m, seed=5000 + n, shift=0.01), storage)
    announce(f"trial pass {storage} n={n} m={m} B={B}")
    s = Solver(inst, storage=storage, tau_bar=1.0, spec_trials=B)
    x, xc = _points(n, B, seed=n)
    xc[B - 1] = x                                   # a zero step
    W = to_np(s.eval_trial_pass(x, xc))
    s.close()
    P = oracle.Problem(inst)
    c = _fp32_bound(n)
    worst = 0.0
    for b in range(B):
        d = xc[b] - x
        ref = oracle.operator(P, d)["U"]
        if not d.any():
            np.testing.assert_array_equal(W[b], 0.0)
            continue
        S = abs_products(inst, d)
        err = np.abs(W[b] - ref)
        assert np.all(err <= c * S), (b, float(np.max(err / np.maximum(S, 1e-300))), c)
        worst = max(worst, float(np.max(err / np.maximum(S, 1e-300))))
    # the sums really run in FP32: some element carries FP32-level rounding
    assert worst > 1e-10, worst
    announce(f"  max |dW| / S = {worst:.2e} (bound {c:.2e})")


@pytest.mark.parametrize("mode", ["direct", "incremental"])
@pytest.mark.parametrize("B", [1, 2, 3, 4])
def test_fp64_trial_pass(mode, B):
    from paper_2605_29291_amd import Solver
    n, m = 517, 4
    inst = qi.random_qcqp(n, m, seed=5100 + B, shift=0.01)
    announce(f"trial pass float64 {mode} n={n} B={B}")
    s = Solver(inst, tau_bar=1.0, spec_trials=B, pass_mode=mode)
    x, xc = _points(n, B, seed=B)
    out = to_np(s.eval_trial_pass(x, xc))
    s.close()
    P = oracle.Problem(inst)
    for b in range(B):
        w = xc[b] if mode == "direct" else xc[b] - x
        ref = oracle.operator(P, w)["U"]
        S = abs_products(inst, w)
        assert np.all(np.abs(out[b] - ref) <= 1e-12 * S), (b, mode)


@pytest.mark.parametrize("B", [1, 2, 3, 4])
def test_packed_symmetric_trial_pass(B):
    from paper_2605_29291_amd import Solver
    n, m = 1100, 3
    inst = qi.random_qcqp(n, m, seed=5200 + B, shift=0.01)
    announce(f"packed trial pass n={n} B={B}")
    s = Solver(inst, tau_bar=1.0, spec_trials=B, sym_pass=1)
    x, xc = _points(n, B, seed=10 + B)
    out = to_np(s.eval_trial_pass(x, xc))
    s.close()
    P = oracle.Problem(inst)
    for b in range(B):
        ref = oracle.operator(P, xc[b])["U"]
        S = abs_products(inst, xc[b])
        assert np.all(np.abs(out[b] - ref) <= 1e-12 * S), b


def test_trial_pass_refuses_a_wrong_candidate_count():
    from paper_2605_29291_amd import Solver, abi
    inst = qi.random_qcqp(50, 2, seed=5300, shift=0.01)
    s = Solver(inst, tau_bar=1.0, spec_trials=2)
    x = np.zeros(50)
    xc = np.zeros((3, 50))
    out = np.empty((3, 3, 50))
    code = abi.load().qcqp_eval_trial_pass(s.handle, x.ctypes.data, xc.ctypes.data, 3,
                                           out.ctypes.data)
    assert code == abi.E_INVALID
    s.close()
