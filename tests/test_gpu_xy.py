"""GPU parity of APDB-xy (Algorithm 1: primal step first, momentum on grad_x Phi, the test
function E_k of eq. (backtracking)) inside rAPDB, against the FP64 oracle's xy routine.

* trajectory: K iterations with tol = 0 -- same iterate, multipliers and trial count as the
  oracle (same accept/reject decisions, rounding-level differences only);
* speculative candidates: spec_trials = 1..4 are bitwise the same sequential backtracking;
* final: relative KKT <= 1e-6 evaluated by the oracle, objective within 1e-6 (1 + |f|) of the
  oracle's own xy solve, for fixed (from the last iterate and from the average), no and
  adaptive restarts;
* precision: BF16 / FP16 / FP32 stored instances (incremental pass) reach the same bar;
* batching: xy and yx requests share one batch and each returns bitwise its alone result;
* parameter validation of Algorithm 1's c_alpha, c_beta, delta.
"""
import numpy as np
import pytest

from tests.gpu_common import announce, oracle, qi, tau_bar_of, to_np

pytestmark = pytest.mark.gpu

XY = dict(variant="xy", c_alpha=0.25, c_beta=0.3, delta=0.4)   # the §5 settings


def _gpu(tb, **kw):
    d = dict(tau_bar=tb, gamma0=0.1, **XY)
    d.update(kw)
    return d


def _orc(tb, **kw):
    return oracle.Options.xy(tau_bar=tb, gamma0=0.1, **kw)


def _solver(inst, **kw):
    from paper_2605_29291_amd import Solver
    return Solver(inst, **kw)


@pytest.mark.parametrize("K", [1, 5, 25])
def test_xy_trajectory_matches_oracle(K):
    inst = qi.random_qcqp(100, 10, qi.config_seed(1))
    tb = tau_bar_of(inst)
    announce(f"xy trajectory K={K}")
    s = _solver(inst, **_gpu(tb, max_iter=K, tol=0.0, spec_trials=1))
    x, y, info = s.solve()
    ref = oracle.solve(oracle.Problem(inst), _orc(tb, max_iter=K, tol=0.0))
    assert info["iters"] == K == ref["info"]["iters"]
    assert info["trials"] == ref["info"]["trials"]
    np.testing.assert_allclose(to_np(x), ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(y), ref["y"], rtol=1e-10, atol=1e-11)


def test_xy_trajectory_with_equalities_and_restarts():
    inst = qi.random_qcqp(64, 3, seed=12, shift=0.01, p=2)
    tb = tau_bar_of(inst)
    announce("xy trajectory p=2, restarts every 7")
    kw = dict(max_iter=30, tol=0.0, restart="fixed", restart_every=7)
    s = _solver(inst, **_gpu(tb, spec_trials=1, **kw))
    x, y, info = s.solve()
    ref = oracle.solve(oracle.Problem(inst), _orc(tb, **kw))
    assert info["iters"] == 30 == ref["info"]["iters"]
    assert info["trials"] == ref["info"]["trials"]
    assert info["restarts"] == ref["info"]["restarts"]
    np.testing.assert_allclose(to_np(x), ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(y), ref["y"], rtol=1e-10, atol=1e-11)


def test_xy_speculative_candidates_are_bitwise_sequential():
    inst = qi.random_qcqp(150, 12, seed=5, shift=0.01)
    tb = tau_bar_of(inst)
    res = []
    for B in (1, 2, 3, 4):
        announce(f"xy spec_trials={B}")
        s = _solver(inst, **_gpu(tb, max_iter=40, tol=0.0, spec_trials=B))
        x, y, info = s.solve()
        res.append((to_np(x), to_np(y), info))
        s.close()
    for x, y, info in res[1:]:
        np.testing.assert_array_equal(x, res[0][0])
        np.testing.assert_array_equal(y, res[0][1])
        assert info["trials"] == res[0][2]["trials"]
        assert info["q_passes"] <= res[0][2]["q_passes"]


@pytest.mark.parametrize("case", [
    dict(n=100, m=10, seed=qi.config_seed(1), shift=0.0, p=0),
    dict(n=257, m=20, seed=11, shift=0.01, p=0),
    dict(n=64, m=3, seed=12, shift=0.01, p=2),
    dict(n=513, m=0, seed=13, shift=0.01, p=0),
])
@pytest.mark.parametrize("restart", [dict(restart="fixed", restart_every=1000),
                                     dict(restart="fixed", restart_every=9),
                                     dict(restart="fixed", restart_every=9, restart_from_average=1),
                                     dict(restart="none", c_nm=0)])
def test_xy_final_solution_parity(case, restart):
    inst = qi.random_qcqp(case["n"], case["m"], case["seed"], shift=case["shift"], p=case["p"])
    tb = tau_bar_of(inst)
    announce(f"xy final {inst.name} {restart}")
    s = _solver(inst, **_gpu(tb, **restart))
    x, y, info = s.solve()
    assert info["status"] == "ok", info
    P = oracle.Problem(inst)
    kk = oracle.kkt(P, to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    ro = dict(restart)
    if "restart_from_average" in ro:
        ro["restart_from_average"] = bool(ro["restart_from_average"])
    ref = oracle.solve(P, _orc(tb, **ro))
    assert ref["info"]["status"] == "converged"
    f_ref = ref["info"]["f"]
    assert abs(kk["f"] - f_ref) <= 1e-6 * (1 + abs(f_ref))
    assert np.all(to_np(y)[inst.p:] >= 0)
    xs = to_np(x)
    assert np.all(xs >= inst.lb) and np.all(xs <= inst.ub)


def test_xy_adaptive_restart_solution():
    inst = qi.random_qcqp(120, 8, seed=21, shift=0.01)
    tb = tau_bar_of(inst)
    announce("xy adaptive restart")
    kw = dict(restart="adaptive", ada_first=5, ada_every=10, c_nm=0)
    s = _solver(inst, **_gpu(tb, **kw))
    x, y, info = s.solve()
    assert info["status"] == "ok", info
    assert info["gap_evals"] >= 1
    P = oracle.Problem(inst)
    kk = oracle.kkt(P, to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6
    ref = oracle.solve(P, _orc(tb, **kw))
    assert abs(kk["f"] - ref["info"]["f"]) <= 1e-6 * (1 + abs(ref["info"]["f"]))


@pytest.mark.parametrize("storage", ["float32", "bfloat16", "float16"])
def test_xy_rounded_instance_solution_parity(storage):
    inst = qi.round_instance(qi.random_qcqp(300, 20, seed=61, shift=0.01), storage)
    P = oracle.Problem(inst)
    tb = tau_bar_of(inst)
    announce(f"xy precision {storage}")
    s = _solver(inst, **_gpu(tb, storage=storage))
    x, y, info = s.solve()
    assert info["status"] == "ok", info
    kk = oracle.kkt(P, to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    assert abs(info["rel_kkt"] - kk["rel_kkt"]) <= 1e-9
    ref = oracle.solve(P, _orc(tb))
    assert abs(kk["f"] - ref["info"]["f"]) <= 1e-6 * (1 + abs(ref["info"]["f"]))


@pytest.mark.parametrize("storage", ["float64", "bfloat16"])
def test_xy_and_yx_share_a_batch_bitwise(storage):
    from paper_2605_29291_amd import Batch
    sizes = [(60, 3), (150, 12), (97, 7), (200, 1)]
    insts = []
    for k, (n, m) in enumerate(sizes):
        inst = qi.random_qcqp(n, m, seed=7000 + k, shift=0.0)
        if storage != "float64":
            inst = qi.round_instance(inst, storage)
        insts.append(inst)
    variants = ["xy", "yx", "xy", "yx"]

    def opts(k):
        kw = dict(tau_bar=tau_bar_of(insts[k]), gamma0=0.1, storage=storage, restart_every=30)
        if variants[k] == "xy":
            kw.update(XY)
        return kw

    alone = []
    for k, inst in enumerate(insts):
        announce(f"alone {variants[k]} {inst.name}")
        x, y, info = _solver(inst, **opts(k)).solve()
        alone.append((to_np(x), to_np(y), info))
    announce("mixed-variant batch")
    b = Batch(max_slots=4, storage=storage)
    slot_of = {}
    for k in (0, 1):
        slot_of[b.admit(_solver(insts[k], **opts(k)))] = k
    b.step(2)
    for k in (2, 3):
        slot_of[b.admit(_solver(insts[k], **opts(k)))] = k
    got = {}
    while len(got) < len(insts):
        b.step(4)
        for slot in b.poll():
            _, x, y, info = b.fetch(slot)
            got[slot_of[slot]] = (to_np(x), to_np(y), info)
    b.close()
    for k in range(len(insts)):
        x, y, info = got[k]
        np.testing.assert_array_equal(x, alone[k][0])
        np.testing.assert_array_equal(y, alone[k][1])
        assert info["iters"] == alone[k][2]["iters"] and info["trials"] == alone[k][2]["trials"]
        assert info["status"] == "ok"
        kk = oracle.kkt(oracle.Problem(insts[k]), x, y)
        assert kk["rel_kkt"] <= 1e-6


def test_xy_parameter_validation():
    from paper_2605_29291_amd import QCQPError
    inst = qi.random_qcqp(20, 2, seed=41, shift=0.01)
    for bad in (dict(c_beta=0.0), dict(c_alpha=0.0), dict(c_alpha=0.3, c_beta=0.3, delta=0.4),
                dict(delta=-0.1)):
        kw = _gpu(1.0)
        kw.update(bad)
        with pytest.raises(QCQPError) as e:
            _solver(inst, **kw)
        assert e.value.code == 1
