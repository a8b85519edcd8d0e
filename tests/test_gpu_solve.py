"""GPU parity of the device-resident rAPDB solve (qcqp_solve) against the FP64 oracle.

* trajectory: with max_iter = K and tol = 0 both sides take exactly K iterations; the GPU's
  iterate, trial count and multipliers must match the oracle's (same decisions; rounding-level
  differences only);
* speculative candidates: spec_trials = 1..4 give bitwise-identical iterates and trial counts
  (the candidates are the same sequential backtracking trials);
* final: the GPU solution reaches relative KKT <= 1e-6 as evaluated BY THE ORACLE, and its
  objective is within 1e-6 (1 + |f|) of the oracle's own solve;
* restarts: fixed (from the last iterate and from the average) and adaptive.
"""
import numpy as np
import pytest

from tests.gpu_common import announce, gpu_opts, oracle, oracle_opts, qi, tau_bar_of, to_np

pytestmark = pytest.mark.gpu


def _solver(inst, **kw):
    from paper_2605_29291_amd import Solver
    return Solver(inst, **kw)


@pytest.mark.parametrize("K", [1, 5, 25])
def test_trajectory_matches_oracle(K):
    inst = qi.random_qcqp(100, 10, qi.config_seed(1))
    tb = tau_bar_of(inst)
    announce(f"trajectory K={K}")
    s = _solver(inst, **gpu_opts(tb, max_iter=K, tol=0.0, spec_trials=1))
    x, y, info = s.solve()
    ref = oracle.solve(oracle.Problem(inst), oracle_opts(tb, max_iter=K, tol=0.0))
    assert info["iters"] == K == ref["info"]["iters"]
    assert info["trials"] == ref["info"]["trials"]
    np.testing.assert_allclose(to_np(x), ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(y), ref["y"], rtol=1e-10, atol=1e-11)


@pytest.mark.parametrize("variant", ["yx", "xy"])
@pytest.mark.parametrize("K", [1, 5, 25])
def test_trajectory_from_a_start_with_positive_multipliers(K, variant):
    """From a given (x^0, y^0) with lambda^0 > 0 and v^0 != 0 on an instance with two equality
    constraints: the first test functions then carry the epoch's starting alpha_0 (and beta_0)
    and A'v, which a start at y^0 = 0 leaves out.  Same iterates and trial counts as the oracle
    from the same start."""
    import dataclasses
    inst = qi.random_qcqp(100, 10, qi.config_seed(1))
    A = np.random.default_rng(13).standard_normal((2, inst.n))
    inst = dataclasses.replace(inst, p=2, A=A, b=A @ np.full(inst.n, 0.05))
    tb = tau_bar_of(inst)
    rng = np.random.default_rng(17)
    x0 = rng.uniform(-0.5, 0.5, inst.n)
    y0 = np.concatenate([rng.standard_normal(2), rng.uniform(0.1, 1.0, inst.m)])
    xy = dict(c_alpha=0.25, c_beta=0.3, delta=0.4) if variant == "xy" else {}
    announce(f"trajectory from (x0, y0) K={K} {variant}")
    s = _solver(inst, **gpu_opts(tb, max_iter=K, tol=0.0, spec_trials=2, variant=variant, **xy))
    x, y, info = s.solve(x0, y0)
    mk = oracle.Options.xy if variant == "xy" else oracle.Options
    ref = oracle.solve(oracle.Problem(inst), mk(tau_bar=tb, gamma0=0.1, max_iter=K, tol=0.0), x0=x0, y0=y0)
    assert info["iters"] == K == ref["info"]["iters"]
    assert info["trials"] == ref["info"]["trials"]
    np.testing.assert_allclose(to_np(x), ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(y), ref["y"][:inst.p + inst.m], rtol=1e-10, atol=1e-11)


def test_speculative_candidates_are_bitwise_sequential():
    inst = qi.random_qcqp(150, 12, seed=5, shift=0.01)
    tb = tau_bar_of(inst)
    res = []
    for B in (1, 2, 3, 4):
        announce(f"spec_trials={B}")
        s = _solver(inst, **gpu_opts(tb, max_iter=40, tol=0.0, spec_trials=B))
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
@pytest.mark.parametrize("restart", [dict(restart="fixed", restart_every=400),
                                     dict(restart="fixed", restart_every=9),
                                     dict(restart="fixed", restart_every=9, restart_from_average=1),
                                     dict(restart="none", c_nm=0)])
def test_final_solution_parity(case, restart):
    inst = qi.random_qcqp(case["n"], case["m"], case["seed"], shift=case["shift"], p=case["p"])
    tb = tau_bar_of(inst)
    announce(f"final {inst.name} {restart}")
    s = _solver(inst, **gpu_opts(tb, **restart))
    x, y, info = s.solve()
    assert info["status"] == "ok", info
    P = oracle.Problem(inst)
    kk = oracle.kkt(P, to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    ro = dict(restart)
    if "restart_from_average" in ro:
        ro["restart_from_average"] = bool(ro["restart_from_average"])
    ref = oracle.solve(P, oracle_opts(tb, **ro))
    assert ref["info"]["status"] == "converged"
    f_ref = ref["info"]["f"]
    assert abs(kk["f"] - f_ref) <= 1e-6 * (1 + abs(f_ref))
    # multipliers are feasible exactly (projection onto R^m_+)
    assert np.all(to_np(y)[inst.p:] >= 0)
    xs = to_np(x)
    assert np.all(xs >= inst.lb) and np.all(xs <= inst.ub)


def test_adaptive_restart_solution():
    inst = qi.random_qcqp(120, 8, seed=21, shift=0.01)
    tb = tau_bar_of(inst)
    announce("adaptive restart")
    kw = dict(restart="adaptive", ada_first=5, ada_every=10, c_nm=0)
    s = _solver(inst, **gpu_opts(tb, **kw))
    x, y, info = s.solve()
    assert info["status"] == "ok", info
    assert info["gap_evals"] >= 1
    P = oracle.Problem(inst)
    kk = oracle.kkt(P, to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6
    ref = oracle.solve(P, oracle_opts(tb, **kw))
    assert abs(kk["f"] - ref["info"]["f"]) <= 1e-6 * (1 + abs(ref["info"]["f"]))


def test_gap_matches_oracle():
    inst = qi.random_qcqp(90, 6, seed=31, shift=0.01)
    P = oracle.Problem(inst)
    s = _solver(inst, tau_bar=1.0)
    rng = np.random.default_rng(3)
    for trial in range(3):
        x = rng.uniform(-1, 1, inst.n)
        y = rng.uniform(0, 0.5, inst.m)
        announce(f"gap point {trial}")
        g = s.eval_gap(x, y, xi=0.04)
        r = oracle.gap(P, x, y, xi=0.04)
        assert abs(g["Py"] - r["Py"]) <= 1e-11 * (1 + abs(r["Py"]))
        assert abs(g["Px"] - r["Px"]) <= 1e-9 * (1 + abs(r["Px"]))
        assert g["G"] >= 0


def test_edge_cases_and_errors():
    from paper_2605_29291_amd import QCQPError
    inst = qi.random_qcqp(20, 2, seed=41, shift=0.01)
    bad = qi.random_qcqp(20, 2, seed=41, shift=0.01)
    bad.lb = bad.lb.copy()
    bad.lb[3] = 11.0
    with pytest.raises(QCQPError) as e:
        _solver(bad, tau_bar=1.0)
    assert e.value.code == 1
    bad2 = qi.random_qcqp(20, 2, seed=41, shift=0.01)
    bad2.q = bad2.q.copy()
    bad2.q[1, 4] = np.nan
    with pytest.raises(QCQPError):
        _solver(bad2, tau_bar=1.0)
    with pytest.raises(QCQPError):
        _solver(inst, tau_bar=1.0, eta=1.5)
    with pytest.raises(QCQPError):
        _solver(inst, tau_bar=1.0, c_alpha=0.6, delta=0.5)
    # max_iter = 0 returns the projected start, not converged
    s = _solver(inst, tau_bar=tau_bar_of(inst), max_iter=0)
    x, y, info = s.solve(x0=np.full(20, 50.0))
    assert info["status"] == "not_converged" and info["iters"] == 0
    np.testing.assert_array_equal(to_np(x), np.full(20, 10.0))
    # n = 1 box QP
    one = qi.Instance(1, 0, 0, np.array([[[1.0]]]), np.array([[-20.0]]), np.zeros(1),
                      np.array([-10.0]), np.array([10.0]))
    s1 = _solver(one, tau_bar=1.0)
    x1, _, info1 = s1.solve()
    assert info1["status"] == "ok" and abs(to_np(x1)[0] - 10.0) < 1e-9


def test_graph_replays_match_eager_launches():
    """Chunks of trial groups replayed from a captured HIP graph give bitwise the eager result,
    on every replay, with eager work and synchronisations between the replays."""
    import torch
    from paper_2605_29291_amd import Batch, Solver
    inst = qi.random_qcqp(180, 9, seed=71, shift=0.01)
    tb = tau_bar_of(inst)
    eager = _solver(inst, **gpu_opts(tb, use_graphs=0, poll_every=8))
    xe, ye, ie = eager.solve()
    xe, ye = to_np(xe), to_np(ye)
    g = _solver(inst, **gpu_opts(tb, use_graphs=1, poll_every=8))
    rng = np.random.default_rng(0)
    for rep in range(3):
        announce(f"graph replay {rep}")
        x, y, info = g.solve()
        np.testing.assert_array_equal(to_np(x), xe)
        np.testing.assert_array_equal(to_np(y), ye)
        assert info["trials"] == ie["trials"] and info["q_passes"] == ie["q_passes"]
        g.eval_operator(rng.uniform(-1, 1, inst.n))          # eager work between replays
        torch.cuda.synchronize()
    # batch: graph-captured steps against eager steps
    res = []
    for use in (0, 1):
        b = Batch(max_slots=4, use_graphs=use)
        s = _solver(inst, **gpu_opts(tb))
        slot = b.admit(s)
        while not b.poll():
            b.step(3)
        _, x, y, info = b.fetch(slot)
        res.append((to_np(x), info["trials"]))
        b.close()
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][0], xe)


@pytest.mark.parametrize("sym", [0, 1])
def test_timing_mode_matches_and_times_every_pass(sym):
    """options.timing records HIP events around every pass of pipelined chunks (two event sets,
    read once a chunk's status snapshot is back): the same iterates as without timing, and
    every streamed pass timed, over several chunks and through a fixed restart."""
    inst = qi.random_qcqp(300, 8, seed=51, shift=0.01)
    tb = tau_bar_of(inst)
    kw = gpu_opts(tb, spec_trials=3, sym_pass=sym, poll_every=3, restart_every=20)
    announce(f"timing mode sym={sym}")
    x0, y0, i0 = _solver(inst, **kw).solve()
    x1, y1, i1 = _solver(inst, timing=1, **kw).solve()
    np.testing.assert_array_equal(to_np(x1), to_np(x0))
    np.testing.assert_array_equal(to_np(y1), to_np(y0))
    assert i1["status"] == "ok" and i1["q_passes"] == i0["q_passes"] and i1["restarts"] >= 1
    assert i1["timed_passes"] == i1["q_passes"]
    assert i1["pass_seconds"] > 0.0
