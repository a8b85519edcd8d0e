"""GPU parity of the dual domains and the objective's identity part against the FP64 oracle.

* the restricted dual domain Y-hat = Y ∩ B of problem (R-min-max) (§3.2): joint ball ||y|| <= B
  and the separable balls ||v|| <= B_v, ||lambda|| <= B_lambda -- trajectories (same iterates and
  trial counts as the oracle while the ball binds) for APDB-yx and APDB-xy, and the closed-form
  restricted saddle points the oracle is pinned to;
* lambda on the unit simplex (the kernel-learning min-max form of §5), with the identity part
  rho I of the objective's Hessian and mu = rho: trajectories, final solutions (relative KKT
  <= 1e-6 by the oracle's natural residual, x within 1e-6 of the oracle's solution, which is
  unique by strong convexity), and the paper's kernel-learning min-max instance;
* rho I in the operator, with and without a stored Q_0, FP64 and BF16 storage.
"""
import numpy as np
import pytest

from tests.gpu_common import announce, oracle, qi, tau_bar_of, to_np

pytestmark = pytest.mark.gpu

XY = dict(variant="xy", c_alpha=0.25, c_beta=0.3, delta=0.4)


def _solver(inst, **kw):
    from paper_2605_29291_amd import Solver
    return Solver(inst, **kw)


def _orc_opts(variant, **kw):
    return (oracle.Options.xy if variant == "xy" else oracle.Options)(**kw)


def _gpu_kw(variant, **kw):
    d = dict(kw)
    if variant == "xy":
        d.update(XY)
    return d


BALLS = [dict(ball=0.6), dict(ball_v=0.3, ball_lambda=0.5), dict(ball_lambda=0.4)]


@pytest.mark.parametrize("variant", ["yx", "xy"])
@pytest.mark.parametrize("ball", BALLS, ids=lambda b: "-".join(f"{k}{v}" for k, v in b.items()))
def test_ball_trajectory_matches_oracle(variant, ball):
    inst = qi.random_qcqp(90, 8, seed=101, shift=0.01, p=2)
    tb = tau_bar_of(inst)
    K = 40
    okw = {("ball_l" if k == "ball_lambda" else k): v for k, v in ball.items()}
    P = oracle.Problem(inst, **okw)
    ref = oracle.solve(P, _orc_opts(variant, tau_bar=tb, gamma0=0.1, max_iter=K, tol=0.0))
    # the ball binds at the end of the reference trajectory
    y = ref["y"]
    binds = [abs(np.linalg.norm(y) - ball["ball"]) < 1e-9] if "ball" in ball else []
    if "ball_v" in ball:
        binds.append(abs(np.linalg.norm(y[:2]) - ball["ball_v"]) < 1e-9)
    if "ball_lambda" in ball:
        binds.append(abs(np.linalg.norm(y[2:]) - ball["ball_lambda"]) < 1e-9)
    assert any(binds), (np.linalg.norm(y[:2]), np.linalg.norm(y[2:]))
    announce(f"ball trajectory {variant} {ball}")
    s = _solver(inst, **ball, **_gpu_kw(variant, tau_bar=tb, gamma0=0.1, max_iter=K, tol=0.0,
                                        spec_trials=2))
    x, yg, info = s.solve()
    assert info["iters"] == K and info["trials"] == ref["info"]["trials"]
    np.testing.assert_allclose(to_np(x), ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(yg), ref["y"], rtol=1e-10, atol=1e-11)


def test_small_balls_give_the_closed_form_saddle_points():
    rng = np.random.default_rng(21)
    n = 6
    A = rng.standard_normal((n, n))
    Q0 = A @ A.T / n + 0.5 * np.eye(n)
    q0 = rng.standard_normal(n) * 3.0
    Q = np.stack([Q0, np.eye(n)])
    q = np.stack([q0, np.zeros(n)])
    c = np.array([0.0, -0.5])
    from tests import pins
    _, lam_star = pins.ball_qp_bisection(Q0, q0, 0.5)
    B = 0.5 * lam_star
    xB = -np.linalg.solve(Q0 + B * np.eye(n), q0)
    inst = qi.Instance(n, 1, 0, Q, q, c, -10 * np.ones(n), 10 * np.ones(n))
    for kw in (dict(ball=B), dict(ball_lambda=B)):
        announce(f"closed-form ball {kw}")
        s = _solver(inst, tau_bar=1.0 / np.linalg.norm(Q0, 2), tol=0.0, max_iter=6000, **kw)
        x, y, _ = s.solve()
        np.testing.assert_allclose(to_np(x), xB, atol=1e-8)
        assert abs(to_np(y)[0] - B) <= 1e-9
        g = s.eval_gap(x, y)
        assert abs(g["G"]) <= 1e-11
    # the v-ball on a single equality constraint
    a = rng.standard_normal(n)
    beta = 2.0
    Qi = np.linalg.inv(Q0)
    v_star = -(beta + a @ Qi @ q0) / (a @ Qi @ a)
    Bv = 0.5 * abs(v_star)
    v = np.sign(v_star) * Bv
    xv = -Qi @ (q0 + v * a)
    inst2 = qi.Instance(n, 0, 1, Q0[None], q0[None], np.zeros(1), -10 * np.ones(n),
                        10 * np.ones(n), a[None], np.array([beta]))
    announce("closed-form v-ball")
    x, y, _ = _solver(inst2, tau_bar=1.0 / np.linalg.norm(Q0, 2), tol=0.0, max_iter=6000,
                      ball_v=Bv).solve()
    np.testing.assert_allclose(to_np(x), xv, atol=1e-8)
    assert abs(to_np(y)[0] - v) <= 1e-9


def _simplex_inst(n, m, seed, p=1, rho=1.0):
    rng = np.random.default_rng(seed)
    Q = []
    for _ in range(m):
        A = rng.standard_normal((n, n))
        Q.append(A @ A.T / n)
    Q = np.stack(Q)
    q = rng.standard_normal((m + 1, n))
    c = rng.uniform(-1, 1, m + 1)
    A = rng.standard_normal((p, n)) if p else None
    b = rng.standard_normal(p) if p else None
    return qi.Instance(n, m, p, Q, q, c, -5 * np.ones(n), 5 * np.ones(n), A, b, False,
                       f"simplex_n{n}_m{m}", lambda_set="simplex", q0_shift=rho)


@pytest.mark.parametrize("variant", ["yx", "xy"])
def test_simplex_trajectory_matches_oracle(variant):
    inst = _simplex_inst(120, 6, seed=7)
    K = 40
    announce(f"simplex trajectory {variant}")
    kw = dict(tau_bar=0.5, gamma0=0.1, mu=1.0, max_iter=K, tol=0.0)
    ref = oracle.solve(oracle.Problem(inst), _orc_opts(variant, **kw))
    x, y, info = _solver(inst, **_gpu_kw(variant, spec_trials=2, **kw)).solve()
    assert info["iters"] == K and info["trials"] == ref["info"]["trials"]
    np.testing.assert_allclose(to_np(x), ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(y), ref["y"], rtol=1e-10, atol=1e-11)
    assert abs(to_np(y)[1:].sum() - 1.0) <= 1e-13


@pytest.mark.parametrize("variant", ["yx", "xy"])
@pytest.mark.parametrize("storage", ["float64", "bfloat16"])
def test_simplex_final_solution(variant, storage):
    inst = _simplex_inst(200, 5, seed=8)
    if storage != "float64":
        inst = qi.round_instance(inst, storage)
    announce(f"simplex final {variant} {storage}")
    kw = dict(tau_bar=0.5, gamma0=0.1, mu=1.0)
    x, y, info = _solver(inst, storage=storage, **_gpu_kw(variant, **kw)).solve()
    assert info["status"] == "ok", info
    P = oracle.Problem(inst)
    kk = oracle.kkt(P, to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    assert abs(info["rel_kkt"] - kk["rel_kkt"]) <= 1e-9
    ref = oracle.solve(P, _orc_opts(variant, tol=1e-9, **kw))
    assert ref["info"]["status"] == "converged"
    np.testing.assert_allclose(to_np(x), ref["x"], atol=1e-5)


def test_kml_minmax_workload_small():
    inst = qi.kml_minmax(300, seed=qi.config_seed(4))
    announce("kml min-max n=300")
    kw = dict(tau_bar=0.5, gamma0=0.1, mu=2.0, restart_every=200)
    s = _solver(inst, **kw)
    x, y, info = s.solve()
    assert info["status"] == "ok", info
    P = oracle.Problem(inst)
    kk = oracle.kkt(P, to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    ref = oracle.solve(P, oracle.Options(tol=1e-9, max_iter=100000, **kw))
    assert ref["info"]["status"] == "converged"
    xs = to_np(x)
    assert np.all(xs >= 0)
    assert np.linalg.norm(xs - ref["x"]) / (1 + np.linalg.norm(ref["x"])) <= 1e-5
    np.testing.assert_allclose(to_np(y)[1:], ref["y"][1:], atol=1e-5)


@pytest.mark.parametrize("has_q0", [True, False])
@pytest.mark.parametrize("storage", ["float64", "bfloat16"])
@pytest.mark.parametrize("sym", [0, 1])
def test_q0_shift_operator_parity(has_q0, storage, sym):
    base = qi.random_qcqp(150, 6, seed=9, shift=0.01)
    Q = base.Q if has_q0 else base.Q[1:]
    inst = qi.Instance(150, 6, 0, Q, base.q, base.c, base.lb, base.ub, None, None, has_q0,
                       "shift", q0_shift=1.7)
    if storage != "float64":
        inst = qi.round_instance(inst, storage)
    announce(f"q0 shift operator has_q0={has_q0} {storage} sym_pass={sym}")
    s = _solver(inst, tau_bar=1.0, storage=storage, sym_pass=sym)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, 150)
    y = rng.uniform(0, 1, 6)
    out = s.eval_operator(x, y)
    ref = oracle.operator(oracle.Problem(inst), x, y)
    U = to_np(out["U"])
    scale = np.max(np.abs(ref["U"]))
    assert np.max(np.abs(U - ref["U"])) <= 1e-12 * scale
    np.testing.assert_allclose(to_np(out["g"]), ref["G"], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(to_np(out["grad"]), ref["grad"], rtol=1e-11,
                               atol=1e-12 * np.max(np.abs(ref["grad"])))
    assert abs(out["f"] - ref["f"]) <= 1e-12 * (1 + abs(ref["f"]))
    # and a solve reaches the oracle's optimum
    x, y, info = s.solve()
    assert info["status"] == "ok", info
    kk = oracle.kkt(oracle.Problem(inst), to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6


def test_dual_domain_validation():
    from paper_2605_29291_amd import QCQPError
    inst = qi.random_qcqp(20, 2, seed=41, shift=0.01)
    for kw in (dict(ball=1.0, ball_v=1.0), dict(ball=-1.0), dict(q0_shift=-1.0),
               dict(lambda_set="simplex", ball=1.0), dict(lambda_set="simplex", ball_lambda=1.0)):
        with pytest.raises(QCQPError) as e:
            _solver(inst, tau_bar=1.0, **kw)
        assert e.value.code == 1, kw
    bad = qi.random_qcqp(20, 0, seed=41, shift=0.01)
    with pytest.raises(QCQPError):
        _solver(bad, tau_bar=1.0, lambda_set="simplex")


@pytest.mark.parametrize("case", ["equality", "ball", "separable_balls", "simplex", "cones"])
def test_gap_matches_oracle_over_dual_domains(case):
    """G_xi (Definition in §4, Remark in §4.2) at given points for each dual domain: the y-part
    projects onto R^p x K* (orthant, simplex, cones) intersected with the requested ball, and
    the x-part's Hessian carries the identity part of the objective (simplex case, rho = 1).
    Py and Px equal the oracle's at the bars of the lambda >= 0 case."""
    from paper_2605_29291_amd import Solver
    kw_gpu, kw_orc = {}, {}
    if case == "simplex":
        inst = _simplex_inst(80, 5, seed=31)
    elif case == "cones":
        inst = qi.random_conic_qcqp(80, 2, [3, 4], seed=37, p=1)
    else:
        inst = qi.random_qcqp(80, 5, seed=29, shift=0.01, p=2)
        if case == "ball":
            kw_gpu = kw_orc = dict(ball=1.5)
        elif case == "separable_balls":
            kw_gpu, kw_orc = dict(ball_v=0.7, ball_lambda=0.9), dict(ball_v=0.7, ball_l=0.9)
    P = oracle.Problem(inst, **kw_orc)
    s = _solver(inst, tau_bar=1.0, **kw_gpu)
    rng = np.random.default_rng(23)
    for trial in range(2):
        x = rng.uniform(-1, 1, inst.n)
        y = np.concatenate([rng.standard_normal(inst.p), rng.uniform(0, 0.5, inst.m)])
        announce(f"G_xi over the {case} domain, point {trial}")
        g = s.eval_gap(x, y, xi=0.04)
        r = oracle.gap(P, x, y, xi=0.04)
        assert abs(g["Py"] - r["Py"]) <= 1e-11 * (1 + abs(r["Py"])), (g, r)
        assert abs(g["Px"] - r["Px"]) <= 1e-9 * (1 + abs(r["Px"])), (g, r)
        assert g["G"] == pytest.approx(g["Py"] + g["Px"], rel=1e-15, abs=1e-300)
    s.close()


def test_simplex_and_ball_requests_share_a_batch_bitwise():
    """A simplex min-max request (identity part, mu = 1), a request whose joint ball binds, one
    with separable balls and an equality constraint, and a plain QCQP run in one batch and
    return bitwise the same iterates, multipliers and counters as when each runs alone.  The
    requests without a binding ball also reach the oracle-evaluated KKT of 1e-6 (a binding ball
    restricts the dual, so its request runs to its iteration cap)."""
    from paper_2605_29291_amd import Batch
    simplex = _simplex_inst(120, 6, seed=62)
    plain = qi.random_qcqp(110, 5, seed=64, shift=0.01)
    items = [(simplex, dict(tau_bar=0.5, gamma0=0.1, mu=1.0), True),
             (qi.random_qcqp(90, 6, seed=61, shift=0.01), dict(ball=0.05, max_iter=300), False),
             (qi.random_qcqp(70, 4, seed=63, shift=0.01, p=1), dict(ball_v=0.5, ball_lambda=1.0, max_iter=300),
              False),
             (plain, {}, True)]
    kws = [dict(dict(tau_bar=tau_bar_of(inst), gamma0=0.1), **kw) for inst, kw, _ in items]
    alone = []
    for (inst, _, _), kw in zip(items, kws):
        announce(f"alone {inst.name} {kw}")
        x, y, info = _solver(inst, **kw).solve()
        alone.append((to_np(x), to_np(y), info))
    announce("mix of simplex, ball and plain requests")
    b = Batch(max_slots=4)
    slot_of = {b.admit(_solver(items[k][0], **kws[k])): k for k in (0, 3)}
    b.step(2)
    for k in (1, 2):
        slot_of[b.admit(_solver(items[k][0], **kws[k]))] = k
    got = {}
    guard = 0
    while len(got) < len(items):
        b.step(4)
        for slot in b.poll():
            _, x, y, info = b.fetch(slot)
            got[slot_of[slot]] = (to_np(x), to_np(y), info)
        guard += 1
        assert guard < 10000
    b.close()
    for k, (inst, _, converges) in enumerate(items):
        np.testing.assert_array_equal(got[k][0], alone[k][0], err_msg=inst.name)
        np.testing.assert_array_equal(got[k][1], alone[k][1], err_msg=inst.name)
        for key in ("iters", "trials", "status"):
            assert got[k][2][key] == alone[k][2][key], (inst.name, key)
        if converges:
            assert got[k][2]["status"] == "ok"
            kk = oracle.kkt(oracle.Problem(inst), got[k][0], got[k][1])
            assert kk["rel_kkt"] <= 1e-6, (inst.name, kk)
