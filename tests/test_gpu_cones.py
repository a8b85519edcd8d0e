"""GPU parity of conic constraints g(x) in -K, K = R^{m0}_+ x Q^{k_1} x ... (second-order cones, the
cone setting of §2.1), and of constraints without a stored matrix, against the FP64 oracle.

* trajectories (same iterates and trial counts as the oracle) for APDB-yx and APDB-xy, with an
  equality constraint, a joint dual ball, and cones of one, small and large (block-projected)
  dimension;
* final solutions (relative KKT with the cone residuals <= 1e-6 by the oracle, x within 1e-5 of
  the oracle's solution), FP64 and BF16 storage;
* min 1/2 ||x - a||^2 over x in Q^n with every constraint affine (only Q_0 stored): x = Pi_Q(a)
  for n = 6 (one thread per cone) and n = 300 (the whole block projects the cone);
* a stored zero matrix and an absent one: bitwise the same trajectory; a conic request and a
  plain QCQP share one batch bitwise as when alone.
"""
import numpy as np
import pytest

from tests.gpu_common import announce, oracle, qi, to_np

pytestmark = pytest.mark.gpu

XY = dict(variant="xy", c_alpha=0.25, c_beta=0.3, delta=0.4)


def _solver(inst, **kw):
    from paper_2605_29291_amd import Solver
    return Solver(inst, **kw)


def _mk(variant):
    return oracle.Options.xy if variant == "xy" else oracle.Options


def _proj_soc(z):
    t, u = z[0], z[1:]
    un = np.linalg.norm(u)
    if un <= t:
        return z.copy()
    if un <= -t:
        return np.zeros_like(z)
    a = 0.5 * (t + un)
    return np.concatenate([[a], u * (a / un)])


CASES = [dict(m_lin=3, dims=[4, 1, 6], p=1, ball=0.0),
         dict(m_lin=0, dims=[150], p=0, ball=0.0),
         dict(m_lin=2, dims=[3, 3], p=0, ball=0.4)]


@pytest.mark.parametrize("variant", ["yx", "xy"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"m{c['m_lin']}-k{c['dims']}-ball{c['ball']}")
def test_conic_trajectory_matches_oracle(variant, case):
    inst = qi.random_conic_qcqp(160, case["m_lin"], case["dims"], seed=11, p=case["p"])
    tb = 1.0 / np.linalg.norm(inst.Q[0], 2)
    K = 40
    kw = dict(tau_bar=tb, gamma0=1.0, max_iter=K, tol=0.0)
    announce(f"conic trajectory {variant} {case}")
    ref = oracle.solve(oracle.Problem(inst, ball=case["ball"]), _mk(variant)(**kw))
    gkw = dict(kw, spec_trials=2, ball=case["ball"])
    if variant == "xy":
        gkw.update(XY)
    x, y, info = _solver(inst, **gkw).solve()
    assert info["iters"] == K and info["trials"] == ref["info"]["trials"]
    np.testing.assert_allclose(to_np(x), ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(y), ref["y"], rtol=1e-10, atol=1e-11)


@pytest.mark.parametrize("variant", ["yx", "xy"])
@pytest.mark.parametrize("storage", ["float64", "bfloat16"])
def test_conic_final_solution(variant, storage):
    inst = qi.random_conic_qcqp(200, 3, [4, 1, 6], seed=12, p=1)
    tb = 1.0 / np.linalg.norm(inst.Q[0], 2)
    if storage != "float64":
        inst = qi.round_instance(inst, storage)
    P = oracle.Problem(inst)
    announce(f"conic final {variant} {storage}")
    gkw = dict(tau_bar=tb, gamma0=1.0, storage=storage)
    if variant == "xy":
        gkw.update(XY)
    x, y, info = _solver(inst, **gkw).solve()
    assert info["status"] == "ok", info
    kk = oracle.kkt(P, to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    assert abs(info["rel_kkt"] - kk["rel_kkt"]) <= 1e-9
    ref = oracle.solve(P, _mk(variant)(tau_bar=tb, gamma0=1.0, tol=1e-9, max_iter=200000))
    assert ref["info"]["status"] == "converged"
    np.testing.assert_allclose(to_np(x), ref["x"], atol=1e-5)
    # multipliers lie in K* = K
    lam = to_np(y)[inst.p:]
    assert np.all(lam[:3] >= 0)
    off = 3
    for k in (4, 1, 6):
        assert np.linalg.norm(lam[off + 1:off + k]) <= lam[off] * (1 + 1e-12) + 1e-15
        off += k


@pytest.mark.parametrize("n", [6, 300])
def test_affine_cone_constraint_gives_the_cone_projection(n):
    rng = np.random.default_rng(5)
    a = rng.standard_normal(n)
    a[0] = -0.3
    x_ref = _proj_soc(a)
    q = np.zeros((n + 1, n))
    q[0] = -a
    q[1, 0] = -1.0
    for j in range(1, n):
        q[1 + j, j] = 1.0
    stored = np.zeros(n + 1, dtype=np.int32)
    stored[0] = 1
    inst = qi.Instance(n, n, 0, np.eye(n)[None], q, np.zeros(n + 1), -10 * np.ones(n),
                       10 * np.ones(n), None, None, True, f"socproj{n}", lambda_set="cones",
                       q_stored=stored, soc_dims=[n])
    announce(f"cone projection problem n={n}")
    x, y, info = _solver(inst, tau_bar=1.0, gamma0=1.0, tol=1e-10, max_iter=200000).solve()
    assert info["status"] == "ok", info
    np.testing.assert_allclose(to_np(x), x_ref, atol=1e-7)
    lam = to_np(y)
    assert np.linalg.norm(lam[1:]) <= lam[0] * (1 + 1e-12)


def test_stored_zero_matrix_and_absent_matrix_agree_bitwise():
    inst = qi.random_qcqp(150, 5, seed=13, shift=0.01)
    Q = np.array(inst.Q)
    Q[2] = 0.0
    Q[4] = 0.0
    tb = 1.0 / np.linalg.norm(Q[0], 2)
    dense = qi.Instance(150, 5, 0, Q, inst.q, inst.c, inst.lb, inst.ub)
    stored = np.array([1, 1, 0, 1, 0, 1], dtype=np.int32)
    sparse = qi.Instance(150, 5, 0, Q[stored == 1], inst.q, inst.c, inst.lb, inst.ub,
                         q_stored=stored)
    res = []
    for name, ii in (("dense", dense), ("sparse", sparse)):
        announce(f"stored map {name}")
        s = _solver(ii, tau_bar=tb, max_iter=50, tol=0.0)
        x, y, info = s.solve()
        res.append((to_np(x), to_np(y), info, s.nbytes()))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][1], res[1][1])
    assert res[0][2]["trials"] == res[1][2]["trials"]
    assert res[1][2]["pass_bytes"] * 6 == res[0][2]["pass_bytes"] * 4   # 4 of 6 matrices streamed
    assert res[1][3] < res[0][3]
    ref = oracle.solve(oracle.Problem(sparse), oracle.Options(tau_bar=tb, max_iter=50, tol=0.0))
    np.testing.assert_allclose(res[1][0], ref["x"], rtol=1e-10, atol=1e-11)


def test_conic_and_plain_requests_share_a_batch_bitwise():
    from paper_2605_29291_amd import Batch
    insts = [qi.random_conic_qcqp(120, 2, [3, 5], seed=14),
             qi.random_qcqp(90, 6, seed=15, shift=0.01),
             qi.random_conic_qcqp(70, 0, [200], seed=16)]
    kws = [dict(tau_bar=1.0 / np.linalg.norm(np.asarray(i.Q)[0], 2), gamma0=1.0) for i in insts]
    alone = []
    for inst, kw in zip(insts, kws):
        announce(f"alone {inst.name}")
        x, y, info = _solver(inst, **kw).solve()
        alone.append((to_np(x), to_np(y), info))
    b = Batch(max_slots=4)
    slot_of = {b.admit(_solver(inst, **kw)): k for k, (inst, kw) in enumerate(zip(insts, kws))}
    got = {}
    while len(got) < len(insts):
        b.step(4)
        for slot in b.poll():
            _, x, y, info = b.fetch(slot)
            got[slot_of[slot]] = (to_np(x), to_np(y), info)
    b.close()
    for k in range(len(insts)):
        np.testing.assert_array_equal(got[k][0], alone[k][0])
        np.testing.assert_array_equal(got[k][1], alone[k][1])
        assert got[k][2]["status"] == "ok"
        kk = oracle.kkt(oracle.Problem(insts[k]), got[k][0], got[k][1])
        assert kk["rel_kkt"] <= 1e-6
