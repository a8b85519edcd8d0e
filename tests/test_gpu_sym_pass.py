"""GPU parity of the packed symmetric pass (options.sym_pass = 1) against the FP64 oracle.

The packed stack holds only the upper-triangle 128 x 128 tiles of every Q_i; the products
(Q_i w)_r are the row dots of tile row I plus the column dots of tile column I.  Checked:

* one pass (qcqp_eval_operator): U = [Q_i x], g, f, grad_x Phi, every element within 1e-12 of
  the sum of its terms' magnitudes, for n a
  multiple of 128, one past it, ragged, a single tile, with an equality block, without Q_0 and
  with affine constraints that store no matrix;
* trajectories: the same iterates as the oracle's (rtol 1e-10) for K iterations with two to
  four speculative candidates, and the row-major pass's iterates within the same bar; at
  n = 1100 (nine tile rows); the APDB-xy routine as well;
* final solutions: relative KKT <= 1e-6 evaluated by the oracle; two solves bitwise equal;
* the random convex QCQP n = 2000, m = 100 (the config-2 workload): converged, relative KKT of
  the returned point by the oracle's evaluation <= 1e-6;
* refusals: FP32 storage with sym_pass, and a batch admitting a sym_pass handle (16-bit
  storage: tests/test_gpu_sym16.py).
"""
import dataclasses

import numpy as np
import pytest

from tests.gpu_common import announce, assert_operator_parity, oracle, qi, tau_bar_of, to_np

pytestmark = pytest.mark.gpu


def _solver(inst, **kw):
    from paper_2605_29291_amd import Solver
    return Solver(inst, **kw)


def _operator_parity(inst, seed=0, tol=1e-12):
    s = _solver(inst, tau_bar=1.0, sym_pass=1)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-3, 3, inst.n)
    y = np.concatenate([rng.standard_normal(inst.p), rng.uniform(0, 2, inst.m)])
    out = s.eval_operator(x, y)
    P = oracle.Problem(inst)
    ref = oracle.operator(P, x, y)
    assert_operator_parity(inst, x, y, out, ref, tol=tol)
    s.close()


@pytest.mark.parametrize("n,m,p", [(128, 3, 0), (129, 4, 1), (300, 6, 0), (40, 2, 0), (513, 3, 2)])
def test_sym_operator_matches_oracle(n, m, p):
    inst = qi.random_qcqp(n, m, seed=3000 + n, shift=0.01, p=p)
    announce(f"sym operator n={n} m={m} p={p}")
    _operator_parity(inst)


def test_sym_operator_without_q0_and_with_unstored_matrices():
    inst = qi.kml_qcqp(npts=300, seed=3)
    announce("sym operator kernel-learning QCQP (no Q_0)")
    _operator_parity(inst)
    base = qi.random_qcqp(260, 5, seed=31, shift=0.01)
    Q = np.array(base.Q)
    stored = np.array([1, 0, 1, 1, 0, 1], dtype=np.int32)
    sparse = qi.Instance(260, 5, 0, Q[stored == 1], base.q, base.c, base.lb, base.ub, q_stored=stored)
    announce("sym operator with unstored matrices")
    _operator_parity(sparse, seed=1)


@pytest.mark.parametrize("spec", [2, 3, 4])
def test_sym_trajectory_matches_oracle_and_row_major(spec):
    inst = qi.random_qcqp(300, 8, seed=41, shift=0.01)
    tb = tau_bar_of(inst)
    K = 60
    kw = dict(tau_bar=tb, gamma0=0.1, max_iter=K, tol=0.0)
    announce(f"sym trajectory spec={spec}")
    ref = oracle.solve(oracle.Problem(inst), oracle.Options(**kw))
    xs, ys, infs = _solver(inst, spec_trials=spec, sym_pass=1, **kw).solve()
    xr, yr, infr = _solver(inst, spec_trials=spec, **kw).solve()
    assert infs["iters"] == K and infs["trials"] == ref["info"]["trials"] == infr["trials"]
    np.testing.assert_allclose(to_np(xs), ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(ys), ref["y"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(xs), to_np(xr), rtol=1e-10, atol=1e-11)


@pytest.mark.parametrize("spec", [2, 4])
def test_sym_trajectory_many_tile_rows(spec):
    """n = 1100: nine tile rows, so the per-row sums of the tile results take more than one
    chunk of eight terms, with several candidates per pass."""
    inst = qi.random_qcqp(1100, 3, seed=48, shift=0.01)
    tb = tau_bar_of(inst)
    K = 20
    kw = dict(tau_bar=tb, gamma0=0.1, max_iter=K, tol=0.0)
    announce(f"sym trajectory n=1100 spec={spec}")
    ref = oracle.solve(oracle.Problem(inst), oracle.Options(**kw))
    x, y, info = _solver(inst, spec_trials=spec, sym_pass=1, **kw).solve()
    assert info["iters"] == K and info["trials"] == ref["info"]["trials"]
    np.testing.assert_allclose(to_np(x), ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(y), ref["y"], rtol=1e-10, atol=1e-11)


def test_sym_xy_trajectory_matches_oracle():
    inst = qi.random_qcqp(260, 6, seed=47, shift=0.01, p=1)
    tb = tau_bar_of(inst)
    K = 50
    kw = dict(tau_bar=tb, gamma0=0.1, max_iter=K, tol=0.0)
    xy = dict(c_alpha=0.25, c_beta=0.3, delta=0.4)
    announce("sym trajectory xy")
    ref = oracle.solve(oracle.Problem(inst), oracle.Options.xy(**kw))
    x, y, info = _solver(inst, spec_trials=2, sym_pass=1, variant="xy", **xy, **kw).solve()
    assert info["iters"] == K and info["trials"] == ref["info"]["trials"]
    np.testing.assert_allclose(to_np(x), ref["x"], rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(to_np(y), ref["y"], rtol=1e-10, atol=1e-11)


def test_sym_final_solution_and_determinism():
    inst = qi.random_qcqp(400, 12, seed=43, shift=0.01, p=2)
    tb = tau_bar_of(inst)
    announce("sym final solution")
    s = _solver(inst, tau_bar=tb, gamma0=0.1, spec_trials=3, sym_pass=1)
    x1, y1, i1 = s.solve()
    x2, y2, i2 = s.solve()
    assert i1["status"] == "ok", i1
    kk = oracle.kkt(oracle.Problem(inst), to_np(x1), to_np(y1))
    assert kk["rel_kkt"] <= 1e-6, kk
    assert abs(i1["rel_kkt"] - kk["rel_kkt"]) <= 1e-9
    np.testing.assert_array_equal(to_np(x1), to_np(x2))
    np.testing.assert_array_equal(to_np(y1), to_np(y2))
    n = inst.n
    assert i1["pass_bytes"] == (inst.m + 1) * (n * (n + 1) // 2) * 8


def test_sym_full_size_random_qcqp():
    """The random convex QCQP n=2000, m=100 solved through the packed symmetric pass; the
    returned point checked by the oracle's KKT evaluation (one host pass over the stack)."""
    import torch
    n, m = 2000, 100
    announce("sym full size n=2000 m=100")
    inst = qi.random_qcqp_exact(n, m, qi.config_seed(2), shift=0.01, device="cuda")
    L0 = float(torch.linalg.matrix_norm(inst.Q[0], ord=2))
    s = _solver(inst, device=True, tau_bar=1.0 / L0, gamma0=0.1, spec_trials=3, sym_pass=1)
    x, y, info = s.solve()
    s.close()
    assert info["status"] == "ok", info
    host = dataclasses.replace(inst, Q=inst.Q.cpu().numpy())
    del inst
    torch.cuda.empty_cache()
    kk = oracle.kkt(oracle.Problem(host), to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    assert abs(info["rel_kkt"] - kk["rel_kkt"]) <= 1e-9


def test_sym_large_n_three_candidates():
    """n = 10000 with three candidates: the row-major pass would need 240 KB of LDS for the staged
    trial points and is refused; the packed pass holds them in registers."""
    import torch
    from paper_2605_29291_amd import QCQPError
    n = 10000
    announce("sym n=10000 spec=3")
    inst = qi.random_qcqp_torch(n, 0, 409, shift=0.01, device="cuda")
    with pytest.raises(QCQPError):
        _solver(inst, device=True, tau_bar=1.0, spec_trials=3)
    s = _solver(inst, device=True, tau_bar=1.0, spec_trials=3, sym_pass=1)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, n)
    out = s.eval_operator(x)
    s.close()
    host = dataclasses.replace(inst, Q=inst.Q.cpu().numpy())
    del inst
    torch.cuda.empty_cache()
    ref = oracle.operator(oracle.Problem(host), x, np.zeros(0))
    assert_operator_parity(host, x, None, out, ref)


def test_sym_refusals():
    from paper_2605_29291_amd import Batch, QCQPError
    inst = qi.random_qcqp(100, 2, seed=45, shift=0.01)
    announce("sym refusals")
    with pytest.raises(QCQPError) as e:
        _solver(qi.round_instance(inst, "float32"), storage="float32", tau_bar=1.0, sym_pass=1)
    assert e.value.code == 1
    s = _solver(inst, tau_bar=1.0, sym_pass=1)
    b = Batch(max_slots=2)
    with pytest.raises(QCQPError) as e:
        b.admit(s)
    assert e.value.code == 1
    b.close()
    x, y, info = s.solve()
    assert info["status"] == "ok"


def test_sym_adaptive_restart_and_gap():
    """The packed FP64 pass with the adaptive restart of eq. (ada_restart): G_xi at a given point
    on the packed handle equals the oracle's (its anchor pass streams the packed tiles, its box
    QP reads the row-major stack), and the solve takes the oracle's restart decisions on the
    schedule (iterations within 1 %, the same restart count)."""
    inst = qi.random_qcqp(300, 8, seed=43, shift=0.01)
    tb = tau_bar_of(inst)
    P = oracle.Problem(inst)
    s = _solver(inst, sym_pass=1, spec_trials=3, tau_bar=tb)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, inst.n)
    y = rng.uniform(0, 0.5, inst.m)
    announce("sym G_xi at a point")
    g = s.eval_gap(x, y, xi=0.04)
    r = oracle.gap(P, x, y, xi=0.04)
    assert abs(g["Py"] - r["Py"]) <= 1e-11 * (1 + abs(r["Py"])), (g, r)
    assert abs(g["Px"] - r["Px"]) <= 1e-9 * (1 + abs(r["Px"])), (g, r)
    s.close()
    kw = dict(tau_bar=tb, gamma0=0.1, tol=1e-9, restart="adaptive", ada_first=10, ada_every=20, max_iter=20000)
    ref = oracle.solve(P, oracle.Options(**kw))
    announce(f"sym adaptive solve: oracle {ref['info']['iters']} iterations, {ref['info']['restarts']} restarts")
    xs, ys, info = _solver(inst, sym_pass=1, spec_trials=3, **kw).solve()
    assert ref["info"]["status"] == "converged" and info["status"] == "ok", (info, ref["info"])
    k, k_ref = info["iters"], ref["info"]["iters"]
    assert abs(k - k_ref) <= max(2, 0.01 * k_ref), (k, k_ref)
    assert info["restarts"] == ref["info"]["restarts"] >= 2, (info["restarts"], ref["info"]["restarts"])
