"""Parity at the benchmark workloads' full sizes, in the launch configuration the benchmark uses.

The oracle cannot run whole solves at these sizes within a test, so it checks what it can compute
in one pass: every row of the operator (or the relative KKT residual of the GPU's solution, which
needs one pass) on exactly the stored instance.
  * n=4000, m=200, BF16 and FP16 stacks (6.4 GB): the GPU solution's relative KKT, evaluated by the
    oracle in FP64 on the stored values, is <= 1e-6;
  * kernel-learning QCQP, 8000 points (n=8001, m=5, Q_0 absent, p=1), FP32 and BF16: operator
    parity (U, g, f, grad) at 1e-12;
  * the paper's kernel-learning min-max form, n=4000 (lambda on the simplex, x >= 0, mu = 2),
    FP64 and BF16: oracle natural-residual KKT of the GPU solution <= 1e-6;
  * serving requests of the full size range, solved together in one batch: oracle KKT <= 1e-6;
  * the random convex QCQP n=2000, m=100 (bit-identical on host and GPU, checked by hash) against
    the oracle's own solve stored under tests/golden: objective within 1e-6 (1 + |f*|), with the
    packed symmetric and the row-major pass.
"""
import numpy as np
import pytest

from tests.gpu_common import announce, assert_operator_parity, oracle, qi, to_np

pytestmark = pytest.mark.gpu


def _host_instance(inst):
    import dataclasses
    return dataclasses.replace(inst, Q=inst.Q.cpu())


@pytest.mark.parametrize("storage", ["bfloat16", "float16"])
def test_precision_workload_full_size_kkt(storage):
    import torch
    from paper_2605_29291_amd import Solver
    announce(f"full size n=4000 m=200 {storage}")
    sd = {"bfloat16": torch.bfloat16, "float16": torch.float16}[storage]
    inst = qi.random_qcqp_torch(4000, 200, qi.config_seed(3), shift=0.01, device="cuda", store_dtype=sd)
    s = Solver(inst, device=True, storage=storage, tau_bar=0.0, gamma0=0.1)
    x, y, info = s.solve()
    s.close()
    assert info["status"] == "ok", info
    host = _host_instance(inst)
    del inst
    torch.cuda.empty_cache()
    announce("oracle KKT evaluation (one host pass over the stored stack)")
    kk = oracle.kkt(oracle.Problem(host), to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    assert abs(kk["rel_kkt"] - info["rel_kkt"]) <= 1e-9


@pytest.mark.parametrize("storage", ["float32", "bfloat16"])
def test_kml_workload_full_size_operator(storage):
    import torch
    from paper_2605_29291_amd import Solver
    announce(f"kml full size {storage}")
    sd = {"float32": torch.float32, "bfloat16": torch.bfloat16}[storage]
    inst = qi.kml_qcqp(npts=8000, seed=qi.config_seed(4), device="cuda", store_dtype=sd)
    s = Solver(inst, device=True, storage=storage, tau_bar=1.0)
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(0, 1, 8000), [3.0]])
    y = np.concatenate([[0.3], rng.uniform(0, 2, 5)])
    out = s.eval_operator(x, y)
    s.close()
    host = _host_instance(inst)
    del inst
    torch.cuda.empty_cache()
    ref = oracle.operator(oracle.Problem(host), x, y)
    assert_operator_parity(host, x, y, out, ref)


@pytest.mark.parametrize("storage", ["float64", "bfloat16"])
def test_kml_minmax_full_size_kkt(storage):
    """The paper's kernel-learning min-max form at its n = 4000 size: lambda on the 3-simplex,
    x >= 0, b'x = 0 through v, mu = 2; the oracle's natural-residual KKT of the GPU solution."""
    import torch
    from paper_2605_29291_amd import Solver
    announce(f"kml min-max full size n=4000 {storage}")
    sd = {"float64": torch.float64, "bfloat16": torch.bfloat16}[storage]
    inst = qi.kml_minmax(4000, seed=qi.config_seed(4), device="cuda", store_dtype=sd)
    s = Solver(inst, device=True, storage=storage, tau_bar=0.5, gamma0=0.1, mu=2.0,
               restart_every=200)
    x, y, info = s.solve()
    s.close()
    assert info["status"] == "ok", info
    host = _host_instance(inst)
    del inst
    torch.cuda.empty_cache()
    kk = oracle.kkt(oracle.Problem(host), to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    assert abs(kk["rel_kkt"] - info["rel_kkt"]) <= 1e-9
    lam = to_np(y)[1:]
    assert np.all(lam >= 0) and abs(lam.sum() - 1.0) <= 1e-12
    assert np.all(to_np(x) >= 0)


def test_serving_requests_full_size_range_in_one_batch():
    import torch
    from paper_2605_29291_amd import Batch, Solver
    trace = qi.serving_trace(6, qi.config_seed(5))
    b = Batch(max_slots=8, storage="bfloat16")
    slot_req = {}
    insts = []
    for k, r in enumerate(trace):
        announce(f"request n={r['n']} m={r['m']}")
        inst = qi.random_qcqp_torch(r["n"], r["m"], r["seed"], device="cuda", store_dtype=torch.bfloat16)
        slot_req[b.admit(Solver(inst, device=True, storage="bfloat16", tau_bar=0.0, gamma0=0.1))] = k
        insts.append(_host_instance(inst))
        del inst
    torch.cuda.empty_cache()
    got = {}
    while len(got) < len(trace):
        b.step(4)
        for slot in b.poll():
            _, x, y, info = b.fetch(slot)
            got[slot_req[slot]] = (to_np(x), to_np(y), info)
    b.close()
    for k, host in enumerate(insts):
        x, y, info = got[k]
        assert info["status"] == "ok"
        kk = oracle.kkt(oracle.Problem(host), x, y)
        assert kk["rel_kkt"] <= 1e-6, (k, kk)


def test_exact_generator_on_the_gpu_equals_the_host_bytes():
    """random_qcqp_exact gives the same stack on the GPU (torch products) as on the host (numpy):
    the products are exact and the division by n is one correctly rounded operation."""
    announce("exact generator: device bytes == host bytes")
    dev = qi.random_qcqp_exact(300, 3, seed=17, shift=0.01, device="cuda")
    host = qi.random_qcqp_exact(300, 3, seed=17, shift=0.01)
    np.testing.assert_array_equal(dev.Q.cpu().numpy(), host.Q)
    np.testing.assert_array_equal(dev.q, host.q)
    np.testing.assert_array_equal(dev.c, host.c)


@pytest.mark.parametrize("sym_pass", [1, 0])
def test_random_qcqp_n2000_objective_matches_the_oracle_solution(sym_pass):
    """The random convex QCQP n = 2000, m = 100 at full size against the oracle's own solve
    (stored by tests/golden/make_golden.py, relative KKT 5.7e-11): the GPU stops at relative
    KKT <= 1e-6 with |f - f*| <= 1e-6 (1 + |f*|); ||x - x*|| / (1 + ||x*||) is reported."""
    import json
    import os
    from paper_2605_29291_amd import Solver
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "random_qcqp_n2000_m100.json")))
    announce(f"n=2000 m=100 objective against the oracle's solution, sym_pass={sym_pass}")
    inst = qi.random_qcqp_exact(2000, 100, qi.config_seed(2), shift=0.01, device="cuda")
    assert qi.stack_sha256(inst.Q) == gold["q_stack_sha256"], "not the stored instance"
    s = Solver(inst, device=True, tau_bar=gold["oracle_options"]["tau_bar"], gamma0=0.1, spec_trials=3,
               sym_pass=sym_pass)
    x, y, info = s.solve()
    s.close()
    assert info["status"] == "ok" and info["rel_kkt"] <= 1e-6, info
    fs = gold["f_star"]
    xs = np.array(gold["x_star"])
    dx = float(np.linalg.norm(to_np(x) - xs) / (1 + np.linalg.norm(xs)))
    print(f"[gpu-test] f = {info['f']:.12f}  f* = {fs:.12f}  |f - f*|/(1+|f*|) = "
          f"{abs(info['f'] - fs) / (1 + abs(fs)):.2e}  ||x - x*||/(1+||x*||) = {dx:.2e}", flush=True)
    assert abs(info["f"] - fs) <= 1e-6 * (1 + abs(fs))
    assert dx <= 1e-4
