"""Sizes at the library's limits and the degenerate cases, on the GPU, against the FP64 oracle.

* n = 16384 (the largest accepted): BF16 storage with two speculative candidates (128 KB of LDS
  for the staged trial points) and FP64 storage with one; operator parity on the stored stack;
* m = 1024 and p = 64 (the largest accepted): solutions reach relative KKT <= 1e-6 by the oracle;
* one past each limit, and FP64 with two candidates at n = 16384 (256 KB of LDS), are refused
  with QCQP_E_INVALID before anything is allocated;
* a batch step with no resident request is a no-op.
"""
import numpy as np
import pytest

from tests.gpu_common import announce, assert_operator_parity, oracle, qi, tau_bar_of, to_np

pytestmark = pytest.mark.gpu


def _host(inst):
    import dataclasses
    return dataclasses.replace(inst, Q=inst.Q.cpu())


@pytest.mark.parametrize("storage,spec", [("bfloat16", 2), ("float64", 1)])
def test_largest_n_operator_parity(storage, spec):
    import torch
    from paper_2605_29291_amd import Solver
    n, m = 16384, (2 if storage == "bfloat16" else 0)
    sd = {"bfloat16": torch.bfloat16, "float64": torch.float64}[storage]
    announce(f"n={n} m={m} {storage} spec_trials={spec}")
    inst = qi.random_qcqp_torch(n, m, 404, shift=0.01, device="cuda", store_dtype=sd)
    s = Solver(inst, device=True, storage=storage, tau_bar=1.0, spec_trials=spec)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(0, 1, m)
    out = s.eval_operator(x, y)
    s.close()
    host = _host(inst)
    del inst
    torch.cuda.empty_cache()
    announce("oracle operator at n=16384")
    ref = oracle.operator(oracle.Problem(host), x, y)
    assert_operator_parity(host, x, y, out, ref)


@pytest.mark.parametrize("n,m,p", [(48, 1024, 0), (200, 12, 64)])
def test_largest_m_and_p_solve(n, m, p):
    from paper_2605_29291_amd import Solver
    inst = qi.random_qcqp(n, m, seed=405, shift=0.01, p=p)
    tb = tau_bar_of(inst)
    announce(f"n={n} m={m} p={p}")
    x, y, info = Solver(inst, tau_bar=tb, gamma0=0.1).solve()
    assert info["status"] == "ok", info
    kk = oracle.kkt(oracle.Problem(inst), to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    assert np.all(to_np(y)[p:] >= 0)


def test_sizes_past_the_limits_are_refused():
    from paper_2605_29291_amd import QCQPError, Solver
    cases = []
    one = qi.random_qcqp(8, 1, seed=406, shift=0.01)
    # n past the limit: only the sizes are inspected before the refusal, so tiny arrays suffice
    big_n = qi.Instance(16385, 0, 0, np.zeros((1, 1, 1)), np.zeros((1, 16385)), np.zeros(1),
                        -np.ones(16385), np.ones(16385))
    cases.append(("n=16385", big_n, {}))
    big_m = qi.random_qcqp(4, 1025, seed=407, shift=0.01)
    cases.append(("m=1025", big_m, {}))
    big_p = qi.random_qcqp(70, 1, seed=408, shift=0.01, p=65)
    cases.append(("p=65", big_p, {}))
    lds = qi.Instance(16384, 0, 0, np.zeros((1, 1, 1)), np.zeros((1, 16384)), np.zeros(1),
                      -np.ones(16384), np.ones(16384))
    cases.append(("FP64 n=16384 with two candidates", lds, dict(spec_trials=2)))
    for name, inst, kw in cases:
        announce(f"refused: {name}")
        with pytest.raises(QCQPError) as e:
            Solver(inst, tau_bar=1.0, **kw)
        assert e.value.code == 1, name
    # and a normal instance still works afterwards
    x, y, info = Solver(one, tau_bar=1.0).solve()
    assert info["status"] == "ok"


def test_empty_batch_step_is_a_no_op():
    from paper_2605_29291_amd import Batch
    b = Batch(max_slots=4)
    b.step(3)
    assert b.poll() == []
    assert b.stats()["running"] == 0
    b.close()
