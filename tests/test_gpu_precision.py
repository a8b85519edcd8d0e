"""Precision form: Q stored as FP32 / BF16 / FP16, FP32 accumulation, FP64 test / restart / KKT.

The instance is the stored (rounded) stack; the FP64 oracle solves exactly those values.  The GPU
solution must reach relative KKT <= 1e-6 as evaluated by the oracle, with the objective within
1e-6 (1 + |f|) of the oracle's own solve of the same stored instance -- in the default incremental
pass mode and in the direct mode (FP32 accumulation of full products).  The stop decision is
re-confirmed on an exact FP64 re-anchor, so the reported rel_kkt equals the exact evaluation.
"""
import numpy as np
import pytest

from tests.gpu_common import announce, oracle, oracle_opts, qi, tau_bar_of, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["float32", "bfloat16", "float16"])
@pytest.mark.parametrize("pass_mode", ["auto", "direct"])
def test_rounded_instance_solution_parity(storage, pass_mode):
    from paper_2605_29291_amd import Solver
    inst = qi.round_instance(qi.random_qcqp(300, 20, seed=61, shift=0.01), storage)
    P = oracle.Problem(inst)
    tb = tau_bar_of(inst)
    announce(f"precision {storage} {pass_mode}")
    s = Solver(inst, tau_bar=tb, gamma0=0.1, storage=storage, pass_mode=pass_mode)
    x, y, info = s.solve()
    assert info["status"] == "ok", info
    kk = oracle.kkt(P, to_np(x), to_np(y))
    assert kk["rel_kkt"] <= 1e-6, kk
    # the GPU's stop test ran on exact FP64 values
    assert abs(info["rel_kkt"] - kk["rel_kkt"]) <= 1e-9
    ref = oracle.solve(P, oracle_opts(tb))
    f_ref = ref["info"]["f"]
    assert abs(kk["f"] - f_ref) <= 1e-6 * (1 + abs(f_ref))


def test_storage_error_against_unrounded_problem_is_reported_scale():
    """Secondary (not a gate in the bench): the rounded-instance solution sits within the
    perturbation the rounding makes -- BF16 (8-bit significand) farther than FP16 (11-bit)."""
    from paper_2605_29291_amd import Solver
    base = qi.random_qcqp(200, 10, seed=62, shift=0.01)
    tb = tau_bar_of(base)
    x64, _, _ = Solver(base, tau_bar=tb).solve()
    x64 = to_np(x64)
    errs = {}
    for storage in ("bfloat16", "float16"):
        inst = qi.round_instance(base, storage)
        x, _, info = Solver(inst, tau_bar=tb, storage=storage).solve()
        errs[storage] = np.linalg.norm(to_np(x) - x64) / (1 + np.linalg.norm(x64))
    assert errs["float16"] < errs["bfloat16"] < 1e-2
