"""GPU parity of one Q-stack pass (qcqp_eval_operator, qcqp_eval_kkt) against the FP64 oracle.

Bar: every element of U = [Q_i x], g, f and grad_x Phi within 1e-12 of the sum of the magnitudes
of its terms (tests/gpu_common.assert_operator_parity), in FP64 storage and for every 32/16-bit
storage type (the operator pass accumulates in FP64 over the stored values, so the oracle on the
same rounded instance differs only by summation order).
"""
import numpy as np
import pytest

from tests.gpu_common import abs_products, announce, assert_operator_parity, oracle, qi, tau_bar_of, to_np

pytestmark = pytest.mark.gpu


def _check_operator(inst, storage="float64", device=False, seed=0, tol=1e-12):
    from paper_2605_29291_amd import Solver
    announce(f"operator {inst.name} n={inst.n} m={inst.m} p={inst.p} storage={storage}")
    s = Solver(inst, device=device, storage=storage, tau_bar=1.0)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-3, 3, inst.n)
    y = np.concatenate([rng.standard_normal(inst.p), rng.uniform(0, 2, inst.m)])
    out = s.eval_operator(x, y)
    P = oracle.Problem(inst)
    ref = oracle.operator(P, x, y)
    assert_operator_parity(inst, x, y, out, ref, tol=tol)
    kk = s.eval_kkt(x, y)
    kr = oracle.kkt(P, x, y)
    for k in ("rel_kkt", "rel_dual", "rel_pri", "rel_comp", "f", "max_violation"):
        assert abs(kk[k] - kr[k]) <= 1e-11 * (abs(kr[k]) + 1e-12), (k, kk[k], kr[k])
    s.close()


@pytest.mark.parametrize("n,m,p", [(100, 10, 0), (37, 3, 0), (129, 5, 2), (1, 2, 0), (301, 0, 0),
                                   (1000, 4, 1), (2001, 2, 0)])
def test_operator_fp64_host_pointers(n, m, p):
    inst = qi.random_qcqp(n, m, seed=1000 + n + m, shift=0.01, p=p)
    _check_operator(inst)


@pytest.mark.parametrize("storage", ["float32", "bfloat16", "float16"])
@pytest.mark.parametrize("n", [100, 333])
def test_operator_rounded_storage_device_pointers(storage, n):
    inst = qi.round_instance(qi.random_qcqp(n, 4, seed=77 + n, shift=0.01), storage)
    import torch
    inst.Q = inst.Q.cuda()
    _check_operator(inst, storage=storage, device=True)


def test_operator_without_q0_and_with_equalities():
    inst = qi.kml_qcqp(npts=300, seed=3)
    _check_operator(inst)


def test_conversion_from_fp64_rounds_to_nearest_even():
    """FP64 input stored as BF16/FP16/FP32 by the library: read the stored values back through
    unit-vector passes and compare with an exact round-to-nearest-even done in numpy."""
    from paper_2605_29291_amd import Solver
    import torch
    n, m = 24, 1
    rng = np.random.default_rng(5)
    Q = rng.standard_normal((m + 1, n, n)) * np.exp(rng.uniform(-8, 8, (m + 1, n, n)))
    # include exact ties for bf16: values halfway between two bf16 numbers
    Q[0, 0, :8] = (1.0 + np.arange(8) * 2.0 ** -7) + 2.0 ** -8
    Q = np.triu(Q) + np.transpose(np.triu(Q, 1), (0, 2, 1))   # the library stores symmetric Q_i
    inst = qi.Instance(n, m, 0, Q, np.zeros((m + 1, n)), np.zeros(m + 1), -np.ones(n), np.ones(n))
    for storage in ("float32", "bfloat16", "float16"):
        announce(f"conversion {storage}")
        s = Solver(inst, storage=storage, tau_bar=1.0)
        got = np.empty((m + 1, n, n))
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            got[:, :, j] = to_np(s.eval_operator(e)["U"])
        if storage == "float32":
            ref = Q.astype(np.float32).astype(np.float64)
        elif storage == "float16":
            ref = Q.astype(np.float16).astype(np.float64)
        else:
            ref = _bf16_rne(Q)
        np.testing.assert_array_equal(got, ref)
        s.close()


def _bf16_rne(a):
    """Exact double -> bfloat16 rounding (nearest, ties to even), via exact integer arithmetic."""
    out = np.empty_like(a)
    flat = a.reshape(-1)
    o = out.reshape(-1)
    for k, v in enumerate(flat):
        if v == 0 or not np.isfinite(v):
            o[k] = v
            continue
        mant, ex = np.frexp(abs(v))          # v = mant * 2^ex, mant in [0.5, 1)
        scaled = mant * 2.0 ** 8             # bf16 keeps 8 significant bits
        lo = np.floor(scaled)
        rem = scaled - lo
        if rem > 0.5 or (rem == 0.5 and int(lo) % 2 == 1):
            lo += 1
        o[k] = np.copysign(lo * 2.0 ** (ex - 8), v)
    return out


def test_operator_config2_full_size():
    """n = 2000, m = 100, FP64 stack of 3.2 GB in the launch configuration the solve uses;
    the oracle computes every row."""
    import torch
    announce("operator config-2 full size")
    inst = qi.random_qcqp_exact(2000, 100, qi.config_seed(2), shift=0.01, device="cuda")
    from paper_2605_29291_amd import Solver
    s = Solver(inst, device=True, tau_bar=1.0)
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 1, inst.n)
    y = rng.uniform(0, 1, inst.m)
    out = s.eval_operator(x, y)
    s.close()
    Qh = inst.Q.cpu().numpy()
    del inst.Q
    torch.cuda.empty_cache()
    inst.Q = Qh
    P = oracle.Problem(inst)
    ref = oracle.operator(P, x, y)
    assert_operator_parity(inst, x, y, out, ref)
