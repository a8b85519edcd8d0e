"""Pins for the oracle's operator: Q-stack products, g, f, grad_x Phi (eq. (qcqp-coupling), §2.1).

Each check uses something other than the oracle's own formula: closed forms (identity, rank-1,
diagonal matrices), numpy's matmul, finite differences of Phi, exact dtype decoders.
"""
import numpy as np
import pytest

import qcqp_inputs as qi


def _phi(Q, q, c, A, b, x, y, p):
    """Phi(x, y) = f(x) + <v, Ax-b> + <lambda, g(x)>, written from the definition."""
    m = q.shape[0] - 1
    val = 0.5 * x @ Q[0] @ x + q[0] @ x + c[0]
    for i in range(1, m + 1):
        val += y[p + i - 1] * (0.5 * x @ Q[i] @ x + q[i] @ x + c[i])
    if p:
        val += y[:p] @ (A @ x - b)
    return val


def test_identity_matrices_closed_form(orc):
    n, m = 7, 3
    rng = np.random.default_rng(0)
    Q = np.stack([np.eye(n)] * (m + 1))
    q = rng.standard_normal((m + 1, n))
    c = rng.standard_normal(m + 1)
    P = orc.Problem(Q=Q, q=q, c=c, lb=-np.ones(n), ub=np.ones(n))
    x = rng.standard_normal(n)
    out = orc.operator(P, x)
    for i in range(m + 1):
        assert np.array_equal(out["U"][i], x)
    g = 0.5 * (x @ x) + q[1:] @ x + c[1:]
    np.testing.assert_allclose(out["G"], g, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(out["f"], 0.5 * (x @ x) + q[0] @ x + c[0], rtol=1e-15)


def test_rank_one_and_diagonal(orc):
    n = 9
    rng = np.random.default_rng(1)
    a = rng.standard_normal(n)
    dvec = rng.uniform(0.1, 2.0, n)
    Q = np.stack([np.outer(a, a), np.diag(dvec)])
    P = orc.Problem(Q=Q, q=np.zeros((2, n)), c=np.zeros(2), lb=-np.ones(n), ub=np.ones(n))
    x = rng.standard_normal(n)
    out = orc.operator(P, x)
    np.testing.assert_allclose(out["U"][0], (a @ x) * a, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(out["U"][1], dvec * x, rtol=1e-15)


def test_against_numpy_matmul_and_symmetry(orc):
    inst = qi.random_qcqp(40, 5, seed=3, shift=0.01, p=2)
    P = orc.Problem(inst)
    rng = np.random.default_rng(2)
    x = rng.uniform(-3, 3, inst.n)
    out = orc.operator(P, x)
    U_np = np.einsum("irj,j->ir", inst.Q, x)
    np.testing.assert_allclose(out["U"], U_np, rtol=1e-12, atol=1e-12)
    # symmetric data: Q_i' x equals Q_i x
    U_t = np.einsum("ijr,j->ir", inst.Q, x)
    np.testing.assert_allclose(out["U"], U_t, rtol=1e-12, atol=1e-12)
    h = inst.A @ x - inst.b
    np.testing.assert_allclose(out["G"][:2], h, rtol=1e-13, atol=1e-14)


def test_gradient_by_finite_differences(orc):
    """grad_x Phi and grad_y Phi against central differences of Phi built from its definition."""
    inst = qi.random_qcqp(12, 4, seed=5, shift=0.01, p=2)
    P = orc.Problem(inst)
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, inst.n)
    y = np.concatenate([rng.standard_normal(2), rng.uniform(0, 2, inst.m)])
    out = orc.operator(P, x, y)
    h = 1e-6
    fd = np.empty(inst.n)
    for j in range(inst.n):
        e = np.zeros(inst.n)
        e[j] = h
        fd[j] = (_phi(inst.Q, inst.q, inst.c, inst.A, inst.b, x + e, y, 2)
                 - _phi(inst.Q, inst.q, inst.c, inst.A, inst.b, x - e, y, 2)) / (2 * h)
    np.testing.assert_allclose(out["grad"], fd, rtol=1e-7, atol=1e-7)
    # Phi is affine in y: its y-gradient is (Ax - b, g(x))
    fdy = np.empty(len(y))
    for l in range(len(y)):
        e = np.zeros(len(y))
        e[l] = 1.0
        fdy[l] = (_phi(inst.Q, inst.q, inst.c, inst.A, inst.b, x, y + e, 2)
                  - _phi(inst.Q, inst.q, inst.c, inst.A, inst.b, x, y, 2))
    np.testing.assert_allclose(out["G"], fdy, rtol=1e-11, atol=1e-11)


def test_quadratic_identity_of_test_function(orc):
    """Phi(x',y) - Phi(x,y) - <grad_x Phi(x,y), x'-x> = 1/2 d'Q(lambda)d (Phi quadratic in x).

    Left side from Phi's definition (numpy); right side from the oracle's U at x and x':
    1/2 [d'(U'_0 - U_0) + sum lambda_i d'(U'_i - U_i)] -- the form the test function uses."""
    inst = qi.random_qcqp(15, 3, seed=8, shift=0.01)
    P = orc.Problem(inst)
    rng = np.random.default_rng(6)
    x = rng.uniform(-2, 2, inst.n)
    d = rng.uniform(-0.5, 0.5, inst.n)
    y = rng.uniform(0, 1.5, inst.m)
    o0 = orc.operator(P, x, y)
    o1 = orc.operator(P, x + d, y)
    lhs = (_phi(inst.Q, inst.q, inst.c, None, None, x + d, y, 0)
           - _phi(inst.Q, inst.q, inst.c, None, None, x, y, 0) - o0["grad"] @ d)
    w = np.concatenate([[1.0], y])
    rhs = 0.5 * sum(w[i] * d @ (o1["U"][i] - o0["U"][i]) for i in range(inst.m + 1))
    Qlam = inst.Q[0] + np.tensordot(y, inst.Q[1:], axes=1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10)
    np.testing.assert_allclose(rhs, 0.5 * d @ Qlam @ d, rtol=1e-12)


@pytest.mark.parametrize("dt", ["float32", "bfloat16", "float16"])
def test_rounded_storage_decodes_exactly(orc, dt):
    """16/32-bit stored Q is upcast exactly: compare with torch's own exact upcast."""
    import torch
    inst = qi.random_qcqp(33, 2, seed=11, shift=0.01)
    r = qi.round_instance(inst, dt)
    Q64 = r.Q.to(torch.float64).numpy()
    P = orc.Problem(r)
    x = np.random.default_rng(3).uniform(-1, 1, inst.n)
    out = orc.operator(P, x)
    ref = np.einsum("irj,j->ir", Q64, x)
    np.testing.assert_allclose(out["U"], ref, rtol=1e-12, atol=1e-13)


def test_float16_decoder_all_codes(orc):
    """Every finite float16 bit pattern through the oracle equals numpy's decoding."""
    codes = np.arange(0, 65536, dtype=np.uint32).astype(np.uint16)
    vals = codes.view(np.float16).astype(np.float64)
    finite = np.isfinite(vals)
    codes, vals = codes[finite], vals[finite]
    k = len(codes)
    n = 256
    rows = (k + n - 1) // n
    pad = rows * n - k
    Qc = np.concatenate([codes, np.zeros(pad, np.uint16)]).reshape(rows, n)
    Qv = np.concatenate([vals, np.zeros(pad)]).reshape(rows, n)
    # rows x n block placed as Q_1 rows (n x n matrices, repeated in chunks of n rows)
    blocks = (rows + n - 1) // n
    Qfull = np.zeros((blocks, n, n), np.uint16)
    Vfull = np.zeros((blocks, n, n))
    Qfull.reshape(-1, n)[:rows] = Qc
    Vfull.reshape(-1, n)[:rows] = Qv
    P = orc.Problem(Q=Qfull.view(np.float16), q=np.zeros((blocks, n)), c=np.zeros(blocks),
                    lb=-np.ones(n), ub=np.ones(n))
    for j in [0, 17, 255]:
        e = np.zeros(n)
        e[j] = 1.0
        out = orc.operator(P, e)
        np.testing.assert_array_equal(out["U"], Vfull[:, :, j])


def test_absent_q0(orc):
    inst = qi.random_qcqp(10, 3, seed=2)
    Qs = inst.Q[1:]
    P = orc.Problem(Q=Qs, q=inst.q, c=inst.c, lb=inst.lb, ub=inst.ub, has_q0=False)
    x = np.linspace(-1, 1, 10)
    out = orc.operator(P, x)
    assert np.all(out["U"][0] == 0)
    np.testing.assert_allclose(out["U"][1:], np.einsum("irj,j->ir", Qs, x), rtol=1e-13)
    np.testing.assert_allclose(out["f"], inst.q[0] @ x + inst.c[0], rtol=1e-14)
