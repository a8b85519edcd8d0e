"""Shared helpers for the GPU parity tests (test infrastructure)."""
import numpy as np

import oracle
import qcqp_inputs as qi


def tau_bar_of(inst):
    Q = inst.q_as_float64_numpy() if hasattr(inst.Q, "detach") else np.asarray(inst.Q, dtype=float)
    if inst.has_q0:
        L = np.linalg.norm(Q[0], 2)
    else:
        L = max(np.linalg.norm(Q[i], 2) for i in range(Q.shape[0]))
    return 1.0 / L if L > 0 else 1.0


def to_np(a):
    if hasattr(a, "detach"):
        return a.detach().cpu().numpy()
    return np.asarray(a)


def oracle_opts(tau_bar, gamma0=0.1, **kw):
    return oracle.Options(tau_bar=tau_bar, gamma0=gamma0, **kw)


def gpu_opts(tau_bar, gamma0=0.1, **kw):
    d = dict(tau_bar=tau_bar, gamma0=gamma0)
    d.update(kw)
    return d


def rel_err(a, b, scale):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / scale)


def _stored_rows(inst):
    """Rows of U = [Q_0 x, ..., Q_m x] that come from a stored matrix, in stack order."""
    if getattr(inst, "q_stored", None) is not None:
        return [i for i, f in enumerate(np.asarray(inst.q_stored)) if f]
    return list(range(0 if inst.has_q0 else 1, inst.m + 1))


def abs_products(inst, x):
    """S[i] = |Q_i| |x| for i = 0..m (zero rows for matrices that are not stored, plus
    q0_shift |x| in row 0), one stored matrix at a time so large stacks need no copy."""
    ax = np.abs(np.asarray(x, dtype=np.float64))
    S = np.zeros((inst.m + 1, inst.n))
    for k, i in enumerate(_stored_rows(inst)):
        Qk = inst.Q[k]
        if hasattr(Qk, "detach"):
            import torch
            Qk = Qk.detach().to("cpu", torch.float64).numpy()
        S[i] = np.abs(np.asarray(Qk, dtype=np.float64)) @ ax
    S[0] += float(getattr(inst, "q0_shift", 0.0) or 0.0) * ax
    return S


def assert_operator_parity(inst, x, y, out, ref, tol=1e-12, S=None):
    """GPU operator outputs against the oracle's, element by element, relative to the sum of the
    magnitudes of the terms each value is made of:

      U_ir = sum_j Q_ij x_j                  scale S_ir = sum_j |Q_ij| |x_j|
      g_i  = 1/2 x'U_i + q_i'x + c_i         scale 1/2 |x|'S_i + |q_i|'|x| + |c_i|
      grad = U_0 + q_0 + sum_i l_i (U_i + q_i) + A'v
                                             scale S_0 + |q_0| + sum_i |l_i| (S_i + |q_i|) + |A|'|v|

    Any FP64 summation order of k terms is within gamma_k = k u / (1 - k u) (u = 2^-53) of the
    exact sum times this scale, so two orders differ by at most 2 gamma_k times it: below
    1e-12 for k <= 4500 in the worst case, and by orders of magnitude in practice (the rounding
    errors are not aligned).  tol = 1e-12 is the bar for every size."""
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros(inst.p + inst.m) if y is None else np.asarray(y, dtype=np.float64)
    ax = np.abs(x)
    S = abs_products(inst, x) if S is None else S
    aq = np.abs(np.asarray(inst.q, dtype=np.float64))
    U = to_np(out["U"])
    dU = np.abs(U - ref["U"])
    bad = dU > tol * S
    assert not bad.any(), ("U", np.max(dU / np.maximum(S, 1e-300)), np.argwhere(bad)[:4])
    gs = 0.5 * (S @ ax) + aq @ ax + np.abs(np.asarray(inst.c, dtype=np.float64))
    if "g" in out and out["g"] is not None and inst.m:
        g = to_np(out["g"]).reshape(-1)
        dg = np.abs(g - ref["G"][inst.p:])
        assert np.all(dg <= tol * gs[1:]), ("g", np.max(dg / np.maximum(gs[1:], 1e-300)))
    if "f" in out and out["f"] is not None:
        f = float(np.asarray(to_np(out["f"])).reshape(-1)[0])
        assert abs(f - ref["f"]) <= tol * gs[0], ("f", f, ref["f"], gs[0])
    if "grad" in out and out["grad"] is not None:
        lam = np.abs(y[inst.p:])
        sc = S[0] + aq[0] + lam @ (S[1:] + aq[1:])
        if inst.p:
            sc = sc + np.abs(np.atleast_2d(inst.A)).T @ np.abs(y[:inst.p])
        dgr = np.abs(to_np(out["grad"]) - ref["grad"])
        assert np.all(dgr <= tol * sc), ("grad", np.max(dgr / np.maximum(sc, 1e-300)))


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


__all__ = ["tau_bar_of", "to_np", "oracle_opts", "gpu_opts", "rel_err", "announce", "qi", "oracle",
           "abs_products", "assert_operator_parity"]
