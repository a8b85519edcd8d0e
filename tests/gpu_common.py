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


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


__all__ = ["tau_bar_of", "to_np", "oracle_opts", "gpu_opts", "rel_err", "announce", "qi", "oracle"]
