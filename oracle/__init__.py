"""ctypes wrapper around the plain FP64 CPU oracle (qcqp_oracle.c).

TEST INFRASTRUCTURE ONLY: the reference the GPU path is checked against.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library.

Conventions (same as the instance generators): Q is (m+1, n, n) (or (m, n, n) with has_q0 False)
in float64 / float32 / bfloat16 / float16; y = (v, lambda) with v in R^p and lambda in R^m_+
(or in the unit simplex, lambda_set="simplex"), optionally restricted to a ball (ball: ||y|| <= B;
ball_v / ball_l: ||v|| <= B_v, ||lambda|| <= B_lambda); the objective's Hessian is Q_0 + q0_shift I.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("p", C.c_int64),
                ("Q", C.c_void_p), ("q_dtype", C.c_int32), ("has_q0", C.c_int32),
                ("q", C.c_void_p), ("c", C.c_void_p), ("A", C.c_void_p), ("b", C.c_void_p),
                ("lb", C.c_void_p), ("ub", C.c_void_p),
                ("lambda_set", C.c_int32), ("pad0", C.c_int32), ("q0_shift", C.c_double),
                ("ball", C.c_double), ("ball_v", C.c_double), ("ball_l", C.c_double),
                ("q_stored", C.c_void_p), ("n_soc", C.c_int64), ("soc_dims", C.c_void_p)]


class _Options(C.Structure):
    _fields_ = [("variant", C.c_int32), ("c_nm", C.c_int32), ("restart", C.c_int32),
                ("restart_from_average", C.c_int32), ("restart_every", C.c_int64),
                ("ada_first", C.c_int64), ("ada_every", C.c_int64), ("max_iter", C.c_int64),
                ("max_inner", C.c_int64),
                ("eta", C.c_double), ("tau_bar", C.c_double), ("gamma0", C.c_double),
                ("mu", C.c_double), ("c_alpha", C.c_double), ("c_beta", C.c_double),
                ("delta", C.c_double), ("xi", C.c_double), ("q_restart", C.c_double),
                ("tol", C.c_double), ("inner_tol", C.c_double),
                ("stop_rule", C.c_int32), ("pad0", C.c_int32), ("f_star", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("trials", C.c_int64), ("restarts", C.c_int64),
                ("gap_evals", C.c_int64), ("status", C.c_int64),
                ("rel_kkt", C.c_double), ("rel_dual", C.c_double), ("rel_pri", C.c_double),
                ("rel_comp", C.c_double), ("f", C.c_double), ("max_violation", C.c_double),
                ("last_gap", C.c_double), ("stop_value", C.c_double)]


def lib():
    global _LIB
    if _LIB is None:
        # ORACLE_LIB names another build: the sanitizer build of the same source, or a copy with
        # a planted mistake that the pins must catch
        path = os.environ.get("ORACLE_LIB") or _build.LIB
        if path == _build.LIB and (not os.path.exists(path) or
                                   os.path.getmtime(path) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = C.CDLL(path)
        vp = C.c_void_p
        L.orc_operator.argtypes = [C.POINTER(_Problem), vp, vp, vp, vp, vp, vp]
        L.orc_grad_from_u.argtypes = [C.POINTER(_Problem), vp, vp, vp]
        L.orc_project_dual.argtypes = [C.POINTER(_Problem), vp]
        L.orc_kkt.argtypes = [C.POINTER(_Problem), vp, vp, vp]
        L.orc_gap.argtypes = [C.POINTER(_Problem), vp, vp, C.c_double, C.c_double, C.c_int64, vp]
        L.orc_solve.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), vp, vp, vp, vp,
                                C.POINTER(_Info), vp, C.c_int64]
        for f in (L.orc_operator, L.orc_grad_from_u, L.orc_project_dual, L.orc_kkt, L.orc_gap,
                  L.orc_solve):
            f.restype = C.c_int
        _LIB = L
    return _LIB


@dataclasses.dataclass
class Options:
    """rAPDB parameters; defaults are the §5 settings for APDB-yx (eta=0.7, c_alpha=0.4,
    delta=0.5, non-monotone) with fixed-frequency restarts every 400 iterations."""
    variant: str = "yx"             # "yx" | "xy"
    c_nm: int = 1
    restart: str = "fixed"          # "none" | "fixed" | "adaptive"
    restart_every: int = 400
    restart_from_average: bool = False
    ada_first: int = 50
    ada_every: int = 500
    max_iter: int = 50000
    max_inner: int = 200000
    eta: float = 0.7
    tau_bar: float = 1.0
    gamma0: float = 0.1
    mu: float = 0.0
    c_alpha: float = 0.4
    c_beta: float = 0.0
    delta: float = 0.5
    xi: float = 0.04
    q_restart: float = 0.5
    tol: float = 1e-6
    inner_tol: float = 1e-12
    stop_rule: str = "kkt"          # "kkt" | "paper" (needs f_star)
    f_star: float = 0.0

    @staticmethod
    def xy(**kw) -> "Options":
        base = dict(variant="xy", c_alpha=0.25, c_beta=0.3, delta=0.4, restart_every=1000,
                    ada_first=100, ada_every=500)
        base.update(kw)
        return Options(**base)

    def _c(self) -> _Options:
        return _Options(0 if self.variant == "yx" else 1, int(self.c_nm),
                        {"none": 0, "fixed": 1, "adaptive": 2}[self.restart],
                        int(self.restart_from_average), int(self.restart_every),
                        int(self.ada_first), int(self.ada_every), int(self.max_iter),
                        int(self.max_inner), float(self.eta), float(self.tau_bar),
                        float(self.gamma0), float(self.mu), float(self.c_alpha),
                        float(self.c_beta), float(self.delta), float(self.xi),
                        float(self.q_restart), float(self.tol), float(self.inner_tol),
                        {"kkt": 0, "paper": 1}[self.stop_rule], 0, float(self.f_star))


_DT = {"float64": 0, "float32": 1, "bfloat16": 2, "float16": 3}


class Problem:
    """Keeps contiguous host copies alive and exposes the C struct."""

    def __init__(self, inst=None, *, Q=None, q=None, c=None, lb=None, ub=None, A=None, b=None,
                 has_q0=True, lambda_set=None, q0_shift=None, ball=0.0, ball_v=0.0,
                 ball_l=0.0, q_stored=None, soc_dims=None):
        if inst is not None:
            Q, q, c, lb, ub, A, b, has_q0 = (inst.Q, inst.q, inst.c, inst.lb, inst.ub, inst.A,
                                             inst.b, inst.has_q0)
            if lambda_set is None:
                lambda_set = getattr(inst, "lambda_set", None)
            if q0_shift is None:
                q0_shift = getattr(inst, "q0_shift", None)
            if q_stored is None:
                q_stored = getattr(inst, "q_stored", None)
            if soc_dims is None:
                soc_dims = getattr(inst, "soc_dims", None)
        lambda_set = "nonneg" if lambda_set is None else lambda_set
        q0_shift = 0.0 if q0_shift is None else q0_shift
        self.lambda_set = lambda_set
        self.q0_shift = float(q0_shift)
        self.ball, self.ball_v, self.ball_l = float(ball), float(ball_v), float(ball_l)
        Qh, dt = _host_q(Q)
        self.Q = Qh
        self.q = np.ascontiguousarray(q, dtype=np.float64)
        self.c = np.ascontiguousarray(c, dtype=np.float64)
        self.lb = np.ascontiguousarray(lb, dtype=np.float64)
        self.ub = np.ascontiguousarray(ub, dtype=np.float64)
        self.n = self.q.shape[1]
        self.m = self.q.shape[0] - 1
        self.has_q0 = bool(has_q0)
        if A is not None and np.size(A) > 0:
            self.A = np.ascontiguousarray(np.atleast_2d(A), dtype=np.float64)
            self.b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
            self.p = self.A.shape[0]
        else:
            self.A = self.b = None
            self.p = 0
        if q_stored is not None:
            self.q_stored = np.ascontiguousarray(q_stored, dtype=np.int32)
            assert self.q_stored.shape == (self.m + 1,)
            nq = int(self.q_stored.sum())
        else:
            self.q_stored = None
            nq = self.m + (1 if self.has_q0 else 0)
        self.soc_dims = None if soc_dims is None else np.ascontiguousarray(soc_dims, dtype=np.int64)
        assert self.Q.shape == (nq, self.n, self.n), (self.Q.shape, nq, self.n)
        self._c = _Problem(self.n, self.m, self.p, self.Q.ctypes.data, dt, int(self.has_q0),
                           self.q.ctypes.data, self.c.ctypes.data,
                           self.A.ctypes.data if self.A is not None else None,
                           self.b.ctypes.data if self.b is not None else None,
                           self.lb.ctypes.data, self.ub.ctypes.data,
                           {"nonneg": 0, "simplex": 1, "cones": 2}[self.lambda_set], 0,
                           self.q0_shift, self.ball, self.ball_v, self.ball_l,
                           _ptr(self.q_stored),
                           0 if self.soc_dims is None else len(self.soc_dims),
                           _ptr(self.soc_dims))

    @property
    def ny(self):
        return self.p + self.m


def _host_q(Q):
    """Return (contiguous host array, dtype code); 16-bit torch tensors become raw uint16."""
    if hasattr(Q, "detach"):
        import torch
        t = Q.detach().to("cpu").contiguous()
        if t.dtype == torch.bfloat16:
            return t.view(torch.int16).numpy().view(np.uint16), 2
        if t.dtype == torch.float16:
            return t.view(torch.int16).numpy().view(np.uint16), 3
        if t.dtype == torch.float32:
            return t.numpy(), 1
        return t.to(torch.float64).numpy(), 0
    a = np.ascontiguousarray(Q)
    if a.dtype == np.float32:
        return a, 1
    if a.dtype == np.float16:
        return a.view(np.uint16), 3
    return np.ascontiguousarray(a, dtype=np.float64), 0


def _ptr(a):
    return None if a is None else a.ctypes.data


def operator(P: Problem, x, y=None):
    """U = [Q_i x], G = grad_y Phi(x) = (Ax-b, g(x)), f(x), grad_x Phi(x,y)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(P.ny) if y is None else np.ascontiguousarray(y, dtype=np.float64)
    U = np.empty((P.m + 1, P.n))
    G = np.empty(P.ny + 1)
    f = np.empty(1)
    gx = np.empty(P.n)
    lib().orc_operator(C.byref(P._c), _ptr(x), _ptr(y), _ptr(U), _ptr(G), _ptr(f), _ptr(gx))
    return dict(U=U, G=G[:P.ny].copy(), f=float(f[0]), grad=gx)


def project_dual(P: Problem, y):
    """Euclidean projection of y = (v, lambda) onto the problem's dual domain Y-hat."""
    out = np.array(y, dtype=np.float64, copy=True)
    lib().orc_project_dual(C.byref(P._c), _ptr(out))
    return out


def grad_from_u(P: Problem, U, y):
    U = np.ascontiguousarray(U, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    gx = np.empty(P.n)
    lib().orc_grad_from_u(C.byref(P._c), _ptr(U), _ptr(y), _ptr(gx))
    return gx


def kkt(P: Problem, x, y):
    """{rel_kkt, rel_dual, rel_pri, rel_comp, f, max_violation} at (x, y)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.empty(6)
    rc = lib().orc_kkt(C.byref(P._c), _ptr(x), _ptr(y), _ptr(out))
    if rc:
        raise MemoryError("oracle kkt")
    return dict(zip(("rel_kkt", "rel_dual", "rel_pri", "rel_comp", "f", "max_violation"),
                    map(float, out)))


def gap(P: Problem, x, y, xi=0.04, inner_tol=1e-12, max_inner=200000):
    """Self-centred smoothed duality gap: {G, Py, Px, inner_iters}."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.empty(4)
    rc = lib().orc_gap(C.byref(P._c), _ptr(x), _ptr(y), float(xi), float(inner_tol),
                       int(max_inner), _ptr(out))
    if rc:
        raise MemoryError("oracle gap")
    return dict(G=float(out[0]), Py=float(out[1]), Px=float(out[2]), inner_iters=int(out[3]))


STATUS = {0: "converged", 1: "invalid", 4: "not_converged", 5: "numerical"}


def solve(P: Problem, opts: Options = None, x0=None, y0=None, trace_cap: int = 0):
    """Run rAPDB; returns dict(x, y, info, trace)."""
    opts = opts or Options()
    x = np.empty(P.n)
    y = np.empty(max(P.ny, 1))
    info = _Info()
    x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    y0a = None if y0 is None else np.ascontiguousarray(y0, dtype=np.float64)
    tr = np.zeros((trace_cap, 5)) if trace_cap else None
    oc = opts._c()
    lib().orc_solve(C.byref(P._c), C.byref(oc), _ptr(x0a), _ptr(y0a), _ptr(x), _ptr(y),
                    C.byref(info), _ptr(tr), int(trace_cap))
    d = {k: getattr(info, k) for k, _ in _Info._fields_}
    d["status"] = STATUS.get(int(d["status"]), str(d["status"]))
    out = dict(x=x, y=y[:P.ny].copy(), info=d)
    if trace_cap:
        out["trace"] = tr[:min(trace_cap, d["iters"])]
    return out
