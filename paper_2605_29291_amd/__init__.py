"""rAPDB for convex QCQPs on MI355X (gfx950): thin Python layer over the C-ABI library.

    from paper_2605_29291_amd import Solver
    s = Solver(instance, storage="float64")        # uploads Q once (qcqp_create)
    x, y, info = s.solve()                         # device-resident rAPDB (qcqp_solve)
    out = s.eval_operator(x, y)                    # one Q-stack pass (qcqp_eval_operator)

Arrays may be numpy (host) or torch CUDA tensors (device); Q may be float64/float32/bfloat16/
float16.  All arithmetic runs in the HIP library; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import abi
from .abi import QCQPError, load

__all__ = ["Solver", "Batch", "QCQPError", "load", "abi"]


def _torch():
    import torch
    return torch


def _is_tensor(a):
    return hasattr(a, "data_ptr") and hasattr(a, "is_cuda")


def _q_dtype_code(Q):
    if _is_tensor(Q):
        torch = _torch()
        return {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2, torch.float16: 3}[Q.dtype]
    return {np.dtype(np.float64): 0, np.dtype(np.float32): 1, np.dtype(np.float16): 3}[np.asarray(Q).dtype]


def _current_stream():
    try:
        torch = _torch()
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return C.c_void_p(None)


class Solver:
    """One QCQP resident on the GPU (a qcqp_handle)."""

    def __init__(self, inst=None, *, Q=None, q=None, c=None, lb=None, ub=None, A=None, b=None,
                 has_q0=True, lambda_set=None, q0_shift=None, ball=0.0, ball_v=0.0,
                 ball_lambda=0.0, q_stored=None, soc_dims=None, device=None, **options):
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
        L = load()
        torch = _torch()
        if device is None:
            device = _is_tensor(Q) and Q.is_cuda
        self.on_device = bool(device)
        self.n = int(np.shape(q)[1])
        self.m = int(np.shape(q)[0]) - 1
        self.p = 0 if A is None or np.size(A) == 0 else int(np.shape(A)[0])
        self._keep = []

        def vec(a, shape=None):
            if a is None:
                return None
            if self.on_device:
                t = a if _is_tensor(a) else torch.as_tensor(np.asarray(a, dtype=np.float64))
                t = t.to(device="cuda", dtype=torch.float64).contiguous()
                if shape is not None:
                    t = t.reshape(shape)
                self._keep.append(t)
                return t.data_ptr()
            arr = np.ascontiguousarray(a.cpu().numpy() if _is_tensor(a) else a, dtype=np.float64)
            if shape is not None:
                arr = arr.reshape(shape)
            self._keep.append(arr)
            return arr.ctypes.data

        if self.on_device:
            Qt = Q if _is_tensor(Q) else torch.as_tensor(np.ascontiguousarray(Q))
            Qt = Qt.to("cuda").contiguous()
            qptr = Qt.data_ptr()
            qcode = _q_dtype_code(Qt)
            self._keep.append(Qt)
        else:
            if _is_tensor(Q):
                Qt = Q.detach().cpu().contiguous()
                qcode = _q_dtype_code(Qt)
                self._keep.append(Qt)
                qptr = Qt.data_ptr()
            else:
                Qa = np.ascontiguousarray(Q)
                qcode = _q_dtype_code(Qa)
                self._keep.append(Qa)
                qptr = Qa.ctypes.data
        qs = None if q_stored is None else np.ascontiguousarray(q_stored, dtype=np.int32)
        sd = None if soc_dims is None else np.ascontiguousarray(soc_dims, dtype=np.int64)
        self._keep += [a for a in (qs, sd) if a is not None]
        prob = abi.Problem(self.n, self.m, self.p, qptr, qcode, 0, 1 if has_q0 else 0,
                           vec(q), vec(c), vec(A) if self.p else None, vec(b) if self.p else None,
                           vec(lb), vec(ub), 1 if self.on_device else 0,
                           {"nonneg": 0, "simplex": 1, "cones": 2}[lambda_set], float(q0_shift),
                           float(ball), float(ball_v), float(ball_lambda),
                           None if qs is None else qs.ctypes.data,
                           0 if sd is None else len(sd), None if sd is None else sd.ctypes.data)
        if "stream" not in options:
            options["stream"] = _current_stream()
        self.options = abi.default_options(**options)
        h = C.c_void_p()
        abi.check(L.qcqp_create(C.byref(prob), C.byref(self.options), C.byref(h)))
        self._h = h
        self._keep = []         # the library copied everything
        if self.on_device:
            torch.cuda.synchronize()

    # -- helpers -------------------------------------------------------------------------
    def _in(self, a, size):
        if a is None:
            return None, None
        if self.on_device:
            torch = _torch()
            t = (a if _is_tensor(a) else torch.as_tensor(np.asarray(a, dtype=np.float64)))
            t = t.to(device="cuda", dtype=torch.float64).contiguous().reshape(-1)
            assert t.numel() == size
            return t, t.data_ptr()
        arr = np.ascontiguousarray(a.cpu().numpy() if _is_tensor(a) else a, dtype=np.float64).reshape(-1)
        assert arr.size == size
        return arr, arr.ctypes.data

    def _out(self, *shape):
        if self.on_device:
            torch = _torch()
            t = torch.empty(shape, dtype=torch.float64, device="cuda")
            return t, t.data_ptr()
        a = np.empty(shape)
        return a, a.ctypes.data

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("solver is closed or owned by a batch")
        return self._h

    # -- API -----------------------------------------------------------------------------
    def solve(self, x0=None, y0=None):
        L = load()
        xk, xp = self._in(x0, self.n)
        yk, yp = self._in(y0, self.p + self.m)
        x, xo = self._out(self.n)
        y, yo = self._out(max(self.p + self.m, 1))
        info = abi.Info()
        abi.check(L.qcqp_solve(self.handle, xp, yp, xo, yo, C.byref(info)))
        return x, y[: self.p + self.m], info.as_dict()

    def eval_operator(self, x, y=None):
        L = load()
        xk, xp = self._in(x, self.n)
        yk, yp = self._in(y, self.p + self.m)
        U, Up = self._out(self.m + 1, self.n)
        g, gp = self._out(max(self.m, 1))
        f, fp = self._out(1)
        gr, grp = self._out(self.n)
        abi.check(L.qcqp_eval_operator(self.handle, xp, yp, Up, gp, fp, grp))
        return dict(U=U, g=g[: self.m], f=f, grad=gr)

    def eval_trial_pass(self, x, xc):
        """The trial group's Q pass at iterate x for the spec_trials points xc (rows):
        [Q_i x_b] (direct mode) or [Q_i (x_b - x)] (incremental mode), shape (B, m+1, n)."""
        L = load()
        B = int(self.options.spec_trials)
        xk, xp = self._in(x, self.n)
        ck, cp = self._in(xc, B * self.n)
        out, op = self._out(B, self.m + 1, self.n)
        abi.check(L.qcqp_eval_trial_pass(self.handle, xp, cp, B, op))
        return out

    def eval_kkt(self, x, y=None):
        L = load()
        xk, xp = self._in(x, self.n)
        yk, yp = self._in(y, self.p + self.m)
        out = np.empty(6)
        abi.check(L.qcqp_eval_kkt(self.handle, xp, yp, out.ctypes.data))
        return dict(zip(("rel_kkt", "rel_dual", "rel_pri", "rel_comp", "f", "max_violation"),
                        map(float, out)))

    def eval_gap(self, x, y=None, xi=0.04, noalloc=False):
        """G_xi at (x, y); noalloc=True calls qcqp_eval_gap_noalloc (n <= abi.NOALLOC_MAX_N)."""
        L = load()
        xk, xp = self._in(x, self.n)
        yk, yp = self._in(y, self.p + self.m)
        out = np.empty(4)
        fn = L.qcqp_eval_gap_noalloc if noalloc else L.qcqp_eval_gap
        abi.check(fn(self.handle, xp, yp, float(xi), out.ctypes.data))
        return dict(G=float(out[0]), Py=float(out[1]), Px=float(out[2]), inner_iters=int(out[3]))

    def time_pass(self, reps=20):
        L = load()
        v = C.c_double()
        abi.check(L.qcqp_time_pass(self.handle, int(reps), C.byref(v)))
        return v.value

    def nbytes(self):
        return int(load().qcqp_handle_bytes(self.handle))

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().qcqp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Continuous batching: resident solves advanced together (qcqp_batch_*)."""

    def __init__(self, max_slots=64, hbm_budget_bytes=0, **options):
        L = load()
        if "stream" not in options:
            options["stream"] = _current_stream()
        self.options = abi.default_options(**options)
        b = C.c_void_p()
        abi.check(L.qcqp_batch_create(C.byref(self.options), int(hbm_budget_bytes), int(max_slots),
                                      C.byref(b)))
        self._b = b
        self._solvers = {}

    def admit(self, solver: Solver, x0=None, y0=None):
        """Returns the slot id, or None when there is no room (slot or HBM budget)."""
        L = load()
        xk, xp = solver._in(x0, solver.n)
        yk, yp = solver._in(y0, solver.p + solver.m)
        slot = C.c_int64()
        code = L.qcqp_batch_admit(self._b, solver.handle, xp, yp, C.byref(slot))
        if code == abi.E_NO_ROOM:
            return None
        abi.check(code)
        self._solvers[slot.value] = solver
        solver._owned_h, solver._h = solver._h, None
        return slot.value

    def step(self, groups=8):
        abi.check(load().qcqp_batch_step(self._b, int(groups)))

    def poll(self, cap=4096):
        arr = np.empty(cap, dtype=np.int64)
        n = C.c_int64()
        abi.check(load().qcqp_batch_poll(self._b, arr.ctypes.data, int(cap), C.byref(n)))
        return [int(v) for v in arr[: n.value]]

    def fetch(self, slot):
        L = load()
        s = self._solvers.pop(slot)
        x, xo = s._out(s.n)
        y, yo = s._out(max(s.p + s.m, 1))
        info = abi.Info()
        h = C.c_void_p()
        abi.check(L.qcqp_batch_fetch(self._b, int(slot), xo, yo, C.byref(info), C.byref(h)))
        s._h = s._owned_h
        s._owned_h = None
        return s, x, y[: s.p + s.m], info.as_dict()

    def stats(self):
        r = C.c_int64()
        b = C.c_size_t()
        abi.check(load().qcqp_batch_stats(self._b, C.byref(r), C.byref(b)))
        return dict(running=r.value, resident_bytes=b.value)

    def pass_stats(self):
        sec, byt, n = C.c_double(), C.c_double(), C.c_int64()
        abi.check(load().qcqp_batch_pass_stats(self._b, C.byref(sec), C.byref(byt), C.byref(n)))
        return dict(pass_seconds=sec.value, pass_bytes=byt.value, passes=n.value)

    def close(self):
        if getattr(self, "_b", None) is not None:
            load().qcqp_batch_destroy(self._b)
            for s in self._solvers.values():
                s._owned_h = None
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
