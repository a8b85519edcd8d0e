"""ctypes binding of include/qcqp.h (argument marshalling only).

Every computation happens inside libqcqp_hip.so (hand-written HIP for gfx950).  There is no
Python or CPU fallback: if the library is missing or no GPU is visible, loading fails loudly.
PyTorch supplies device memory (tensors) and the stream, nothing else.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqcqp_hip.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_NOT_CONVERGED, E_NUMERICAL, E_NO_ROOM = range(7)
NOALLOC_MAX_N = 1024   # QCQP_NOALLOC_MAX_N of include/qcqp.h
STATUS_NAMES = {0: "ok", 1: "invalid", 2: "nomem", 3: "device", 4: "not_converged",
                5: "numerical", 6: "no_room"}
DTYPES = {"float64": 0, "float32": 1, "bfloat16": 2, "float16": 3}
RESTARTS = {"none": 0, "fixed": 1, "adaptive": 2}
PASS_MODES = {"auto": 0, "direct": 1, "incremental": 2}


class QCQPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("p", C.c_int64),
                ("Q", C.c_void_p), ("Q_dtype", C.c_int), ("ldq", C.c_int64), ("has_q0", C.c_int),
                ("q", C.c_void_p), ("c", C.c_void_p), ("A", C.c_void_p), ("b", C.c_void_p),
                ("lb", C.c_void_p), ("ub", C.c_void_p), ("on_device", C.c_int),
                ("lambda_set", C.c_int), ("q0_shift", C.c_double), ("ball", C.c_double),
                ("ball_v", C.c_double), ("ball_lambda", C.c_double), ("q_stored", C.c_void_p),
                ("n_soc", C.c_int64), ("soc_dims", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("variant", C.c_int), ("c_nm", C.c_int),
                ("eta", C.c_double), ("tau_bar", C.c_double), ("gamma0", C.c_double),
                ("mu", C.c_double), ("c_alpha", C.c_double), ("c_beta", C.c_double),
                ("delta", C.c_double),
                ("restart", C.c_int), ("restart_every", C.c_int64), ("restart_from_average", C.c_int),
                ("xi", C.c_double), ("q_restart", C.c_double), ("ada_first", C.c_int64),
                ("ada_every", C.c_int64), ("max_iter", C.c_int64), ("tol", C.c_double),
                ("storage", C.c_int), ("pass_mode", C.c_int), ("spec_trials", C.c_int),
                ("poll_every", C.c_int64), ("timing", C.c_int), ("inner_tol", C.c_double),
                ("max_inner", C.c_int64), ("use_graphs", C.c_int), ("stream", C.c_void_p),
                ("stop_rule", C.c_int), ("f_star", C.c_double), ("sym_pass", C.c_int)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("trials", C.c_int64), ("q_passes", C.c_int64),
                ("restarts", C.c_int64), ("gap_evals", C.c_int64), ("status", C.c_int64),
                ("rel_kkt", C.c_double), ("rel_dual", C.c_double), ("rel_pri", C.c_double),
                ("rel_comp", C.c_double), ("f", C.c_double), ("max_violation", C.c_double),
                ("seconds", C.c_double), ("pass_seconds", C.c_double), ("last_gap", C.c_double),
                ("pass_bytes", C.c_int64), ("timed_passes", C.c_int64), ("stop_value", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status"] = STATUS_NAMES.get(int(d["status"]), d["status"])
        return d


SYMBOLS = ["qcqp_options_default", "qcqp_last_error", "qcqp_create", "qcqp_solve",
           "qcqp_eval_operator", "qcqp_eval_trial_pass", "qcqp_eval_kkt", "qcqp_eval_gap",
           "qcqp_eval_gap_noalloc", "qcqp_destroy",
           "qcqp_batch_create", "qcqp_batch_admit", "qcqp_batch_step", "qcqp_batch_poll",
           "qcqp_batch_fetch", "qcqp_batch_stats", "qcqp_batch_pass_stats", "qcqp_batch_destroy",
           "qcqp_handle_bytes", "qcqp_time_pass"]

_LIB = None


def load(path: str = LIB_PATH):
    """Load the HIP library and declare signatures.  Raises if it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build()")
    # PyTorch (which supplies device memory and streams) carries its own HIP runtime.  Load it
    # first so that this library's libamdhip64.so.7 dependency resolves to that same runtime;
    # otherwise the process would hold two HIP runtimes and neither would see a device.
    import torch  # noqa: F401
    L = C.CDLL(path)
    vp, i64, st = C.c_void_p, C.c_int64, C.c_int
    P = C.POINTER
    L.qcqp_options_default.argtypes = [P(Options)]
    L.qcqp_options_default.restype = None
    L.qcqp_last_error.argtypes = []
    L.qcqp_last_error.restype = C.c_char_p
    L.qcqp_create.argtypes = [P(Problem), P(Options), P(vp)]
    L.qcqp_solve.argtypes = [vp, vp, vp, vp, vp, P(Info)]
    L.qcqp_eval_operator.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.qcqp_eval_trial_pass.argtypes = [vp, vp, vp, i64, vp]
    L.qcqp_eval_kkt.argtypes = [vp, vp, vp, vp]
    L.qcqp_eval_gap.argtypes = [vp, vp, vp, C.c_double, vp]
    L.qcqp_eval_gap_noalloc.argtypes = [vp, vp, vp, C.c_double, vp]
    L.qcqp_destroy.argtypes = [vp]
    L.qcqp_batch_create.argtypes = [P(Options), C.c_size_t, i64, P(vp)]
    L.qcqp_batch_admit.argtypes = [vp, vp, vp, vp, P(i64)]
    L.qcqp_batch_step.argtypes = [vp, i64]
    L.qcqp_batch_poll.argtypes = [vp, vp, i64, P(i64)]
    L.qcqp_batch_fetch.argtypes = [vp, i64, vp, vp, P(Info), P(vp)]
    L.qcqp_batch_stats.argtypes = [vp, P(i64), P(C.c_size_t)]
    L.qcqp_batch_pass_stats.argtypes = [vp, P(C.c_double), P(C.c_double), P(i64)]
    L.qcqp_batch_destroy.argtypes = [vp]
    L.qcqp_handle_bytes.argtypes = [vp]
    L.qcqp_handle_bytes.restype = C.c_size_t
    L.qcqp_time_pass.argtypes = [vp, i64, P(C.c_double)]
    for name in SYMBOLS:
        f = getattr(L, name)
        if name not in ("qcqp_options_default", "qcqp_last_error", "qcqp_handle_bytes"):
            f.restype = st
    _LIB = L
    return L


def check(code):
    if code != OK and code != E_NOT_CONVERGED:
        msg = load().qcqp_last_error().decode(errors="replace")
        raise QCQPError(code, msg)
    return code


def default_options(**kw) -> Options:
    o = Options()
    load().qcqp_options_default(C.byref(o))
    for k, v in kw.items():
        if k == "variant":
            v = {"yx": 0, "xy": 1}.get(v, v)
        elif k == "restart":
            v = RESTARTS.get(v, v)
        elif k == "storage":
            v = DTYPES.get(v, v)
        elif k == "pass_mode":
            v = PASS_MODES.get(v, v)
        elif k == "stop_rule":
            v = {"kkt": 0, "paper": 1}.get(v, v)
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o
