"""Write the stored reference solutions of the full-size workloads (calls only oracle/ and the
instance generators; nothing here touches the GPU library).

    python tests/golden/make_golden.py random_qcqp_n2000_m100    # ~10 min on one core
    python tests/golden/make_golden.py paper_random_n1000_m10    # four instances, one core each

random_qcqp_n2000_m100.json
    The random convex QCQP n = 2000, m = 100 (Q_i = A_i A_i'/n + 0.01 I, q_i ~ N(0, I),
    c_i ~ U(-1, -0.1), X = [-10, 10]^n) from random_qcqp_exact, whose matrices are
    bit-identical on any machine; the sha256 of its stack is stored so a test can prove it
    solved the same bytes.  The oracle's rAPDB-yx solve (non-monotone, fixed restarts every
    400 iterations, tau_bar = 1/||Q_0||_2, gamma_0 = 0.1) to relative KKT <= 1e-10 gives f*,
    x* and y*.

paper_random_n1000_m10.json
    The four random QCQPs of the §5.1 experiment's generator (n = 1000, m = 10, seeds
    config_seed(6, k)).  Their matrices come from a QR factorisation and products that may
    round differently on another machine, so each entry stores a fingerprint (sha256 of q and
    c, which are exact draws, and sum Q / sum |Q| per matrix to compare at 1e-12) beside the
    oracle's f* at relative KKT <= 1e-11.
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import qcqp_inputs as qi  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _sha(a) -> str:
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def random_qcqp_n2000_m100():
    n, m = 2000, 100
    t0 = time.time()
    inst = qi.random_qcqp_exact(n, m, qi.config_seed(2), shift=0.01)
    sha = qi.stack_sha256(inst.Q)
    L0 = float(np.linalg.norm(inst.Q[0], 2))
    print(f"generated in {time.time() - t0:.1f} s, sha256 {sha}, ||Q_0||_2 = {L0:.12g}", flush=True)
    opts = oracle.Options(tau_bar=1.0 / L0, gamma0=0.1, tol=1e-10, max_iter=50000)
    t0 = time.time()
    r = oracle.solve(oracle.Problem(inst), opts)
    secs = time.time() - t0
    info = r["info"]
    print(f"oracle: {info['status']} iters={info['iters']} trials={info['trials']} "
          f"rel_kkt={info['rel_kkt']:.3e} f={info['f']:.15g} in {secs:.0f} s", flush=True)
    assert info["status"] == "converged", info
    out = dict(
        workload="random convex QCQP n=2000 m=100 (random_qcqp_exact, config_seed(2), shift 0.01)",
        generator="qcqp_inputs.random_qcqp_exact(2000, 100, qcqp_inputs.config_seed(2), shift=0.01)",
        q_stack_sha256=sha, q_sha256=_sha(inst.q), c_sha256=_sha(inst.c),
        oracle_options=dict(variant="yx", c_nm=1, restart="fixed", restart_every=400,
                            tau_bar=1.0 / L0, gamma0=0.1, tol=1e-10),
        oracle_info={k: (v if isinstance(v, (int, str)) else float(v)) for k, v in info.items()},
        oracle_seconds=secs,
        f_star=float(info["f"]), x_star=[float(v) for v in r["x"]], y_star=[float(v) for v in r["y"]],
        command="python tests/golden/make_golden.py random_qcqp_n2000_m100")
    path = os.path.join(HERE, "random_qcqp_n2000_m100.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}", flush=True)


def paper_fingerprint(inst) -> dict:
    Q = np.asarray(inst.Q)
    return dict(q_sha256=_sha(inst.q), c_sha256=_sha(inst.c),
                q_sum=[float(Q[i].sum()) for i in range(Q.shape[0])],
                q_abs_sum=[float(np.abs(Q[i]).sum()) for i in range(Q.shape[0])])


def _paper_one(k):
    inst = qi.paper_random_qcqp(1000, 10, seed=qi.config_seed(6, k))
    L0 = float(np.linalg.norm(inst.Q[0], 2))
    opts = oracle.Options(tau_bar=1.0 / L0, gamma0=0.1, tol=1e-11, max_iter=400000)
    t0 = time.time()
    r = oracle.solve(oracle.Problem(inst), opts)
    info = r["info"]
    print(f"instance {k}: {info['status']} iters={info['iters']} rel_kkt={info['rel_kkt']:.3e} "
          f"f={info['f']:.15g} in {time.time() - t0:.0f} s", flush=True)
    assert info["status"] == "converged", info
    return dict(seed=qi.config_seed(6, k), fingerprint=paper_fingerprint(inst),
                f_star=float(info["f"]), oracle_iters=int(info["iters"]),
                oracle_rel_kkt=float(info["rel_kkt"]))


def paper_random_n1000_m10():
    with mp.Pool(4) as pool:
        rows = pool.map(_paper_one, range(4))
    out = dict(workload="the random QCQPs of the §5.1 experiment's generator, n=1000, m=10",
               generator="qcqp_inputs.paper_random_qcqp(1000, 10, seed=qcqp_inputs.config_seed(6, k))",
               oracle_options=dict(variant="yx", c_nm=1, restart="fixed", restart_every=400,
                                   tau_bar="1/||Q_0||_2", gamma0=0.1, tol=1e-11),
               instances=rows, command="python tests/golden/make_golden.py paper_random_n1000_m10")
    path = os.path.join(HERE, "paper_random_n1000_m10.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    targets = {"random_qcqp_n2000_m100": random_qcqp_n2000_m100,
               "paper_random_n1000_m10": paper_random_n1000_m10}
    for name in sys.argv[1:] or list(targets):
        targets[name]()
