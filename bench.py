"""Benchmark: rAPDB solves/s and Q-pass HBM bandwidth on one MI355X.

Default line: random convex QCQP, n = 2000, m = 100, Q_i = A_i A_i'/n + 0.01 I, q_i ~ N(0,I),
c_i ~ U(-1,-0.1), box [-10,10]^n, FP64 Q stack (3.23 GB; 1.62 GB as packed upper triangles),
solved to relative KKT <= 1e-6 by rAPDB-yx (non-monotone, fixed restarts every 400 iterations,
3 speculative candidates per pass).  A "step" is one complete solve (every part of the hot path:
Q-stack passes, epilogues, projections, backtracking tests, step-size/averaging bookkeeping,
restarts, KKT stop test) with the instance already resident in HBM.  Beside the headline the
same JSON line carries the pass roofline, the oracle's CPU baseline, the objective against the
oracle's stored solution, and (unless --quick) sections for the n=100 m=10 workload, serving
(512 BF16 requests, continuous batching, Poisson arrivals, FP64 FIFO comparison) and the
n=4000 m=200 BF16/FP16 precision form.  Printed as ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
                    [--workload config2|serving|precision|kml|kml_minmax|paper_random|batch_pass|small|traffic]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "QCQP solves/s & Q-pass HBM GB/s at rel-KKT<=1e-6; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pass_source_hash(csrc):
    """sha256 over the pass kernel's source and the device layout it reads."""
    import hashlib
    h = hashlib.sha256()
    for f in ("qpass.hip", "qcqp_device.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def measured_traffic(key):
    """HBM bytes per pass launch from the committed FETCH_SIZE/WRITE_SIZE summary, or None when
    the kernel source changed since those counters were taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "k_pass_traffic_random_qcqp_n2000_m100.md")
    csrc = os.path.join(ROOT, "paper_2605_29291_amd", "csrc")
    try:
        fields = dict(line.split(": ", 1) for line in open(prof).read().splitlines() if ": " in line
                      and line.split(": ", 1)[0] in ("kernel_source_sha256", key))
        cur = pass_source_hash(csrc)
        if fields.get("kernel_source_sha256", "").strip() != cur:
            return None
        return float(fields[key])
    except (OSError, KeyError, ValueError):
        return None


def spectral_norm_gpu(Q0):
    import torch
    return float(torch.linalg.eigvalsh(Q0.to(torch.float64)).abs().max())


def run_solves(solver, steps, warmup):
    import torch
    for _ in range(warmup):
        solver.solve()
    torch.cuda.synchronize()
    lat, infos = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        t = time.perf_counter()
        x, y, info = solver.solve()
        lat.append(time.perf_counter() - t)
        infos.append(info)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, lat, infos, x, y


def pass_stats(infos):
    ps = sum(i["pass_seconds"] for i in infos)
    tp = sum(i["timed_passes"] for i in infos)
    avg = ps / max(tp, 1)
    return avg, tp


def cpu_baseline(inst_host, tau_bar, gamma0, trials_per_solve, budget_s=30.0):
    """The oracle (plain single-threaded FP64 C) on a bounded sample of the same workload:
    rAPDB iterations of the same instance until ~budget_s of CPU time, then scaled to a solve
    by the trial count the full solve needs (every trial costs one Q-stack pass)."""
    import oracle
    P = oracle.Problem(inst_host)
    it = 1
    while True:
        t = time.perf_counter()
        r = oracle.solve(P, oracle.Options(tau_bar=tau_bar, gamma0=gamma0, max_iter=it, tol=0.0))
        dt = time.perf_counter() - t
        # stop once the sample is at least half the budget or the next doubling would exceed it
        if dt >= budget_s / 2 or 2 * dt > budget_s or it >= 256:
            break
        it *= 2
    trials = r["info"]["trials"]
    per_trial = dt / max(trials, 1)
    solves_per_s = 1.0 / (per_trial * trials_per_solve)
    return dict(value=solves_per_s, unit="solves/s", cores=1, kind="oracle",
                sample=f"{it} rAPDB iterations ({trials} trials, {dt:.1f} s) of the same instance on "
                       f"one host core; solves/s = 1 / (s per trial x {trials_per_solve} trials per "
                       f"solve, the GPU solve's count)")


def cpu_info():
    """The host the CPU baselines run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return dict(cpu_model=model, nproc=os.cpu_count(), cores_available=avail)


def cpu_workers():
    """Oracle processes for the throughput baselines: the cores this job may use, at most 16."""
    return max(1, min(16, cpu_info()["cores_available"] or 1))


def run_threads(jobs, workers):
    """Run the callables in `workers` threads; the oracle's C calls release the GIL, so each
    thread is one single-threaded oracle on its own core."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda f: f(), jobs))


def stream_ceilings(Q):
    """Context for the pass's roofline fraction: what plain library streams reach on the same
    device -- a device-to-device copy of 2 GiB (read + write bytes) and torch's sum over the
    resident FP64 stack (read only), best of 5 each, timed with events."""
    import torch
    out = {}
    src = torch.empty(2 ** 30 // 4, dtype=torch.float64, device="cuda")   # 2 GiB
    src.fill_(1.0)
    dst = torch.empty_like(src)
    for name, fn, nbytes in (("d2d_copy_read_plus_write_GBs", lambda: dst.copy_(src), 2 * src.numel() * 8),
                             ("torch_sum_read_GBs", lambda: Q.sum(), Q.numel() * Q.element_size())):
        best = 1e9
        for _ in range(6):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b) * 1e-3)
        out[name] = nbytes / best / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


# speculative candidates per pass for the config-2 solves: the iterates and trial counts are
# those of sequential backtracking for any value; 3 streams 60 passes per solve instead of 67
CONFIG2_SPEC = 3
# candidates for the packed symmetric pass, whose per-wave registers grow with B
CONFIG2_SYM_SPEC = 3


def workload_config2(args):
    """The default bench line.  Three solvers over the same FP64 instance: the packed symmetric
    pass (options.sym_pass, the line's value), the row-major FP64 pass and FP32 storage (both
    reported beside it)."""
    import torch
    import qcqp_inputs as qi
    from paper_2605_29291_amd import Solver
    n, m = 2000, 100
    log(f"generating n={n} m={m} on the GPU")
    inst = qi.random_qcqp_exact(n, m, qi.config_seed(2), shift=0.01, device="cuda")
    L0 = spectral_norm_gpu(inst.Q[0])
    tau_bar, gamma0 = 1.0 / L0, 0.1
    res = {}
    for name, storage, sym in (("sym", "float64", 1), ("float64", "float64", 0), ("float32", "float32", 0)):
        spec = CONFIG2_SYM_SPEC if sym else CONFIG2_SPEC
        Qs = inst.Q if storage == "float64" else inst.Q.to(torch.float32)
        inst_s = qi.Instance(n, m, 0, Qs, inst.q, inst.c, inst.lb, inst.ub)
        s = Solver(inst_s, device=True, storage=storage, tau_bar=tau_bar, gamma0=gamma0, timing=1,
                   spec_trials=spec, sym_pass=sym)
        if storage != "float64":
            del Qs
        wall, lat, infos, x, y = run_solves(s, args.steps, args.warmup)
        avg_pass, tp = pass_stats(infos)
        pb = infos[0]["pass_bytes"]
        ok = all(i["status"] == "ok" and i["rel_kkt"] <= 1e-6 for i in infos)
        res[name] = dict(wall=wall, lat=lat, infos=infos, avg_pass=avg_pass, timed=tp,
                         pass_bytes=pb, ok=ok, x=x.cpu().numpy(), y=y.cpu().numpy(), spec=spec)
        log(f"{name}: {args.steps} solves in {wall:.3f} s; iters={infos[0]['iters']} "
            f"trials={infos[0]['trials']} passes={infos[0]['q_passes']} rel_kkt={infos[0]['rel_kkt']:.2e} "
            f"pass {avg_pass * 1e6:.1f} us = {pb / avg_pass / 1e9:.0f} GB/s")
        s.close()
    r = res["sym"]
    ceilings = stream_ceilings(inst.Q)
    Qhost = inst.Q.cpu().numpy()
    inst_h = qi.Instance(n, m, 0, Qhost, inst.q, inst.c, inst.lb, inst.ub)
    del inst
    torch.cuda.empty_cache()
    # result check by the oracle's own KKT evaluation (one host pass)
    import oracle
    kk = oracle.kkt(oracle.Problem(inst_h), r["x"], r["y"])
    cpu = None
    if not args.no_cpu:
        cpu = dict(cpu_baseline(inst_h, tau_bar, gamma0, r["infos"][0]["trials"]), **cpu_info())
    # the objective against the oracle's own solve of this instance (stored by
    # tests/golden/make_golden.py; the instance hash proves it is the same one)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "random_qcqp_n2000_m100.json")))
    same = qi.stack_sha256(inst_h.Q) == gold["q_stack_sha256"]
    xs = np.array(gold["x_star"])
    vs_oracle = dict(instance_matches=same, f_star=gold["f_star"],
                     f_rel_err=abs(kk["f"] - gold["f_star"]) / (1 + abs(gold["f_star"])),
                     x_rel_err=float(np.linalg.norm(r["x"] - xs) / (1 + np.linalg.norm(xs))),
                     oracle_rel_kkt=gold["oracle_info"]["rel_kkt"])
    del inst_h, Qhost
    solves_s = args.steps / r["wall"]
    lat_ms = np.array(r["lat"]) * 1e3
    achieved = r["pass_bytes"] / r["avg_pass"] / 1e9

    def side(rr):
        gbs = rr["pass_bytes"] / rr["avg_pass"] / 1e9
        return {"solves_per_s": args.steps / rr["wall"], "q_pass_us": rr["avg_pass"] * 1e6,
                "q_pass_bytes": rr["pass_bytes"], "q_pass_GBs": gbs, "q_pass_frac": gbs / HBM_PEAK_GBS,
                "iters": rr["infos"][0]["iters"], "q_passes": rr["infos"][0]["q_passes"],
                "rel_kkt": rr["infos"][0]["rel_kkt"], "all_converged": rr["ok"], "spec_trials": rr["spec"]}

    out = {
        "metric": METRIC,
        "value": solves_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "random convex QCQP n=2000 m=100, Q_i=A_iA_i'/n+0.01I, FP64 (3.23 GB "
                               "row-major, 1.62 GB upper triangles), rAPDB-yx non-monotone, fixed "
                               "restart 400, rel-KKT<=1e-6",
                   "n": 2000, "m": 100, "storage": "float64", "sym_pass": 1,
                   "spec_trials": CONFIG2_SYM_SPEC, "tau_bar": tau_bar, "gamma0": gamma0},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("traffic_bytes_per_launch_f64_sym"),
                     "traffic_unit": "bytes per pass (rocprofv3 FETCH_SIZE + WRITE_SIZE of k_spass and "
                                     "k_sred, copy-calibrated)",
                     "kernel": f"k_spass<{CONFIG2_SYM_SPEC}> + k_sred<{CONFIG2_SYM_SPEC}> (packed upper-triangle "
                               "tiles; algorithmic bytes (m+1) n(n+1)/2 x 8)",
                     "avg_pass_us": r["avg_pass"] * 1e6, "bytes_per_pass": r["pass_bytes"],
                     "timed_passes": r["timed"]},
        "cpu_baseline": cpu,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "solve": {"iters": r["infos"][0]["iters"], "trials": r["infos"][0]["trials"],
                  "q_passes": r["infos"][0]["q_passes"], "rel_kkt": r["infos"][0]["rel_kkt"],
                  "rel_kkt_oracle_eval": kk["rel_kkt"], "f": kk["f"], "all_converged": r["ok"]},
        "stream_ceilings": ceilings,
        "row_major_fp64": dict(side(res["float64"]),
                               traffic=measured_traffic("traffic_bytes_per_launch_f64")),
        "fp32_storage": side(res["float32"]),
        "objective_vs_oracle_solution": vs_oracle,
    }
    if not args.quick:
        t = time.perf_counter()
        out["config1"] = config1_section(args)
        log(f"config 1 section {time.perf_counter() - t:.0f} s")
        t = time.perf_counter()
        out["serving"] = serving_section(args)
        log(f"serving section {time.perf_counter() - t:.0f} s")
        t = time.perf_counter()
        out["precision"] = precision_section(args)
        log(f"precision section {time.perf_counter() - t:.0f} s")
    return out


# ----------------------------------------------------------------------------------------------
# sections of the default line beside the config-2 headline

def config1_section(args):
    """Random convex QCQP n=100, m=10 (0.88 MB FP64 stack, cache-resident): single-solve
    latency on the GPU, 100 instances as one batch, and P oracle threads solving instances of
    the same recipe (throughput baseline, P = cores available, at most 16)."""
    import torch
    import oracle
    import qcqp_inputs as qi
    from paper_2605_29291_amd import Batch, Solver
    insts = [qi.random_qcqp(100, 10, qi.config_seed(1, k)) for k in range(100)]
    tb = [1.0 / float(np.linalg.norm(i.Q[0], 2)) for i in insts]
    s = Solver(insts[0], device=True, tau_bar=tb[0], gamma0=0.1)
    for _ in range(3):
        s.solve()
    lat = []
    for _ in range(50):
        t = time.perf_counter()
        x, y, info = s.solve()
        lat.append(time.perf_counter() - t)
    s.close()
    single = dict(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                  solves_per_s=1.0 / float(np.mean(lat)), iters=info["iters"], q_passes=info["q_passes"],
                  rel_kkt=info["rel_kkt"], status=info["status"])
    solvers = [Solver(inst, device=True, tau_bar=t, gamma0=0.1) for inst, t in zip(insts, tb)]
    torch.cuda.synchronize()
    b = Batch(max_slots=len(insts))
    t0 = time.perf_counter()
    for sv in solvers:
        b.admit(sv)
    infos = []
    while len(infos) < len(insts):
        b.step(16)
        for slot in b.poll():
            infos.append(b.fetch(slot)[3])
    wall = time.perf_counter() - t0
    b.close()
    ok = sum(i["status"] == "ok" and i["rel_kkt"] <= 1e-6 for i in infos)
    batched = dict(instances=len(insts), seconds=wall, solves_per_s=ok / wall, converged=ok)
    log(f"config 1: single {single}; batched {batched}")
    # CPU: P oracle threads, each solving instances of the recipe to relative KKT 1e-6
    P = cpu_workers()
    probs = [oracle.Problem(i) for i in insts]
    budget = 10.0

    def job(w):
        def run():
            times, k = [], w
            t_end = time.perf_counter() + budget
            while time.perf_counter() < t_end:
                t = time.perf_counter()
                r = oracle.solve(probs[k % len(probs)], oracle.Options(tau_bar=tb[k % len(probs)], gamma0=0.1))
                times.append((time.perf_counter() - t, r["info"]["status"] == "converged"))
                k += P
            return times
        return run

    t0 = time.perf_counter()
    res = run_threads([job(w) for w in range(P)], P)
    wall = time.perf_counter() - t0
    all_t = [t for r in res for t, ok_ in r if ok_]
    cpu = dict(value=len(all_t) / wall, unit="solves/s", cores=P, kind="oracle",
               sample=f"{P} oracle threads (one core each) solving n=100, m=10 instances of the same "
                      f"recipe to relative KKT 1e-6 for {budget:.0f} s: {len(all_t)} solves",
               per_solve_ms_p50=float(np.percentile(np.array(all_t) * 1e3, 50)) if all_t else None,
               **cpu_info())
    return dict(workload="random convex QCQP n=100 m=10, FP64 (0.88 MB stack, cache-resident)",
                gpu_single=single, gpu_batch_of_100=batched, cpu_baseline=cpu)


def serving_section(args, requests=512, check=16):
    """Serving (continuous batching): `requests` random QCQP requests n~U[200,3000],
    m~U[5,200], BF16 stacks, FP64 checks.  Closed loop (all at t=0) with pass events (for the
    pass roofline) and with graph replay (the throughput), then Poisson arrivals at 0.7 x the
    closed-loop rate, and the same Poisson trace through the plain FP64 single-instance path one
    request at a time.  Latency includes admission (qcqp_create); instance synthesis does not.
    A subset is checked by the oracle on the stored instances, and P oracle threads give the
    CPU throughput on requests of the trace (bounded sample, scaled by the GPU trial counts)."""
    import torch
    import oracle
    import qcqp_inputs as qi
    free, _ = torch.cuda.mem_get_info()
    budget = int(free - 24e9)
    args.check = max(args.check, check)
    trace = qi.serving_trace(requests, qi.config_seed(5), rate=None)
    reqs_t, total_t, gen_t, ps = serve_batched(trace, "bfloat16", args, budget, timing=1)
    timed = _lat_summary(reqs_t, total_t)
    gbs = ps["pass_bytes"] / ps["pass_seconds"] / 1e9 if ps["pass_seconds"] > 0 else None
    log(f"serving closed loop, pass events: {timed}  pass {gbs} GB/s")
    reqs, total, gen, _ = serve_batched(trace, "bfloat16", args, budget, timing=0)
    closed = _lat_summary(reqs, total)
    log(f"serving closed loop, graphs: {closed}")
    rate = 0.7 * closed["solves_per_s"]
    trace_p = qi.serving_trace(requests, qi.config_seed(5), rate=rate)
    reqs_p, total_p, gen_p, _ = serve_batched(trace_p, "bfloat16", args, budget, timing=0)
    poisson = _lat_summary(reqs_p, total_p)
    log(f"serving Poisson {rate:.1f}/s: {poisson}")
    reqs_f, total_f, gen_f = serve_fifo(trace_p, "float64", args)
    fifo = _lat_summary(reqs_f, total_f)
    log(f"FP64 single-instance FIFO, same trace: {fifo}")
    # oracle: relative KKT of GPU results on the stored (BF16) instances
    checks = []
    for r in reqs[:check]:
        inst = _gen_request(r, "bfloat16")
        host = qi.Instance(inst.n, inst.m, 0, inst.Q.cpu(), inst.q, inst.c, inst.lb, inst.ub)
        del inst
        kk = oracle.kkt(oracle.Problem(host), r["x"], r["y"])
        checks.append(dict(n=r["n"], m=r["m"], rel_kkt_oracle=kk["rel_kkt"], gpu_rel_kkt=r["info"]["rel_kkt"]))
    torch.cuda.empty_cache()
    # CPU: P oracle threads on the first P requests, a few iterations each
    P = cpu_workers()
    hosts = []
    for r in reqs[:P]:
        inst = _gen_request(r, "bfloat16")
        hosts.append((qi.Instance(inst.n, inst.m, 0, inst.Q.cpu(), inst.q, inst.c, inst.lb, inst.ub),
                      r["info"]["trials"]))
        del inst
    torch.cuda.empty_cache()

    def job(h, trials_full):
        def run():
            Pr = oracle.Problem(h)
            it = 1
            while True:
                t = time.perf_counter()
                rr = oracle.solve(Pr, oracle.Options(tau_bar=0.1, gamma0=0.1, max_iter=it, tol=0.0))
                dt = time.perf_counter() - t
                if dt >= 6.0 or it >= 64:
                    break
                it *= 2
            return dt / max(rr["info"]["trials"], 1) * trials_full
        return run

    t0 = time.perf_counter()
    est = run_threads([job(h, tr) for h, tr in hosts], P)
    cpu_wall = time.perf_counter() - t0
    cpu = dict(value=P / float(np.mean(est)), unit="solves/s", cores=P, kind="oracle",
               sample=f"{P} oracle threads (one core each), each on one request of the trace (BF16 "
                      f"stack read by the oracle) for a bounded number of iterations ({cpu_wall:.0f} s); "
                      f"seconds per solve = seconds per trial x the GPU's trial count for that request",
               per_solve_s_mean=float(np.mean(est)), **cpu_info())
    del hosts
    return dict(
        workload=f"serving: {requests} random QCQP requests n~U[200,3000], m~U[5,200], BF16 stack "
                 "(FP32 accumulation, FP64 tests/restarts/KKT), continuous batching admitted by free HBM",
        closed_loop=closed, closed_loop_with_pass_events=timed, poisson=dict(poisson, rate_per_s=rate),
        fp64_single_instance_fifo=fifo,
        pass_roofline={"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": gbs / HBM_PEAK_GBS if gbs else None,
                       "kernel": _batch_pass_kernel(args) + " over all resident requests"},
        oracle_checks=checks, max_oracle_rel_kkt=max(c["rel_kkt_oracle"] for c in checks),
        instance_synthesis_s=gen, cpu_baseline=cpu, budget_bytes=budget, spec_trials=args.spec,
        groups_per_step=args.groups)


def precision_section(args, solves=3):
    """Random convex QCQP n=4000, m=200 stored BF16 and FP16 (6.43 GB), FP32 accumulation, FP64
    tests/restarts/KKT; the oracle's relative KKT of each result on the stored instance, and the
    distance from the FP64 solution of the unrounded instance (the FP64 path on a 25.7 GB stack)."""
    import torch
    import oracle
    import qcqp_inputs as qi
    from paper_2605_29291_amd import Solver
    n, m = 4000, 200
    inst64 = qi.random_qcqp_torch(n, m, qi.config_seed(3), shift=0.01, device="cuda")
    tau_bar = 1.0 / spectral_norm_gpu(inst64.Q[0])
    s64 = Solver(inst64, device=True, storage="float64", tau_bar=tau_bar, gamma0=0.1, timing=1)
    x64, y64, i64 = s64.solve()
    x64n = x64.cpu().numpy()
    out = {}
    for storage in ("bfloat16", "float16"):
        Qr = inst64.Q.to({"bfloat16": torch.bfloat16, "float16": torch.float16}[storage])
        instr = qi.Instance(n, m, 0, Qr, inst64.q, inst64.c, inst64.lb, inst64.ub)
        s = Solver(instr, device=True, storage=storage, tau_bar=tau_bar, gamma0=0.1, timing=1)
        wall, lat, infos, x, y = run_solves(s, solves, 1)
        avg_pass, _ = pass_stats(infos)
        pb = infos[0]["pass_bytes"]
        kk_unrounded = s64.eval_kkt(x, y)
        xr = x.cpu().numpy()
        s.close()
        # the packed 16-bit pass (sym_pass): upper-triangle tiles of the stored values
        sp = Solver(instr, device=True, storage=storage, tau_bar=tau_bar, gamma0=0.1, timing=1, sym_pass=1)
        wall_p, lat_p, infos_p, xp, yp = run_solves(sp, solves, 1)
        # trial passes at the solve's last candidate points (a fresh handle's candidates are no
        # step of the method, and its passes ran up to 13 % faster than the passes in solves)
        sp_pass = min(sp.time_pass(10) for _ in range(2))
        sp.close()
        pb_p = infos_p[0]["pass_bytes"]
        xpn, ypn = xp.cpu().numpy(), yp.cpu().numpy()
        host = qi.Instance(n, m, 0, Qr.cpu(), inst64.q, inst64.c, inst64.lb, inst64.ub)
        del Qr, instr
        torch.cuda.empty_cache()
        kk = oracle.kkt(oracle.Problem(host), xr, y.cpu().numpy())
        kk_p = oracle.kkt(oracle.Problem(host), xpn, ypn)
        del host
        out[storage] = dict(
            solves_per_s=solves / wall, p50_ms=float(np.percentile(np.array(lat) * 1e3, 50)),
            iters=infos[0]["iters"], q_passes=infos[0]["q_passes"], rel_kkt=infos[0]["rel_kkt"],
            rel_kkt_oracle_on_stored=kk["rel_kkt"], f=kk["f"],
            all_converged=all(i["status"] == "ok" and i["rel_kkt"] <= 1e-6 for i in infos),
            pass_roofline={"bound": "hbm", "achieved": pb / avg_pass / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": pb / avg_pass / 1e9 / HBM_PEAK_GBS, "us": avg_pass * 1e6, "bytes": pb,
                           "kernel": "k_pass<16-bit, 2> (incremental: W = [Q_i d] in FP32 per lane, FP64 across)"},
            error_vs_fp64_unrounded=dict(
                x_rel=float(np.linalg.norm(xr - x64n) / (1 + np.linalg.norm(x64n))),
                f_rel=float(abs(kk_unrounded["f"] - i64["f"]) / (1 + abs(i64["f"]))),
                rel_kkt_on_unrounded=kk_unrounded["rel_kkt"]),
            packed_pass=dict(
                solves_per_s=solves / wall_p, p50_ms=float(np.percentile(np.array(lat_p) * 1e3, 50)),
                iters=infos_p[0]["iters"], q_passes=infos_p[0]["q_passes"],
                rel_kkt_oracle_on_stored=kk_p["rel_kkt"], f=kk_p["f"],
                all_converged=all(i["status"] == "ok" and i["rel_kkt"] <= 1e-6 for i in infos_p),
                pass_roofline={"bound": "hbm", "achieved": pb_p / sp_pass / 1e9, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": pb_p / sp_pass / 1e9 / HBM_PEAK_GBS,
                               "us": sp_pass * 1e6, "bytes": pb_p,
                               "kernel": "k_spass16<16-bit, 2> + k_sred16 (packed upper triangles, "
                                         "(m+1) n(n+1)/2 x 2 bytes; trial passes)"}))
        log(f"precision {storage}: {out[storage]}")
    s64.close()
    del inst64
    torch.cuda.empty_cache()
    return dict(workload="random convex QCQP n=4000 m=200, Q_i=A_iA_i'/n+0.01I stored BF16 / FP16 "
                         "(6.43 GB), FP32 accumulation, FP64 test/restart/KKT",
                per_storage=out,
                fp64_unrounded_reference=dict(iters=i64["iters"], rel_kkt=i64["rel_kkt"], f=i64["f"],
                                              pass_GBs=i64["pass_bytes"] / (i64["pass_seconds"] / max(i64["timed_passes"], 1)) / 1e9))


# ----------------------------------------------------------------------------------------------
# other workloads (not the default bench line): --workload serving | precision | kml

def _est_bytes(n, m, storage, B=2, sym=0):
    es = {"float64": 8, "float32": 4, "bfloat16": 2, "float16": 2}[storage]
    ld = -(-n // (128 // es)) * (128 // es)
    inc = 0 if storage == "float64" else B
    packed = 0
    if sym:
        nt = -(-n // 256)
        packed = (m + 1) * nt * (nt + 1) // 2 * (256 * 256 * 2 + 2 * B * 256 * 4)
    return (m + 1) * n * ld * es + packed + 8 * (m + 1) * n * (3 + B + inc) + (4 << 20)


def _sym16(args, n):
    """Whether a serving request of size n streams the packed 16-bit pass."""
    return 1 if args.sym16_min_n and n >= args.sym16_min_n else 0


def _gen_request(req, storage):
    import torch
    import qcqp_inputs as qi
    sd = {"float64": torch.float64, "bfloat16": torch.bfloat16, "float16": torch.float16,
          "float32": torch.float32}[storage]
    return qi.random_qcqp_torch(req["n"], req["m"], req["seed"], shift=0.0, device="cuda", store_dtype=sd)


def serve_batched(trace, storage, args, budget, timing=1):
    """Continuous batching: requests are admitted as slots and HBM free up; every batch step
    runs one pass kernel over all resident requests.  The serving clock excludes the time
    spent synthesizing each request's instance (reported separately).  timing=1 records HIP
    events around every pass (eager launches); timing=0 replays captured graphs."""
    import torch
    from paper_2605_29291_amd import Batch, Solver
    b = Batch(max_slots=args.max_slots, hbm_budget_bytes=budget, storage=storage,
              spec_trials=args.spec, timing=timing)
    reqs = [dict(r) for r in trace]
    idx, done, gen = 0, 0, 0.0
    slot_req = {}
    resident = 0
    t0 = time.perf_counter()
    held = None
    while done < len(reqs):
        now = time.perf_counter() - t0 - gen
        while idx < len(reqs) and reqs[idx]["arrival"] <= now:
            r = reqs[idx]
            est = _est_bytes(r["n"], r["m"], storage, sym=_sym16(args, r["n"]))
            if slot_req and resident + est > budget:
                break
            if held is None:
                # instance synthesis is the client's work and stays off the clock; admission
                # (qcqp_create: copy, conversion, checks, step-size estimate) is on it
                tg = time.perf_counter()
                inst = _gen_request(r, storage)
                torch.cuda.synchronize()
                gen += time.perf_counter() - tg
                ta = time.perf_counter()
                held = Solver(inst, device=True, storage=storage, tau_bar=0.0, gamma0=0.1,
                              spec_trials=args.spec, sym_pass=_sym16(args, r["n"]))
                r["admission_ms"] = (time.perf_counter() - ta) * 1e3
                del inst
            nb = held.nbytes()
            slot = b.admit(held)
            if slot is None:
                break
            r["admitted"] = time.perf_counter() - t0 - gen
            r["bytes"] = nb
            resident += r["bytes"]
            slot_req[slot] = idx
            held = None
            idx += 1
        if not slot_req:
            if idx < len(reqs):
                wait = reqs[idx]["arrival"] - (time.perf_counter() - t0 - gen)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
            continue
        b.step(args.groups)
        for slot in b.poll():
            s, x, y, info = b.fetch(slot)
            k = slot_req.pop(slot)
            reqs[k]["done"] = time.perf_counter() - t0 - gen
            reqs[k]["info"] = info
            resident -= reqs[k]["bytes"]
            if args.check and k < args.check:
                reqs[k]["x"], reqs[k]["y"] = x.cpu().numpy(), y.cpu().numpy()
            s.close()
            done += 1
            if done % 64 == 0:
                log(f"  batched {storage}: {done}/{len(reqs)} done, {len(slot_req)} resident, "
                    f"generation {gen:.1f} s")
    total = time.perf_counter() - t0 - gen
    ps = b.pass_stats()
    b.close()
    return reqs, total, gen, ps


def _batch_pass_kernel(args):
    if not args.sym16_min_n:
        return f"k_pass<DT_BF16,{args.spec}> (algorithmic bytes (m+1) n^2 x 2 per request pass)"
    return (f"k_spass16<DT_BF16,{args.spec}> + k_sred16 for requests with n >= {args.sym16_min_n} (packed "
            f"upper triangles, (m+1) n(n+1)/2 x 2 bytes), k_pass<DT_BF16,{args.spec}> for the others "
            f"((m+1) n^2 x 2 bytes)")


def serve_fifo(trace, storage, args):
    """The plain single-instance path: one request at a time, in arrival order."""
    import torch
    from paper_2605_29291_amd import Solver
    reqs = [dict(r) for r in trace]
    gen = 0.0
    t0 = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t0 - gen
        if r["arrival"] > now:
            time.sleep(r["arrival"] - now)
        tg = time.perf_counter()
        inst = _gen_request(r, storage)
        torch.cuda.synchronize()
        gen += time.perf_counter() - tg
        ta = time.perf_counter()
        s = Solver(inst, device=True, storage=storage, tau_bar=0.0, gamma0=0.1,
                   spec_trials=args.spec, timing=1)
        r["admission_ms"] = (time.perf_counter() - ta) * 1e3
        del inst
        r["admitted"] = time.perf_counter() - t0 - gen
        x, y, info = s.solve()
        r["done"] = time.perf_counter() - t0 - gen
        r["info"] = info
        s.close()
        if (len([q for q in reqs if "done" in q])) % 64 == 0:
            log(f"  fifo {storage}: {len([q for q in reqs if 'done' in q])}/{len(reqs)} done")
    total = time.perf_counter() - t0 - gen
    return reqs, total, gen


def _lat_summary(reqs, total):
    """Request latency = completion - arrival, with admission (qcqp_create) inside it; only
    requests that reach relative KKT <= 1e-6 count as solves."""
    lat = np.array([r["done"] - r["arrival"] for r in reqs]) * 1e3
    adm = np.array([r.get("admission_ms", 0.0) for r in reqs])
    ok = [r["info"]["status"] == "ok" and r["info"]["rel_kkt"] <= 1e-6 for r in reqs]
    return dict(solves_per_s=sum(ok) / total, requests=len(reqs), converged=int(sum(ok)),
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                admission_p50_ms=float(np.percentile(adm, 50)), admission_p99_ms=float(np.percentile(adm, 99)),
                total_s=total, max_rel_kkt=float(max(r["info"]["rel_kkt"] for r in reqs)))


def workload_serving(args):
    import torch
    import qcqp_inputs as qi
    free, total_mem = torch.cuda.mem_get_info()
    budget = int(free - 24e9)
    trace = qi.serving_trace(args.requests, qi.config_seed(5), rate=None)
    log(f"serving: {len(trace)} requests, closed loop, BF16 continuous batching, budget {budget/1e9:.0f} GB")
    reqs_t, total_t, gen_t, ps = serve_batched(trace, "bfloat16", args, budget, timing=1)
    timed = _lat_summary(reqs_t, total_t)
    gbs = ps["pass_bytes"] / ps["pass_seconds"] / 1e9 if ps["pass_seconds"] > 0 else None
    log(f"batched closed loop, pass events: {timed}  pass {gbs} GB/s  gen {gen_t:.1f} s")
    reqs, total, gen, _ = serve_batched(trace, "bfloat16", args, budget, timing=0)
    closed = _lat_summary(reqs, total)
    log(f"batched closed loop, graphs: {closed}  gen {gen:.1f} s")
    rate = 0.7 * closed["solves_per_s"]
    trace_p = qi.serving_trace(args.requests, qi.config_seed(5), rate=rate)
    reqs_p, total_p, gen_p, ps_p = serve_batched(trace_p, "bfloat16", args, budget, timing=0)
    poisson = _lat_summary(reqs_p, total_p)
    log(f"batched Poisson rate {rate:.2f}/s: {poisson}")
    fifo = None
    if not args.no_fifo:
        reqs_f, total_f, gen_f = serve_fifo(trace_p, "float64", args)
        fifo = _lat_summary(reqs_f, total_f)
        log(f"FP64 FIFO same Poisson trace: {fifo}")
    # oracle check of a subset: relative KKT of the GPU results on the stored (rounded) instances
    checks = []
    if args.check:
        import oracle
        for r in reqs[: args.check]:
            inst = _gen_request(r, "bfloat16")
            P = oracle.Problem(inst)
            kk = oracle.kkt(P, r["x"], r["y"])
            checks.append(dict(n=r["n"], m=r["m"], rel_kkt_oracle=kk["rel_kkt"], gpu_rel_kkt=r["info"]["rel_kkt"]))
            del inst
    cpu = None
    value = closed["solves_per_s"]
    return {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": len(trace),
        "warmup": 0, "ms_per_step": 1e3 / value if value else None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16-storage/f32-acc/f64-checks", "data": "synthetic",
        "config": {"workload": f"serving: {len(trace)} random QCQP requests n~U[200,3000], m~U[5,200], BF16 "
                               "stack, continuous batching admitted by free HBM", "max_slots": args.max_slots,
                   "groups_per_step": args.groups, "budget_bytes": budget, "spec_trials": args.spec},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS if gbs else None, "traffic": None,
                     "kernel": f"k_pass<DT_BF16,{args.spec}> over all resident requests"},
        "cpu_baseline": cpu,
        "latency_ms": {"p50": closed["p50_ms"], "p99": closed["p99_ms"]},
        "closed_loop": closed, "closed_loop_with_pass_events": timed,
        "poisson": dict(poisson, rate_per_s=rate), "fp64_fifo_same_trace": fifo,
        "generation_s": gen, "oracle_checks": checks,
    }


def workload_precision(args):
    import torch
    import qcqp_inputs as qi
    from paper_2605_29291_amd import Solver
    n, m = 4000, 200
    seed = qi.config_seed(3)
    log("precision: generating n=4000 m=200 (FP64 on the GPU)")
    inst64 = qi.random_qcqp_torch(n, m, seed, shift=0.01, device="cuda")
    L0 = spectral_norm_gpu(inst64.Q[0])
    tau_bar = 1.0 / L0
    # reference: the unrounded FP64 instance on the FP64 path
    s64 = Solver(inst64, device=True, storage="float64", tau_bar=tau_bar, gamma0=0.1, timing=1)
    x64, y64, i64 = s64.solve()
    log(f"fp64 reference: iters={i64['iters']} rel_kkt={i64['rel_kkt']:.2e} f={i64['f']:.10f}")
    out = {}
    for storage, sym in (("bfloat16", 0), ("float16", 0), ("bfloat16", 1), ("float16", 1)):
        Qr = inst64.Q.to({"bfloat16": torch.bfloat16, "float16": torch.float16}[storage])
        instr = qi.Instance(n, m, 0, Qr, inst64.q, inst64.c, inst64.lb, inst64.ub)
        s = Solver(instr, device=True, storage=storage, tau_bar=tau_bar, gamma0=0.1, timing=1, sym_pass=sym)
        wall, lat, infos, x, y = run_solves(s, args.steps, args.warmup)
        avg_pass, tp = pass_stats(infos)
        pb = infos[0]["pass_bytes"]
        # error against the FP64 solution of the unrounded problem, and KKT there
        kk_unrounded = s64.eval_kkt(x, y)
        xr, x64n = x.cpu().numpy(), x64.cpu().numpy()
        err = dict(x_rel=float(np.linalg.norm(xr - x64n) / (1 + np.linalg.norm(x64n))),
                   f_rel=float(abs(kk_unrounded["f"] - i64["f"]) / (1 + abs(i64["f"]))),
                   rel_kkt_on_unrounded=kk_unrounded["rel_kkt"])
        # KKT on the stored instance, evaluated in FP64 on the GPU (parity of this evaluation
        # with the oracle is a GPU test)
        kk_stored = s.eval_kkt(x, y)
        key = storage + ("_packed" if sym else "")
        out[key] = dict(solves_per_s=args.steps / wall, p50_ms=float(np.percentile(np.array(lat) * 1e3, 50)),
                            p99_ms=float(np.percentile(np.array(lat) * 1e3, 99)),
                            iters=infos[0]["iters"], q_passes=infos[0]["q_passes"],
                            rel_kkt=infos[0]["rel_kkt"], rel_kkt_stored_fp64_eval=kk_stored["rel_kkt"],
                            q_pass_us=avg_pass * 1e6, q_pass_GBs=pb / avg_pass / 1e9,
                            q_pass_frac=pb / avg_pass / 1e9 / HBM_PEAK_GBS, bytes_per_pass=pb,
                            error_vs_fp64_unrounded=err,
                            all_converged=all(i["status"] == "ok" for i in infos))
        log(f"{key}: {out[key]}")
        s.close()
        del Qr, instr
        torch.cuda.empty_cache()
    b = out["bfloat16"]
    return {
        "metric": METRIC, "value": b["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 / b["solves_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16-storage/f32-acc/f64-checks", "data": "synthetic",
        "config": {"workload": "random convex QCQP n=4000 m=200, Q_i=A_iA_i'/n+0.01I stored BF16 (6.43 GB) "
                               "and FP16, FP32 accumulation, FP64 test/restart/KKT"},
        "roofline": {"bound": "hbm", "achieved": b["q_pass_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": b["q_pass_frac"], "traffic": None, "kernel": "k_pass<DT_BF16,2>"},
        "cpu_baseline": None,
        "latency_ms": {"p50": b["p50_ms"], "p99": b["p99_ms"]},
        "fp64_reference": dict(iters=i64["iters"], rel_kkt=i64["rel_kkt"], f=i64["f"],
                               q_pass_GBs=i64["pass_bytes"] / (i64["pass_seconds"] / max(i64["timed_passes"], 1)) / 1e9),
        "per_storage": out,
    }


def workload_kml(args):
    import torch
    import qcqp_inputs as qi
    from paper_2605_29291_amd import Solver
    log("kml: generating 8000 points, m=5 RBF kernels")
    out = {}
    for storage in ("float32", "bfloat16"):
        sd = {"float32": torch.float32, "bfloat16": torch.bfloat16}[storage]
        inst = qi.kml_qcqp(npts=8000, seed=qi.config_seed(4), device="cuda", store_dtype=sd)
        s = Solver(inst, device=True, storage=storage, tau_bar=0.0, gamma0=0.1, max_iter=args.kml_iters,
                   timing=1)
        t = time.perf_counter()
        x, y, info = s.solve()
        wall = time.perf_counter() - t
        avg = info["pass_seconds"] / max(info["timed_passes"], 1)
        out[storage] = dict(seconds=wall, iters=info["iters"], q_passes=info["q_passes"],
                            iters_per_s=info["iters"] / wall, rel_kkt=info["rel_kkt"], status=info["status"],
                            q_pass_us=avg * 1e6, q_pass_GBs=info["pass_bytes"] / avg / 1e9,
                            bytes_per_pass=info["pass_bytes"])
        log(f"{storage}: {out[storage]}")
        s.close()
        del inst
        torch.cuda.empty_cache()
    f = out["float32"]
    return {
        "metric": METRIC, "value": f["iters_per_s"], "unit": "iterations/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": f["seconds"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-storage", "data": "synthetic",
        "config": {"workload": f"kernel-learning QCQP, 8000 points, m=5 RBF kernels, n=8001, Q_0 absent, "
                               f"p=1; capped at {args.kml_iters} iterations"},
        "roofline": {"bound": "hbm", "achieved": f["q_pass_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": f["q_pass_GBs"] / HBM_PEAK_GBS, "traffic": None, "kernel": "k_pass<DT_F32,2>"},
        "cpu_baseline": None, "per_storage": out,
    }


def workload_kml_minmax(args):
    """The paper's kernel-learning min-max form (§5): min over x >= 0 with b'x = 0, max over the
    3-simplex; three normalised kernels (polynomial, Gaussian, linear) on a synthetic stand-in
    for SIDO0; mu = 2; rAPDB-yx non-monotone with restarts every 200 iterations (the §5
    setting); relative KKT <= 1e-6.  n = 4000 and n = 10000 as in §5, FP64 and BF16 storage."""
    import torch
    import qcqp_inputs as qi
    from paper_2605_29291_amd import Solver
    out = {}
    for npts in (4000, 10000):
        for label, storage, sym in (("float64", "float64", 0), ("float64_sym", "float64", 1),
                                    ("bfloat16", "bfloat16", 0)):
            sd = {"float64": torch.float64, "bfloat16": torch.bfloat16}[storage]
            log(f"kml min-max: n={npts} {label}")
            inst = qi.kml_minmax(npts, seed=qi.config_seed(4), device="cuda", store_dtype=sd)
            kw = dict(tau_bar=0.5, gamma0=0.1, mu=2.0, restart_every=200, sym_pass=sym)
            s = Solver(inst, device=True, storage=storage, **kw)
            wall, lat, infos, x, y = run_solves(s, args.steps, args.warmup)
            st = Solver(inst, device=True, storage=storage, timing=1, **kw)
            _, _, tinfos, _, _ = run_solves(st, 1, 0)
            avg, tp = pass_stats(tinfos)
            info = infos[-1]
            pb = info["pass_bytes"]
            # solves count only when every timed solve stopped at relative KKT <= 1e-6
            ok = all(i["status"] == "ok" and i["rel_kkt"] <= 1e-6 for i in infos)
            out[f"n{npts}_{label}"] = dict(
                solves_per_s=args.steps / wall if ok else None, ms_per_solve=wall / args.steps * 1e3,
                all_converged=ok,
                iters=info["iters"], trials=info["trials"], q_passes=info["q_passes"],
                rel_kkt=info["rel_kkt"], status=info["status"],
                q_pass_us=avg * 1e6, q_pass_GBs=pb / avg / 1e9, bytes_per_pass=pb,
                lambda_=[float(v) for v in y[1:].tolist()])
            log(f"  {out[f'n{npts}_{label}']}")
            s.close()
            st.close()
            del inst
            torch.cuda.empty_cache()
    h = out["n10000_float64"]
    return {
        "metric": METRIC, "value": h["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": h["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "kernel-learning min-max (paper's form): n=10000 points, 3 normalised "
                               "kernels, lambda on the simplex, b'x = 0, x >= 0, mu = 2, FP64 stack "
                               "2.4 GB, rAPDB-yx non-monotone, restart 200, rel-KKT<=1e-6"},
        "roofline": {"bound": "hbm", "achieved": h["q_pass_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": h["q_pass_GBs"] / HBM_PEAK_GBS, "traffic": None, "kernel": "k_pass<DT_F64,2>"},
        "cpu_baseline": None, "per_case": out,
    }


PAPER_ROWS = {
    "mono rAPDB-xy": dict(variant="xy", c_nm=0, restart="fixed", restart_every=2000),
    "mono rAPDB-yx": dict(variant="yx", c_nm=0, restart="fixed", restart_every=800),
    "mono rAPDB-xy-ada": dict(variant="xy", c_nm=0, restart="adaptive", ada_first=100, ada_every=500),
    "mono rAPDB-yx-ada": dict(variant="yx", c_nm=0, restart="adaptive", ada_first=50, ada_every=200),
    "mono APDB-xy": dict(variant="xy", c_nm=0, restart="none"),
    "mono APDB-yx": dict(variant="yx", c_nm=0, restart="none"),
    "non-mono rAPDB-xy": dict(variant="xy", c_nm=1, restart="fixed", restart_every=1000),
    "non-mono rAPDB-yx": dict(variant="yx", c_nm=1, restart="fixed", restart_every=400),
    "non-mono rAPDB-xy-ada": dict(variant="xy", c_nm=1, restart="adaptive", ada_first=100, ada_every=500),
    "non-mono rAPDB-yx-ada": dict(variant="yx", c_nm=1, restart="adaptive", ada_first=50, ada_every=500),
    "non-mono APDB-xy": dict(variant="xy", c_nm=1, restart="none"),
    "non-mono APDB-yx": dict(variant="yx", c_nm=1, restart="none"),
}
# the paper's reported iteration counts and A100 GPU seconds for these rows (context only:
# its instances, f* and step parameters are not available)
PAPER_TABLE = {
    "mono rAPDB-xy": (20686, 58), "mono rAPDB-yx": (4609, 18), "mono rAPDB-xy-ada": (28404, 113),
    "mono rAPDB-yx-ada": (10319, 52), "mono APDB-xy": (50000, 136), "mono APDB-yx": (34947, 133),
    "non-mono rAPDB-xy": (3008, 18), "non-mono rAPDB-yx": (873, 6), "non-mono rAPDB-xy-ada": (3040, 22),
    "non-mono rAPDB-yx-ada": (877, 10), "non-mono APDB-xy": (3026, 18), "non-mono APDB-yx": (871, 6),
}


def same_paper_instance(inst, fp):
    """The stored f* belongs to this instance: q and c bit-identical, and every matrix's entry sum
    and absolute sum within 1e-12 (the matrices come from a QR factorisation and products whose
    rounding may differ between machines)."""
    import hashlib

    def sha(a):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()

    if sha(inst.q) != fp["q_sha256"] or sha(inst.c) != fp["c_sha256"]:
        return False
    Q = np.asarray(inst.Q)
    for i in range(Q.shape[0]):
        if abs(float(Q[i].sum()) - fp["q_sum"][i]) > 1e-12 * fp["q_abs_sum"][i]:
            return False
        if abs(float(np.abs(Q[i]).sum()) - fp["q_abs_sum"][i]) > 1e-12 * fp["q_abs_sum"][i]:
            return False
    return True


def workload_paper_random(args):
    """The random-QCQP experiment of §5.1 with its twelve method rows: n = 1000, m = 10, four
    fresh instances of the paper's generator, FP64, the criterion of §5.1 at 1e-7 with f* from
    the oracle's solve to relative KKT <= 1e-11 (stored by tests/golden/make_golden.py), at most
    50000 iterations; eta, c_alpha, c_beta,
    delta, restart frequencies and adaptive schedules as §5.1 gives them; gamma_0 and tau_bar
    (unstated in the paper) from the command line and 1 / ||Q_0||."""
    import torch
    import qcqp_inputs as qi
    from paper_2605_29291_amd import Solver
    n, m = 1000, 10
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_random_n1000_m10.json")))
    insts = []
    for k in range(4):
        log(f"paper random QCQP instance {k}")
        inst = qi.paper_random_qcqp(n, m, seed=qi.config_seed(6, k))
        g = gold["instances"][k]
        if not same_paper_instance(inst, g["fingerprint"]):
            raise RuntimeError(f"paper random instance {k} differs from the one the stored f* belongs to")
        L = float(np.linalg.norm(inst.Q[0], 2))
        log(f"  f* = {g['f_star']:.12g} (the oracle's solve at relative KKT {g['oracle_rel_kkt']:.1e})")
        insts.append((inst, 1.0 / L, g["f_star"]))
    rows = {}
    only = [r.strip() for r in args.rows.split(",")] if args.rows else list(PAPER_ROWS)
    for name, row in PAPER_ROWS.items():
        if name not in only:
            continue
        kw = dict(row)
        if kw["variant"] == "xy":
            kw.update(c_alpha=0.25, c_beta=0.3, delta=0.4)
        its, secs, ok = [], [], 0
        for inst, tb, fs in insts:
            s = Solver(inst, tau_bar=tb, gamma0=args.gamma0, tol=1e-7, stop_rule="paper", f_star=fs,
                       max_iter=50000, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, y, info = s.solve()
            secs.append(time.perf_counter() - t)
            its.append(info["iters"])
            ok += info["status"] == "ok"
            s.close()
        pi, pg = PAPER_TABLE[name]
        rows[name] = dict(iters=float(np.mean(its)), iters_each=its, gpu_s=float(np.mean(secs)),
                          converged=ok, paper_iters=pi, paper_a100_gpu_s=pg)
        log(f"{name}: {rows[name]}")
    best = rows.get("non-mono rAPDB-yx") or next(iter(rows.values()))
    return {
        "metric": METRIC, "value": 1.0 / best["gpu_s"], "unit": "solves/s", "n_gpus": 1, "steps": 4,
        "warmup": 0, "ms_per_step": best["gpu_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"the paper's random QCQPs (Q_i = L_i' S_i L_i): n=1000, m=10, 4 instances, "
                               f"criterion of the experiments at 1e-7, non-mono rAPDB-yx restart 400, "
                               f"gamma0={args.gamma0}"},
        "roofline": None, "cpu_baseline": None, "rows": rows,
    }


def workload_batch_pass(args):
    """Pass bandwidth of a full continuous batch at steady state: requests of the serving trace
    (n ~ U[200, 3000], m ~ U[5, 200], BF16 storage) are admitted up to a byte budget, two
    groups run untimed (start anchors), then 8 groups are timed with HIP events around each
    pass launch; bytes are the live slots' stacks.  Live sets of 1, 8, 32, 128 and all that fit
    in 64 GB."""
    import torch
    import qcqp_inputs as qi
    from paper_2605_29291_amd import Batch, Solver
    storage = "bfloat16"
    trace = qi.serving_trace(512, qi.config_seed(5))
    out = {}
    for k in (1, 8, 32, 128, 512):
        b = Batch(max_slots=k, hbm_budget_bytes=int(64e9), storage=storage, spec_trials=args.spec,
                  timing=1)
        admitted, held = 0, []
        for r in trace[:k]:
            inst = _gen_request(r, storage)
            s = Solver(inst, device=True, storage=storage, tau_bar=0.0, gamma0=0.1,
                       spec_trials=args.spec, sym_pass=_sym16(args, r["n"]))
            del inst
            if b.admit(s) is None:
                s.close()
                break
            held.append(s)
            admitted += 1
        torch.cuda.synchronize()
        b.step(2)
        st0 = b.pass_stats()
        b.step(8)
        st1 = b.pass_stats()
        s0, by0, s1, by1 = st0["pass_seconds"], st0["pass_bytes"], st1["pass_seconds"], st1["pass_bytes"]
        gbs = (by1 - by0) / max(s1 - s0, 1e-12) / 1e9
        out[f"slots{admitted}"] = dict(slots=admitted, pass_GBs=gbs, frac=gbs / HBM_PEAK_GBS,
                                       bytes_per_group=(by1 - by0) / 8, us_per_group_pass=(s1 - s0) / 8 * 1e6)
        log(f"batch pass: {out[f'slots{admitted}']}")
        b.close()
        for s in held:
            s.close()
        torch.cuda.empty_cache()
        if admitted < k:
            break
    last = list(out.values())[-1]
    return {"metric": METRIC, "value": last["pass_GBs"], "unit": "GB/s", "n_gpus": 1, "steps": 8,
            "warmup": 2, "ms_per_step": last["us_per_group_pass"] / 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16-storage", "data": "synthetic",
            "config": {"workload": "continuous batch of serving-trace requests, BF16, steady-state pass",
                       "spec_trials": args.spec, "packed_from_n": args.sym16_min_n},
            "roofline": {"bound": "hbm", "achieved": last["pass_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": last["frac"], "traffic": None,
                         "kernel": _batch_pass_kernel(args)},
            "cpu_baseline": None, "per_batch": out}


def workload_traffic(args):
    """Dispatches for the HBM-traffic counters (run under rocprofv3 --pmc FETCH_SIZE, then
    WRITE_SIZE): a plain device copy of known size (the calibration), then the config-2 FP64
    row-major pass and the packed symmetric pass (k_spass + k_sred) exactly as the config-2
    solves launch them (trial mode, CONFIG2_SPEC candidates), and a BF16 pass as the serving
    batches launch it (2 candidates), row-major and packed (k_spass16 + k_sred16)."""
    import torch
    import qcqp_inputs as qi
    from paper_2605_29291_amd import Solver
    nbytes = 2 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").normal_()
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()
    out = {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}
    inst = qi.random_qcqp_exact(2000, 100, qi.config_seed(2), shift=0.01, device="cuda")
    s = Solver(inst, device=True, storage="float64", tau_bar=1.0, spec_trials=CONFIG2_SPEC)
    s.time_pass(reps=3)
    out["f64_pass_bytes"] = 101 * 2000 * 2000 * 8
    s.close()
    s = Solver(inst, device=True, storage="float64", tau_bar=1.0, spec_trials=CONFIG2_SYM_SPEC, sym_pass=1)
    s.time_pass(reps=3)
    out["f64_sym_pass_bytes"] = 101 * (2000 * 2001 // 2) * 8
    s.close()
    Qb = inst.Q.to(torch.bfloat16)
    ib = qi.Instance(2000, 100, 0, Qb, inst.q, inst.c, inst.lb, inst.ub)
    s = Solver(ib, device=True, storage="bfloat16", tau_bar=1.0, spec_trials=2)
    s.time_pass(reps=3)
    out["bf16_pass_bytes"] = 101 * 2000 * 2000 * 2
    s.close()
    s = Solver(ib, device=True, storage="bfloat16", tau_bar=1.0, spec_trials=2, sym_pass=1)
    s.time_pass(reps=3)
    out["bf16_sym_pass_bytes"] = 101 * (2000 * 2001 // 2) * 2
    s.close()
    return out


def workload_small(args):
    """Config-1-sized problems (n=100, m=10): latency of one solve, and 100 independent instances
    served as one batch (one pass kernel per trial group covers all of them)."""
    import torch
    import qcqp_inputs as qi
    from paper_2605_29291_amd import Batch, Solver
    insts = [qi.random_qcqp(100, 10, qi.config_seed(1, k)) for k in range(100)]
    tb = [1.0 / float(np.linalg.norm(i.Q[0], 2)) for i in insts]
    s = Solver(insts[0], device=True, tau_bar=tb[0], gamma0=0.1)
    for _ in range(args.warmup + 1):
        s.solve()
    lat = []
    for _ in range(max(args.steps, 20)):
        t = time.perf_counter()
        x, y, info = s.solve()
        lat.append(time.perf_counter() - t)
    s.close()
    single = dict(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                  solves_per_s=1.0 / float(np.mean(lat)), iters=info["iters"], q_passes=info["q_passes"])
    log(f"single: {single}")
    solvers = [Solver(inst, device=True, tau_bar=t, gamma0=0.1) for inst, t in zip(insts, tb)]
    torch.cuda.synchronize()
    b = Batch(max_slots=len(insts))
    t0 = time.perf_counter()
    for sv in solvers:
        b.admit(sv)
    done = 0
    infos = []
    while done < len(insts):
        b.step(16)
        for slot in b.poll():
            _, x, y, info = b.fetch(slot)
            infos.append(info)
            done += 1
    wall = time.perf_counter() - t0
    b.close()
    batched = dict(instances=len(insts), seconds=wall, solves_per_s=len(insts) / wall,
                   converged=sum(i["status"] == "ok" for i in infos),
                   max_rel_kkt=max(i["rel_kkt"] for i in infos))
    log(f"batched: {batched}")
    return {
        "metric": METRIC, "value": batched["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": len(insts), "warmup": args.warmup, "ms_per_step": 1e3 / batched["solves_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "random convex QCQP n=100 m=10 (0.88 MB FP64 stack, cache-resident), "
                               "100 instances as one batch; single-solve latency beside"},
        "roofline": None, "cpu_baseline": None,
        "latency_ms": {"p50": single["p50_ms"], "p99": single["p99_ms"]},
        "single": single, "batched": batched,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="config2")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--quick", action="store_true",
                    help="config2: the headline only, without the config-1, serving and precision sections")
    ap.add_argument("--requests", type=int, default=512, help="serving: number of requests")
    ap.add_argument("--max-slots", type=int, default=512, help="serving: batch slots")
    ap.add_argument("--groups", type=int, default=4, help="serving: trial groups per batch step")
    ap.add_argument("--check", type=int, default=8, help="serving: requests checked by the oracle")
    ap.add_argument("--no-fifo", action="store_true", help="serving: skip the FP64 FIFO comparison")
    ap.add_argument("--sym16-min-n", type=int, default=0,
                    help="serving/batch_pass: requests with n at least this stream the packed BF16 pass "
                         "(0, the default: every request streams the row-major pass)")
    ap.add_argument("--spec", type=int, default=2,
                    help="serving, batch_pass: speculative candidates per pass")
    ap.add_argument("--kml-iters", type=int, default=20000, help="kml: iteration cap")
    ap.add_argument("--gamma0", type=float, default=0.1, help="paper_random: gamma_0")
    ap.add_argument("--rows", default="", help="paper_random: comma-separated method rows (default all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "config2":
        out = workload_config2(args)
    elif args.workload == "serving":
        out = workload_serving(args)
    elif args.workload == "precision":
        out = workload_precision(args)
    elif args.workload == "kml":
        out = workload_kml(args)
    elif args.workload == "batch_pass":
        out = workload_batch_pass(args)
    elif args.workload == "paper_random":
        out = workload_paper_random(args)
    elif args.workload == "kml_minmax":
        out = workload_kml_minmax(args)
    elif args.workload == "traffic":
        out = workload_traffic(args)
    elif args.workload == "small":
        out = workload_small(args)
    else:
        print(json.dumps({"error": f"unknown workload {args.workload}"}))
        sys.exit(2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
