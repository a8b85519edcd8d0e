"""Continuous batching (qcqp_batch_*): each request's result is the same alone and in a mix.

Every kernel reduces per slot in a fixed order, so a request solved inside a batch with other,
differently sized requests -- admitted at different times -- must return bitwise the same
iterate, multipliers and counters as when it is solved alone.  Results are also checked against
the FP64 oracle (relative KKT <= 1e-6 on the stored instance), and admission must refuse a
request that does not fit the HBM budget.
"""
import numpy as np
import pytest

from tests.gpu_common import announce, oracle, qi, tau_bar_of, to_np

pytestmark = pytest.mark.gpu

SIZES = [(60, 3), (150, 12), (333, 25), (97, 7), (512, 40), (200, 1), (41, 0)]


def _instances(storage):
    out = []
    for k, (n, m) in enumerate(SIZES):
        inst = qi.random_qcqp(n, m, seed=5000 + k, shift=0.0)
        if storage != "float64":
            inst = qi.round_instance(inst, storage)
        out.append(inst)
    return out


def _opts(inst, storage):
    return dict(tau_bar=tau_bar_of(inst), gamma0=0.1, storage=storage, restart_every=30)


@pytest.mark.parametrize("storage", ["float64", "float32", "bfloat16", "float16"])
def test_alone_equals_mix(storage):
    from paper_2605_29291_amd import Batch, Solver
    insts = _instances(storage)
    alone = []
    for inst in insts:
        announce(f"alone {inst.name}")
        s = Solver(inst, **_opts(inst, storage))
        x, y, info = s.solve()
        alone.append((to_np(x), to_np(y), info))
        b = Batch(max_slots=1, storage=storage)
        slot = b.admit(s)
        while not b.poll():
            b.step(4)
        _, xb, yb, ib = b.fetch(slot)
        np.testing.assert_array_equal(to_np(xb), alone[-1][0])
        np.testing.assert_array_equal(to_np(yb), alone[-1][1])
        assert ib["iters"] == info["iters"] and ib["trials"] == info["trials"]
        b.close()
        s.close()
    announce("mix")
    b = Batch(max_slots=8, storage=storage)
    solvers = [Solver(inst, **_opts(inst, storage)) for inst in insts]
    slot_of = {}
    for k in (0, 2, 4):
        slot_of[b.admit(solvers[k])] = k
    b.step(3)                                   # the first requests run alone for a while
    for k in (1, 3, 5, 6):
        slot_of[b.admit(solvers[k])] = k
    results = {}
    guard = 0
    while len(results) < len(insts):
        b.step(5)
        for slot in b.poll():
            s, x, y, info = b.fetch(slot)
            results[slot_of[slot]] = (to_np(x), to_np(y), info)
        guard += 1
        assert guard < 10000
    b.close()
    for k, inst in enumerate(insts):
        x, y, info = results[k]
        np.testing.assert_array_equal(x, alone[k][0], err_msg=inst.name)
        np.testing.assert_array_equal(y, alone[k][1], err_msg=inst.name)
        assert info["iters"] == alone[k][2]["iters"] and info["trials"] == alone[k][2]["trials"]
        assert info["status"] == "ok"
        kk = oracle.kkt(oracle.Problem(inst), x, y)
        assert kk["rel_kkt"] <= 1e-6, (inst.name, kk)


def test_admission_respects_hbm_budget():
    from paper_2605_29291_amd import Batch, Solver
    insts = _instances("float64")[:3]
    solvers = [Solver(i, **_opts(i, "float64")) for i in insts]
    sizes = [s.nbytes() for s in solvers]
    budget = max(sizes[0], sizes[1]) + min(sizes[0], sizes[1]) // 2   # each fits alone, not both
    b = Batch(max_slots=8, hbm_budget_bytes=budget)
    assert b.admit(solvers[0]) is not None
    assert b.admit(solvers[1]) is None            # would exceed the budget
    st = b.stats()
    assert st["running"] == 1 and st["resident_bytes"] == sizes[0]
    while not b.poll():
        b.step(8)
    slot = b.poll()[0]
    b.fetch(slot)
    assert b.admit(solvers[1]) is not None        # room again after the fetch
    b.close()
    b2 = Batch(max_slots=1)
    assert b2.admit(solvers[2]) is not None
    assert b2.admit(Solver(insts[0], **_opts(insts[0], "float64"))) is None   # no free slot
    b2.close()


def test_adaptive_restarts_inside_a_batch():
    """A slot whose schedule asks for the smoothed gap is parked, its G_xi evaluated on the
    device (one cooperative launch for the inner box QP) and the decision taken there; the result
    matches the same solve alone."""
    from paper_2605_29291_amd import Batch, Solver
    insts = [qi.random_qcqp(n, m, seed=7000 + n, shift=0.01) for n, m in ((120, 8), (90, 5))]
    kw = dict(restart="adaptive", ada_first=5, ada_every=10, c_nm=0)
    alone = []
    for inst in insts:
        s = Solver(inst, tau_bar=tau_bar_of(inst), gamma0=0.1, **kw)
        x, y, info = s.solve()
        assert info["gap_evals"] >= 1
        alone.append((to_np(x), info))
    b = Batch(max_slots=4, restart="adaptive")
    slots = {b.admit(Solver(inst, tau_bar=tau_bar_of(inst), gamma0=0.1, **kw)): k
             for k, inst in enumerate(insts)}
    got = {}
    while len(got) < len(insts):
        b.step(4)
        for slot in b.poll():
            _, x, y, info = b.fetch(slot)
            got[slots[slot]] = (to_np(x), info)
    b.close()
    for k in range(len(insts)):
        np.testing.assert_array_equal(got[k][0], alone[k][0])
        assert got[k][1]["gap_evals"] == alone[k][1]["gap_evals"]
        assert got[k][1]["status"] == "ok"


def test_mixed_adaptive_and_fixed_restarts_alone_equals_mix():
    """Adaptive-restart slots evaluate G_xi on the batch's side stream while fixed-restart and
    other adaptive slots keep stepping; the decision is taken on the device from the device's
    G_xi.  Every request returns the same bits (and the same restart and gap counts) alone and
    in the mix."""
    from paper_2605_29291_amd import Batch, Solver
    specs = [((150, 10), dict(restart="adaptive", ada_first=5, ada_every=10, c_nm=0)),
             ((97, 6), dict(restart="fixed", restart_every=15)),
             ((60, 3), dict(restart="adaptive", ada_first=8, ada_every=12, c_nm=1)),
             ((211, 12), dict(restart="fixed", restart_every=40, c_nm=0)),
             ((120, 8), dict(restart="adaptive", ada_first=5, ada_every=7, c_nm=0))]
    insts = [qi.random_qcqp(n, m, seed=7100 + k, shift=0.01) for k, ((n, m), _) in enumerate(specs)]
    alone = []
    for inst, (_, kw) in zip(insts, specs):
        announce(f"alone {inst.name} {kw['restart']}")
        b = Batch(max_slots=1)
        slot = b.admit(Solver(inst, tau_bar=tau_bar_of(inst), gamma0=0.1, **kw))
        while not b.poll():
            b.step(3)
        _, x, y, info = b.fetch(slot)
        b.close()
        assert info["status"] == "ok"
        if kw["restart"] == "adaptive":
            assert info["gap_evals"] >= 2
        alone.append((to_np(x), to_np(y), info))
    announce("mix of adaptive and fixed restarts")
    b = Batch(max_slots=8)
    slot_of = {}
    for k in (0, 1, 2):
        slot_of[b.admit(Solver(insts[k], tau_bar=tau_bar_of(insts[k]), gamma0=0.1, **specs[k][1]))] = k
    b.step(2)
    for k in (3, 4):
        slot_of[b.admit(Solver(insts[k], tau_bar=tau_bar_of(insts[k]), gamma0=0.1, **specs[k][1]))] = k
    got, guard = {}, 0
    while len(got) < len(insts):
        b.step(2)
        for slot in b.poll():
            _, x, y, info = b.fetch(slot)
            got[slot_of[slot]] = (to_np(x), to_np(y), info)
        guard += 1
        assert guard < 20000
    b.close()
    for k in range(len(insts)):
        np.testing.assert_array_equal(got[k][0], alone[k][0])
        np.testing.assert_array_equal(got[k][1], alone[k][1])
        for key in ("iters", "trials", "restarts", "gap_evals"):
            assert got[k][2][key] == alone[k][2][key], (k, key)


@pytest.mark.parametrize("storage", ["float64", "bfloat16"])
def test_requests_with_equality_constraints_alone_equals_mix(storage):
    """Requests with different numbers of equality constraints (p = 0..3, so y = (v, lambda)
    has a different split in every slot) return bitwise the same result alone and in one
    batch, admitted at different times, and reach the oracle-evaluated KKT of 1e-6."""
    from paper_2605_29291_amd import Batch, Solver
    specs = [(150, 6, 2), (80, 0, 3), (220, 10, 0), (97, 4, 1)]
    insts = []
    for k, (n, m, p) in enumerate(specs):
        inst = qi.random_qcqp(n, m, seed=5300 + k, shift=0.01, p=p)
        insts.append(qi.round_instance(inst, storage) if storage != "float64" else inst)
    alone = []
    for inst in insts:
        announce(f"alone {inst.name} p={inst.p}")
        s = Solver(inst, **_opts(inst, storage))
        x, y, info = s.solve()
        alone.append((to_np(x), to_np(y), info))
        s.close()
    announce("mix with equality constraints")
    b = Batch(max_slots=4, storage=storage)
    solvers = [Solver(inst, **_opts(inst, storage)) for inst in insts]
    slot_of = {b.admit(solvers[0]): 0, b.admit(solvers[2]): 2}
    b.step(2)
    for k in (1, 3):
        slot_of[b.admit(solvers[k])] = k
    results = {}
    guard = 0
    while len(results) < len(insts):
        b.step(5)
        for slot in b.poll():
            _, x, y, info = b.fetch(slot)
            results[slot_of[slot]] = (to_np(x), to_np(y), info)
        guard += 1
        assert guard < 10000
    b.close()
    for k, inst in enumerate(insts):
        x, y, info = results[k]
        np.testing.assert_array_equal(x, alone[k][0], err_msg=inst.name)
        np.testing.assert_array_equal(y, alone[k][1], err_msg=inst.name)
        assert info["iters"] == alone[k][2]["iters"] and info["trials"] == alone[k][2]["trials"]
        assert info["status"] == "ok", info
        kk = oracle.kkt(oracle.Problem(inst), x, y)
        assert kk["rel_kkt"] <= 1e-6, (inst.name, kk)
