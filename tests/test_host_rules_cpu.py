"""Host rules of the library on the CPU (include/bfal_host.h): the argument
checks every device entry point applies, the stall rule of Section 5.2 and the
serving engine's admission policy driven by a stub executor.  No GPU: these
functions make no HIP call, so they run where libbfal.so merely loads."""
import heapq
import os

import numpy as np
import pytest

import scenes
from paper_2512_12151_amd import bfal

pytestmark = pytest.mark.skipif(not os.path.exists(bfal.LIB_PATH), reason="libbfal.so not built")

OK, INVALID, DEGENERATE = bfal.BF_OK, -1, -5


@pytest.fixture(scope="module")
def tiny():
    return scenes.tiny()


def mesh_args(sc, **kw):
    a = dict(tets=sc["tets"], rest=sc["rest"], E=sc["E"], nu=sc["nu"], rho=sc["rho"], fixed=sc["fixed"])
    a.update(kw)
    return a


# ------------------------------------------------------------------ mesh

def test_valid_scene_passes_every_check(tiny):
    sc = tiny
    assert bfal.check_mesh(**mesh_args(sc)) == (OK, "")
    assert bfal.check_state(len(sc["rest"]), sc["x"], sc["x_hat"], sc["x_tilde"], sc["dt"]) == (OK, "")
    assert bfal.check_constraints(len(sc["rest"]), sc["pt"], sc["ee"], sc["lam"], sc["gamma"], sc["kappa"],
                                  sc["delta"]) == (OK, "")
    assert bfal.check_solve_opts() == (OK, "")


@pytest.mark.parametrize("what,edit,reason", [
    ("index", lambda a: a["tets"].__setitem__((3, 2), 10**6), "out of range"),
    ("negative index", lambda a: a["tets"].__setitem__((0, 0), -1), "out of range"),
    ("repeated vertex", lambda a: a["tets"].__setitem__((5, 1), a["tets"][5, 0]), "repeated vertex"),
    ("E <= 0", lambda a: a["E"].__setitem__(7, 0.0), "material"),
    ("nu = 0.5", lambda a: a["nu"].__setitem__(7, 0.5), "material"),
    ("rho NaN", lambda a: a["rho"].__setitem__(7, np.nan), "material"),
    ("rest inf", lambda a: a["rest"].__setitem__((2, 1), np.inf), "non-finite"),
    ("material code", lambda a: a.__setitem__("material", np.full(len(a["tets"]), 3, np.int32)), "material code"),
])
def test_mesh_errors(tiny, what, edit, reason):
    a = mesh_args(tiny, tets=tiny["tets"].copy(), rest=tiny["rest"].copy(), E=tiny["E"].copy(),
                  nu=tiny["nu"].copy(), rho=tiny["rho"].copy())
    edit(a)
    st, msg = bfal.check_mesh(**a)
    assert st == INVALID, what
    assert reason in msg


def test_mesh_sizes():
    one = dict(tets=np.array([[0, 1, 2, 3]]), rest=np.eye(4, 3), E=[1e5], nu=[0.3], rho=[1e3])
    assert bfal.check_mesh(**one)[0] == OK
    st, msg = bfal.check_mesh(tets=np.zeros((0, 4)), rest=np.eye(4, 3), E=[], nu=[], rho=[])
    assert st == INVALID and "positive" in msg
    # the three material codes are all accepted
    assert bfal.check_mesh(**one, material=[2])[0] == OK


# ------------------------------------------------------------------ state

def test_state_errors(tiny):
    sc, N = tiny, len(tiny["rest"])
    for dt in (0.0, -0.01, np.inf, np.nan):
        st, msg = bfal.check_state(N, sc["x"], sc["x_hat"], sc["x_tilde"], dt)
        assert st == INVALID and "dt" in msg
    xh = sc["x_hat"].copy()
    xh[4, 2] = np.nan
    assert bfal.check_state(N, sc["x"], xh, sc["x_tilde"], sc["dt"]) == (INVALID, "non-finite state value")
    st, msg = bfal.check_state(N, None, sc["x_hat"], sc["x_tilde"], sc["dt"])
    assert st == INVALID and "NULL" in msg


# ------------------------------------------------------------ constraints

def cons(sc, **kw):
    a = dict(pt=sc["pt"].copy(), ee=sc["ee"].copy(), lam=sc["lam"].copy(), gamma=sc["gamma"].copy(),
             kappa=sc["kappa"], delta=sc["delta"])
    a.update(kw)
    return a


@pytest.mark.parametrize("what,edit,status,reason", [
    ("pt index", lambda a: a["pt"].__setitem__((0, 1), 10**6), INVALID, "out of range"),
    ("ee index", lambda a: a["ee"].__setitem__((1, 3), -2), INVALID, "out of range"),
    ("shared vertex", lambda a: a["pt"].__setitem__((2, 3), a["pt"][2, 0]), DEGENERATE, "repeated vertex"),
    ("lambda < 0", lambda a: a["lam"].__setitem__(4, -1.0), INVALID, "lambda"),
    ("lambda NaN", lambda a: a["lam"].__setitem__(4, np.nan), INVALID, "lambda"),
    ("gamma 0", lambda a: a["gamma"].__setitem__(0, 0.0), INVALID, "gamma"),
    ("gamma > 1", lambda a: a["gamma"].__setitem__(0, 1.5), INVALID, "gamma"),
    ("kappa 0", lambda a: a.__setitem__("kappa", 0.0), INVALID, "kappa"),
    ("kappa inf", lambda a: a.__setitem__("kappa", np.inf), INVALID, "kappa"),
    ("delta < 0", lambda a: a.__setitem__("delta", -1e-3), INVALID, "delta"),
])
def test_constraint_errors(tiny, what, edit, status, reason):
    a = cons(tiny)
    edit(a)
    st, msg = bfal.check_constraints(len(tiny["rest"]), **a)
    assert st == status, what
    assert reason in msg


def test_empty_constraint_set_and_default_gamma(tiny):
    z = np.zeros((0, 4), np.int32)
    assert bfal.check_constraints(10, z, z, np.zeros(0), None, 1e4, 0.0)[0] == OK
    assert bfal.check_constraints(len(tiny["rest"]), **cons(tiny, gamma=None))[0] == OK


def test_solve_opts_errors():
    assert bfal.check_solve_opts(tol=0.0)[0] == INVALID
    assert bfal.check_solve_opts(max_iter=-1)[0] == INVALID
    assert bfal.check_solve_opts(precision=7)[0] == INVALID
    assert bfal.check_solve_opts(precision=bfal.BF_PREC_BF16_REFINE, refine_tol=0.0)[0] == INVALID
    assert bfal.check_solve_opts(max_iter=0)[0] == OK


# ------------------------------------------------------------- stall rule

def test_stall_rule_on_a_hand_made_alpha_sequence():
    """Section 5.2: 50 consecutive steps below 1e-4 double the penalty and halve
    the offset; a step at or above 1e-4 restarts the count; the count restarts
    after a doubling too."""
    r = bfal.StallRule(1e-4, 50)
    kappa, delta = 1e4, 1e-3
    seq = [1e-5] * 49 + [1e-4] + [5e-5] * 50 + [2e-6] * 100 + [0.5]
    fired_at = []
    for i, a in enumerate(seq):
        fired, kappa, delta = r.step(a, kappa, delta)
        if fired:
            fired_at.append(i)
    # the 49 small steps are cut by alpha = 1e-4 (not below it); then 50 at 5e-5
    # fire at index 99; the next 100 small ones fire twice (149, 199)
    assert fired_at == [99, 149, 199]
    assert kappa == 1e4 * 8 and delta == 1e-3 / 8
    assert r.r.count == 0


def test_stall_rule_never_fires_on_a_healthy_sequence():
    r = bfal.StallRule()
    rng = np.random.default_rng(0)
    k, d = 1.0, 1.0
    for a in rng.uniform(1e-4, 1.0, 500):
        fired, k, d = r.step(a, k, d)
        assert not fired
    assert (k, d) == (1.0, 1.0)


# -------------------------------------------------------------- admission

def simulate(adm, reqs, service):
    """Event-driven stub executor: requests (id, arrival, footprint) are pushed
    at their arrival times, admitted by the policy whenever something changes,
    and finish `service(id)` seconds after admission.  Returns the admission
    log, rejections, and the largest budget use seen."""
    events = [(t, 0, i) for i, (_, t, _) in enumerate(reqs)]   # (time, kind 0 arrive / 1 finish, index)
    heapq.heapify(events)
    fp = {rid: f for rid, _, f in reqs}
    slot_of, log, rejected, peak = {}, [], [], 0
    while events:
        t, kind, i = heapq.heappop(events)
        if kind == 0:
            adm.push(reqs[i][0], reqs[i][2])
        else:
            rid = reqs[i][0]
            assert adm.release(slot_of.pop(rid), fp[rid]) == bfal.BF_OK
        while True:
            d, rid, slot = adm.next()
            if d == 0:
                break
            if d < 0:
                rejected.append(rid)
                continue
            assert slot not in slot_of.values()
            slot_of[rid] = slot
            log.append((t, rid, slot))
            peak = max(peak, adm.used())
            j = next(k for k, r in enumerate(reqs) if r[0] == rid)
            heapq.heappush(events, (t + service(rid), 1, j))
    return log, rejected, peak


def test_admission_fifo_budget_and_slots():
    rng = np.random.default_rng(7)
    n, budget, slots = 200, 1000, 4
    reqs = [(100 + i, float(t), int(f)) for i, (t, f) in
            enumerate(zip(np.cumsum(rng.exponential(1.0, n)), rng.integers(50, 700, n)))]
    adm = bfal.Admission(budget, slots)
    log, rejected, peak = simulate(adm, reqs, lambda rid: 3.0 + (rid % 5))
    assert not rejected
    # arrival order is kept (head-of-line: nobody overtakes a waiting request)
    assert [rid for _, rid, _ in log] == [r[0] for r in reqs]
    assert peak <= budget
    assert adm.used() == 0 and adm.active() == 0 and adm.waiting() == 0
    # never more than `slots` admitted at once
    t_adm = {rid: t for t, rid, _ in log}
    for t, rid, _ in log:
        running = [r for r in t_adm if t_adm[r] <= t < t_adm[r] + 3.0 + (r % 5)]
        assert len(running) <= slots


def test_admission_rejects_what_can_never_fit_without_blocking():
    adm = bfal.Admission(1000, 2)
    for rid, f in [(1, 400), (2, 5000), (3, 400), (4, 300)]:
        adm.push(rid, f)
    assert adm.next() == (1, 1, 0)
    assert adm.next() == (-1, 2, -1)          # larger than the whole budget: rejected at the head
    assert adm.next() == (1, 3, 1)
    assert adm.next() == (0, None, None)      # 4 fits the budget (800 + 300 > 1000? no: waits for a slot)
    assert adm.used() == 800 and adm.waiting() == 1 and adm.active() == 2
    assert adm.release(0, 400) == bfal.BF_OK
    assert adm.next() == (1, 4, 0)            # the freed slot is reused
    assert adm.used() == 700


def test_admission_waits_for_budget_not_only_slots():
    adm = bfal.Admission(1000, 8)
    adm.push(1, 600)
    adm.push(2, 600)
    assert adm.next()[0] == 1
    assert adm.next() == (0, None, None)      # a slot is free but 1200 > 1000
    assert adm.release(0, 600) == 0
    assert adm.next()[:2] == (1, 2)


def test_admission_release_is_checked():
    adm = bfal.Admission(1000, 2)
    adm.push(1, 100)
    assert adm.next()[0] == 1
    assert adm.release(1, 100) == INVALID     # slot 1 is not in use
    assert adm.release(0, 99) == INVALID      # not the footprint admitted there
    assert adm.release(0, 100) == OK
    assert adm.release(0, 100) == INVALID     # already free


# ------------------------------------------------------------- slice plan

def plan_reference(wu, wl, pairs, nparts):
    """The plan restated in Python: eight windows of equal cost (by the cost
    prefix); each window in blocks of two slices per part, and inside a block
    the costliest slices first (stable), each to the least-loaded part of the
    XCD."""
    cost = (np.maximum(wu, wl) + pairs - 1) // pairs + 1
    ns, per_x = len(cost), nparts // 8
    load = np.zeros(nparts, np.int64)
    part_of = np.empty(ns, np.int64)
    before = np.concatenate([[0], np.cumsum(cost)[:-1]])   # cost of the slices before each one
    tot = int(cost.sum())
    win = [0] + [int(np.argmax(8 * before >= x * tot)) if (8 * before >= x * tot).any() else ns
                 for x in range(1, 8)] + [ns]
    for x in range(8):
        lx = load[x * per_x:(x + 1) * per_x]
        for b0 in range(win[x], win[x + 1], 2 * per_x):
            blk = np.arange(b0, min(b0 + 2 * per_x, win[x + 1]))
            for s in blk[np.argsort(-cost[blk], kind="stable")]:
                b = int(np.argmin(lx))
                lx[b] += cost[s]
                part_of[s] = x * per_x + b
    return part_of, load


@pytest.mark.parametrize("ns,nparts,seed", [(1, 8, 0), (37, 32, 1), (700, 1024, 2), (6300, 1024, 3), (5000, 64, 4)])
def test_slice_plan_lists_every_slice_once_in_its_window(ns, nparts, seed):
    rng = np.random.default_rng(seed)
    wu = rng.integers(0, 9, ns)
    wl = rng.integers(0, 9, ns)
    hot = rng.random(ns) < 0.05            # clustered wide (contact) slices
    wu[hot] += 20
    slot_u = np.concatenate([[0], np.cumsum(64 * wu)])
    slot_l = np.concatenate([[0], np.cumsum(64 * wl)])
    st, ptr, out = bfal.slice_plan(slot_u, slot_l, 2, nparts)
    assert st == OK
    assert ptr[0] == 0 and ptr[-1] == ns and np.all(np.diff(ptr) >= 0)
    assert np.array_equal(np.sort(out), np.arange(ns))            # every slice exactly once
    part_of, load = plan_reference(wu, wl, 2, nparts)
    for p in range(nparts):
        lst = out[ptr[p]:ptr[p + 1]]
        assert np.all(np.diff(lst) > 0)                           # increasing, the order it is processed in
        assert np.all(part_of[lst] == p)                          # the restated rule's assignment
    # balance: no part exceeds the even share by more than one slice's cost
    cost = (np.maximum(wu, wl) + 1) // 2 + 1
    per_x = nparts // 8
    for x in range(8):
        lx = load[x * per_x:(x + 1) * per_x]
        assert lx.max() - lx.min() <= cost.max()


def test_slice_plan_balances_better_than_round_robin():
    """Clustered wide slices (contact interfaces) as on the large workload:
    the plan's heaviest part carries less than round-robin's."""
    ns, nparts = 6300, 1024
    wu = np.full(ns, 7)
    for c in (1220, 2480, 3740, 5000):
        wu[c:c + 80] = 25
    slot = np.concatenate([[0], np.cumsum(64 * wu)])
    st, ptr, out = bfal.slice_plan(slot, slot, 2, nparts)
    assert st == OK
    cost = (wu + 1) // 2 + 1
    plan_max = max(cost[out[ptr[p]:ptr[p + 1]]].sum() for p in range(nparts))
    rr_max = max(cost[p::nparts].sum() for p in range(nparts))
    assert plan_max < rr_max
    assert plan_max <= cost.sum() / nparts + cost.max()


def test_slice_plan_argument_errors():
    good = np.arange(0, 64 * 5, 64)
    assert bfal.slice_plan(good, good, 2, 12)[0] == INVALID          # not a multiple of 8
    assert bfal.slice_plan(good, good, 0, 8)[0] == INVALID           # pairs < 1
    assert bfal.slice_plan(good + 1, good, 2, 8)[0] == INVALID       # not multiples of 64
    assert bfal.slice_plan(good[::-1].copy(), good, 2, 8)[0] == INVALID   # decreasing
    st, ptr, out = bfal.slice_plan(good[::-1].copy(), good, 2, 8)
    assert np.all(ptr == -7) and np.all(out == -7)                 # nothing written on an error
