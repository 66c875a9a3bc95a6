"""Pins for the admission oracle (oracle/sched.py): hand-worked fixtures,
closed forms, brute-force enumeration and invariants.  CPU only."""
import itertools
import os

import numpy as np
import pytest

from oracle import sched as S
from workloads import c2_queue, random_queue

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
POL = {"FIFO": S.FIFO, "MMU": S.MMU, "PFIFO": S.PRIO_FIFO, "PMMU": S.PRIO_MMU}


def _ints(s):
    s = s.strip()
    return [int(x) for x in s.split()] if s and s != "-" else []


def load_policy_cases():
    cases = []
    with open(os.path.join(GOLDEN, "policies.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            pol, R, d, p, adm, R2 = [x.strip() for x in line.split("|")]
            cases.append((POL[pol], int(R), _ints(d), _ints(p) or None, _ints(adm), int(R2)))
    return cases


@pytest.mark.parametrize("case", load_policy_cases())
def test_golden_policy_passes(case):
    pol, R, d, p, adm, R2 = case
    admit, Rout = S.policy_pass(pol, np.array(d, np.int64), R, p)
    assert list(np.nonzero(admit)[0]) == adm
    assert Rout == R2


# ---------------------------------------------------------------- brute force
def brute_fifo(d, R):
    """Longest prefix of present entries with sum <= R, by enumerating every
    prefix length."""
    best = 0
    for m in range(len(d) + 1):
        if sum(x for x in d[:m] if x >= 0) <= R:
            best = m
        else:
            break
    # a prefix that ends on holes is equivalent; admitted = present in [0, best)
    return [i for i in range(best) if d[i] >= 0]


def fixed_point_subsets(d, R):
    """Every subset A of present entries with  i in A <=> d_i <= R - sum_{j<i, j in A} d_j."""
    n = len(d)
    sols = []
    for mask in range(1 << n):
        A = [i for i in range(n) if mask >> i & 1]
        if any(d[i] < 0 for i in A):
            continue
        ok = True
        for i in range(n):
            if d[i] < 0:
                continue
            room = R - sum(d[j] for j in A if j < i)
            if (i in A) != (d[i] <= room):
                ok = False
                break
        if ok:
            sols.append(A)
    return sols


def knapsack_best(d, R):
    best = 0
    items = [x for x in d if x >= 0]
    for r in range(len(items) + 1):
        for comb in itertools.combinations(items, r):
            s = sum(comb)
            if s <= R:
                best = max(best, s)
    return best


@pytest.mark.parametrize("seed", range(200))
def test_fifo_equals_prefix_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 12))
    d = random_queue(seed, n, 20, holes=0.2 if seed % 2 else 0.0)
    R = int(rng.integers(0, 60))
    admit, R2 = S.fifo_pass(d, R)
    ref = brute_fifo(list(d), R)
    assert list(np.nonzero(admit)[0]) == ref
    assert R2 == R - sum(d[i] for i in ref)


@pytest.mark.parametrize("seed", range(300))
def test_mmu_is_unique_fixed_point(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(0, 11))
    d = random_queue(1000 + seed, n, 16, holes=0.15 if seed % 3 == 0 else 0.0)
    R = int(rng.integers(0, 50))
    admit, R2 = S.mmu_pass(d, R)
    sols = fixed_point_subsets(list(d), R)
    assert len(sols) == 1
    assert list(np.nonzero(admit)[0]) == sols[0]
    assert R2 == R - sum(d[i] for i in sols[0])
    assert S.first_fit_fixed_point(d, R, admit)
    # greedy never beats the best packing (it is not optimal in general)
    assert R - R2 <= knapsack_best(list(d), R)


def test_mmu_not_optimal_example():
    d = np.array([6, 5, 5], np.int64)
    admit, R2 = S.mmu_pass(d, 10)
    assert 10 - R2 == 6 and knapsack_best(list(d), 10) == 10


@pytest.mark.parametrize("seed", range(300))
def test_rounds_equal_greedy(seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(0, 400))
    d = random_queue(5000 + seed, n, int(rng.integers(1, 1000)), holes=0.1 if seed % 2 else 0.0)
    R = int(rng.integers(0, 20000))
    a1, r1 = S.mmu_pass(d, R)
    a2, r2, _ = S.mmu_pass_rounds(d, R)
    assert np.array_equal(a1, a2) and r1 == r2


def test_rounds_adversarial_needs_many_rounds():
    R = 1000
    d = np.array([x for k in range(50) for x in (1, R - k)], np.int64)
    a1, r1 = S.mmu_pass(d, R)
    a2, r2, rounds = S.mmu_pass_rounds(d, R)
    assert np.array_equal(a1, a2) and r1 == r2
    assert a1.sum() == 50 and rounds >= 50


@pytest.mark.parametrize("seed", range(100))
def test_fifo_prefix_of_mmu_and_maximality(seed):
    rng = np.random.default_rng(9000 + seed)
    d = random_queue(9000 + seed, int(rng.integers(1, 300)), 100, holes=0.1)
    R = int(rng.integers(0, 3000))
    af, rf = S.fifo_pass(d, R)
    am, rm = S.mmu_pass(d, R)
    # FIFO's admitted set is MMU's admitted set restricted to FIFO's prefix
    k = np.nonzero(af)[0]
    last = int(k[-1]) + 1 if k.size else 0
    assert np.array_equal(af[:last], am[:last])
    assert rm <= rf
    # MMU is maximal: every present, rejected entry exceeds the final free memory
    rej = (~am) & (d >= 0)
    assert np.all(d[rej] > rm)


def test_closed_forms():
    for d0 in (1, 7, 4096):
        for n in (0, 1, 5, 100):
            for R in (0, d0 - 1, d0, 3 * d0 + 1, 1000 * d0):
                d = np.full(n, d0, np.int64)
                for f in (S.fifo_pass, S.mmu_pass):
                    admit, R2 = f(d, R)
                    k = min(n, R // d0)
                    assert admit.sum() == k and np.all(admit[:k])
                    assert R2 == R - k * d0
    d = np.array([5, 3, 9], np.int64)
    assert S.fifo_pass(d, 17)[0].all() and S.mmu_pass(d, 17)[0].all()      # R >= sum
    assert not S.fifo_pass(d, 4)[0].any()                                    # R < d0


def test_fixed_point_checker_rejects_any_single_flip():
    for seed in range(50):
        d = random_queue(seed, 60, 50, holes=0.1)
        R = 600
        admit, _ = S.mmu_pass(d, R)
        assert S.first_fit_fixed_point(d, R, admit)
        for i in range(d.size):
            bad = admit.copy()
            bad[i] = ~bad[i]
            assert not S.first_fit_fixed_point(d, R, bad)


def test_batching_changes_mmu_but_not_fifo():
    # two passes (R = 5, then 8 more freed) vs one coalesced pass (R = 13)
    d = np.array([10, 4], np.int64)
    a1, r1 = S.mmu_pass(d, 5)
    a2, _ = S.mmu_pass(d[~a1], r1 + 8)
    assert list(np.nonzero(a1)[0]) == [1] and not a2.any()
    a3, _ = S.mmu_pass(d, 13)
    assert list(np.nonzero(a3)[0]) == [0]
    f1, q1 = S.fifo_pass(d, 5)
    f2, _ = S.fifo_pass(d[~f1], q1 + 8)
    f3, _ = S.fifo_pass(d, 13)
    assert (f1.sum() + f2.sum()) == f3.sum() == 1


def test_priority_order_and_policies():
    prio = np.array([2, 0, 1, 0, 2, 1])
    assert list(S.priority_order(prio)) == [1, 3, 2, 5, 0, 4]
    rng = np.random.default_rng(7)
    for _ in range(200):
        n = int(rng.integers(0, 30))
        d = rng.integers(1, 30, size=n).astype(np.int64)
        p = rng.integers(0, 3, size=n)
        R = int(rng.integers(0, 200))
        order = sorted(range(n), key=lambda i: (p[i], i))
        for pol, base in ((S.PRIO_FIFO, S.fifo_pass), (S.PRIO_MMU, S.mmu_pass)):
            a, r = S.policy_pass(pol, d, R, p)
            b, rb = base(d[order], R)
            assert r == rb
            assert sorted(np.nonzero(a)[0]) == sorted(np.array(order, int)[b]) if n else True
        # equal priorities reduce to the plain policies
        for pol, base in ((S.PRIO_FIFO, S.fifo_pass), (S.PRIO_MMU, S.mmu_pass)):
            a, r = S.policy_pass(pol, d, R, np.zeros(n, int))
            b, rb = base(d, R)
            assert np.array_equal(a, b) and r == rb


# ------------------------------------------------------------ scheduler state
def test_scheduler_lifecycle_checks():
    s = S.Scheduler(100, S.MMU)
    j = s.register(0, 1000)
    assert s.admit(j, 1, 10) == S.E_INVALID          # bad device
    assert s.admit(j, 0, 0) == S.E_INVALID           # no bytes
    assert s.admit(99, 0, 5) == S.E_INVALID          # unknown job
    assert s.admit(j, 0, 101) == S.E_TOOBIG
    assert s.admit(j, 0, 60) == S.OK
    k = s.register()
    assert s.admit(k, 0, 50) == S.NOT_READY
    assert s.release(j, 0, 61) == S.E_INVALID        # more than held
    assert s.release(j, 0, 10) == S.OK               # partial: 50 free -> k admitted
    assert s.jobs[k]["res"] == 50 and s.used == 100
    assert s.release(j, -1, 0) == S.OK               # all of it, every device
    assert s.jobs[j]["res"] == 0 and s.used == 50
    s.check_invariants()


def test_scheduler_withdraw_and_idempotent_pass():
    s = S.Scheduler(10, S.FIFO)
    a, b, c = s.register(), s.register(), s.register()
    assert s.admit(a, 0, 8) == S.OK
    assert s.admit(b, 0, 5) == S.NOT_READY
    assert s.admit(c, 0, 1) == S.NOT_READY           # FIFO: blocked behind b
    assert s.withdraw(b) == 1
    assert s.run_pass() == [2]                         # c no longer blocked
    assert s.run_pass() == []                          # nothing new: admits nothing
    s.release(a, 0, 0)
    assert s.jobs[b]["res"] == 0                       # withdrawn, never admitted later


def test_scheduler_serial_special_case():
    C = 1000
    s = S.Scheduler(C, S.MMU)
    jobs = [s.register() for _ in range(6)]
    states = [s.admit(j, 0, C) for j in jobs]
    assert states == [S.OK] + [S.NOT_READY] * 5
    for i in range(5):
        s.release(jobs[i], 0, 0)
        running = [j for j in jobs if s.jobs[j]["res"] > 0]
        assert running == [jobs[i + 1]]


@pytest.mark.parametrize("policy", [S.FIFO, S.MMU, S.PRIO_FIFO, S.PRIO_MMU])
def test_scheduler_random_invariants(policy):
    rng = np.random.default_rng(policy)
    s = S.Scheduler(1000, policy)
    jobs = [s.register(int(rng.integers(0, 3))) for _ in range(40)]
    for step in range(400):
        j = jobs[int(rng.integers(0, len(jobs)))]
        op = rng.random()
        if op < 0.5:
            s.admit(j, 0, int(rng.integers(1, 400)))
        elif op < 0.9:
            s.release(j, -1, 0 if rng.random() < 0.5 else int(rng.integers(0, s.jobs[j]["res"] + 1)))
        else:
            s.withdraw(j)
        s.check_invariants()
    # every pass in the log is reproduced exactly by a fresh single pass
    for rec in s.log:
        a, r = S.policy_pass(policy, np.array(rec.demands, np.int64), rec.R_before,
                             np.array(rec.prios, np.int64))
        assert [rid for rid, x in zip(rec.pending_rids, a) if x] == rec.admitted_rids
        assert r == rec.R_after
        if policy == S.FIFO:
            # FIFO order: nothing admitted while an earlier request keeps waiting
            got = set(rec.admitted_rids)
            waiting = [rid for rid in rec.pending_rids if rid not in got]
            if waiting:
                assert all(rid < waiting[0] for rid in got)


def test_release_rounds_invariants_small():
    q = c2_queue(seed=11, n=1 << 12, capacity=3 * 10**10)
    res = S.release_rounds(q.demand, q.capacity, q.coins, q.rounds, S.MMU)
    running = np.zeros(q.n, bool)
    pend = np.ones(q.n, bool)
    for r, rr in enumerate(res):
        running[rr.released] = False
        assert np.all(pend[rr.admitted]) and not np.any(running[rr.admitted])
        R = q.capacity - int(q.demand[running].sum())
        # the pass over the waiting queue is the unique first-fit fixed point
        idx = np.nonzero(pend)[0]
        admit = np.isin(idx, rr.admitted)
        assert S.first_fit_fixed_point(q.demand[idx], R, admit)
        running[rr.admitted] = True
        pend[rr.admitted] = False
        assert rr.used_after == int(q.demand[running].sum()) <= q.capacity
        assert rr.R_after == q.capacity - rr.used_after


def test_c2_shape():
    q = c2_queue(seed=2, n=1 << 16)
    assert q.demand.min() >= 4096 and q.demand.max() < 4 * 2**30
    assert np.all(q.demand % 4096 == 0)
    assert q.coins.shape == (7, 1 << 16)
    assert 280 * 10**9 % 4096 == 0


# --------------------------------------------------------------------------
# Sanity check (Sec. III-B third robustness feature, Sec. IV): memory of
# clients whose process has ended is reclaimed for the waiting clients
# --------------------------------------------------------------------------
def _sched_with_dead(dead):
    sc = S.Scheduler(capacity=10_000, policy=S.MMU)
    sc.alive = lambda pid: pid not in dead
    return sc


def test_sanity_reclaims_on_insufficient_memory():
    dead = set()
    sc = _sched_with_dead(dead)
    a, b, c = sc.register(), sc.register(), sc.register()
    assert sc.set_owner(a, 101) == S.OK and sc.set_owner(b, 102) == S.OK
    assert sc.admit(a, 0, 6000) == S.OK and sc.admit(b, 0, 3000) == S.OK
    dead.add(101)                      # a's process ends without post-freeing
    # c does not fit beside a and b (6000 + 3000 + 2000 > 10000): the sanity
    # check frees a's 6000 bytes and c is admitted in the same call
    assert sc.admit(c, 0, 2000) == S.OK
    assert sc.jobs[a]["res"] == 0 and sc.jobs[b]["res"] == 3000 and sc.jobs[c]["res"] == 2000
    assert sc.used == 5000 and sc.check_invariants()
    assert sc.jobs[a]["owner"] == 0    # reclaimed once


def test_sanity_withdraws_requests_of_dead_jobs():
    dead = set()
    sc = _sched_with_dead(dead)
    a, b = sc.register(), sc.register()
    sc.set_owner(a, 201)
    assert sc.admit(a, 0, 7000) == S.OK
    assert sc.admit(a, 0, 5000) == S.NOT_READY     # a's second request waits
    dead.add(201)
    assert sc.sanity(sc.alive) == (1, 7000)
    # the waiting request was withdrawn, not admitted by the reclaim pass
    assert [r.state for r in sc.requests] == ["ADMITTED", "WITHDRAWN"]
    assert sc.used == 0 and sc.admit(b, 0, 10_000) == S.OK


def test_sanity_keeps_live_and_ownerless_holders():
    sc = _sched_with_dead({301})
    a, b, c = sc.register(), sc.register(), sc.register()
    sc.set_owner(a, 300)               # alive
    # b has no owner (0): never reclaimed, whatever the liveness answers
    assert sc.admit(a, 0, 4000) == S.OK and sc.admit(b, 0, 5000) == S.OK
    n_pass = len(sc.log)
    assert sc.admit(c, 0, 3000) == S.NOT_READY
    assert len(sc.log) == n_pass + 1   # the admit's own pass only: nothing reclaimed
    assert sc.sanity(sc.alive) == (0, 0) and sc.used == 9000


def test_sanity_at_shutdown_serves_waiters():
    dead = set()
    sc = _sched_with_dead(dead)
    a, b, c = sc.register(), sc.register(), sc.register()
    sc.set_owner(a, 401)
    assert sc.admit(a, 0, 5000) == S.OK and sc.admit(b, 0, 4000) == S.OK
    assert sc.admit(c, 0, 6000) == S.NOT_READY
    dead.add(401)
    # b's shutdown (release of everything) frees 4000 -- not enough for c --
    # then checks the other holders: a's 5000 come back and c is admitted
    assert sc.release(b, 0, 0) == S.OK
    assert sc.jobs[c]["res"] == 6000 and sc.used == 6000 and sc.check_invariants()


def test_set_owner_rejects_bad_args():
    sc = S.Scheduler(capacity=100)
    a = sc.register()
    assert sc.set_owner(a, -1) == S.E_INVALID and sc.set_owner(7, 1) == S.E_INVALID


def _fifo_python(d, R):
    """Policy 1 with Python integers, entry by entry (no numpy sums)."""
    admit, s = [], 0
    for v in d:
        v = int(v)
        if v < 0:
            admit.append(False)
            continue
        if s + v > R:
            break
        s += v
        admit.append(True)
    admit += [False] * (len(d) - len(admit))
    return np.array(admit, bool), R - s


@pytest.mark.parametrize("seed", range(20))
def test_fifo_pass_exact_for_huge_demands(seed):
    """Demands near 2^62: the prefix sums leave the int64 range, where an
    int64 cumsum wraps (five such demands after a 1 sum to 1 modulo 2^64 and
    would read as fitting R = 10).  The pass equals the entry-by-entry Python
    integer walk."""
    d = np.array([1] + [1 << 62] * 4, np.int64)
    a, R2 = S.fifo_pass(d, 10)
    assert list(a) == [True, False, False, False, False] and R2 == 9
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    d = rng.integers(0, 1000, n).astype(np.int64)
    big = rng.random(n) < 0.3
    d[big] = (1 << 62) - rng.integers(0, 1 << 20, int(big.sum()))
    d[rng.random(n) < 0.1] = -1
    for R in (0, 10, 5000, (1 << 62) + 7, (1 << 63) - 1):
        a, R2 = S.fifo_pass(d, R)
        ra, rR2 = _fifo_python(d, R)
        assert np.array_equal(a, ra) and R2 == rR2
        assert S.fifo_prefix_check(d, R, a)
