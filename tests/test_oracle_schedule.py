"""Pins for the virtual-clock schedule oracle (oracle/schedule.py)."""
import os

import numpy as np
import pytest

from oracle import sched as S
from oracle import schedule as V
from workloads import c1_jobs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_cases():
    out = []
    with open(os.path.join(GOLDEN, "schedules.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            pol, cap, arr, dem, dur, ta, te = [x.strip() for x in line.split("|")]
            fl = lambda s: [float(x) for x in s.split()]
            out.append((S.FIFO if pol == "FIFO" else S.MMU, int(cap), fl(arr),
                        [int(x) for x in dem.split()], fl(dur), fl(ta), fl(te)))
    return out


@pytest.mark.parametrize("case", load_cases())
def test_golden_schedules(case):
    pol, cap, arr, dem, dur, ta, te = case
    r = V.simulate(arr, dem, dur, cap, pol)
    assert list(r["t_admit"]) == ta
    assert list(r["t_end"]) == te


def _running_never_exceeds(r, demand, cap):
    ev = []
    for j in range(len(demand)):
        if np.isnan(r["t_admit"][j]):
            continue
        ev.append((r["t_admit"][j], 1, demand[j]))
        ev.append((r["t_end"][j], 0, -demand[j]))
    ev.sort()
    cur = 0
    for _, _, dv in ev:
        cur += dv
        assert 0 <= cur <= cap


@pytest.mark.parametrize("policy", [S.FIFO, S.MMU])
def test_serial_closed_form(policy):
    """Demand := capacity (exclusive mode, Sec. IX) gives one job at a time in
    arrival order: admit_j = max(arrival_j, end_{j-1})."""
    rng = np.random.default_rng(3)
    n = 50
    arr = np.cumsum(rng.exponential(1.0, n))
    dur = rng.uniform(0.1, 3.0, n)
    C = 1000
    r = V.simulate(arr, np.full(n, C), dur, C, policy)
    prev = -np.inf
    for j in range(n):
        exp = max(arr[j], prev)
        assert r["t_admit"][j] == exp
        prev = exp + dur[j]


def test_unbounded_capacity_admits_on_arrival():
    q = c1_jobs(1)
    r = V.simulate(q.arrival_s, q.demand, np.full(q.n, 1e-3), 10**15, S.MMU)
    assert np.array_equal(r["t_admit"], q.arrival_s)


@pytest.mark.parametrize("policy", [S.FIFO, S.MMU])
def test_random_schedule_invariants(policy):
    rng = np.random.default_rng(10 + policy)
    n = 300
    arr = np.cumsum(rng.exponential(0.2, n))
    dem = rng.integers(1, 60, n)
    dur = rng.uniform(0.1, 5.0, n)
    C = 100
    r = V.simulate(arr, dem, dur, C, policy)
    assert np.all(r["t_admit"] >= arr)
    _running_never_exceeds(r, dem, C)
    if policy == S.FIFO:
        # FIFO: admission times are non-decreasing in arrival order
        assert np.all(np.diff(r["t_admit"]) >= 0)


def test_toobig_rejected():
    r = V.simulate([0.0, 1.0], [5, 50], [1.0, 1.0], 10, S.MMU)
    assert r["t_admit"][0] == 0.0 and np.isnan(r["t_admit"][1])


def test_percentile_nearest_rank():
    x = [15, 20, 35, 40, 50]
    assert V.percentile(x, 30) == 20
    assert V.percentile(x, 40) == 20
    assert V.percentile(x, 50) == 35
    assert V.percentile(x, 100) == 50
    assert V.percentile(list(range(1, 101)), 99) == 99


def test_head_of_line_fifo_vs_mmu():
    """The head-of-line case of Sec. V: a waiting request that does not fit
    holds every later one under FIFO, while MMU serves the later ones that fit
    (and, here, does not delay the blocker: the small jobs end long before the
    long job frees its memory)."""
    from workloads import HOL_BLOCKER, HOL_LONG, HOL_SMALL, hol_jobs, job_table
    mix = hol_jobs()
    jt = job_table(mix)
    cls = mix.extra["cls"]
    long_i = int(np.flatnonzero(cls == HOL_LONG)[0])
    blk = int(np.flatnonzero(cls == HOL_BLOCKER)[0])
    small = cls == HOL_SMALL
    # the blocker fits only once the long job has ended
    assert mix.demand[long_i] + mix.demand[blk] > mix.capacity
    out = {}
    for policy in (S.FIFO, S.MMU):
        ref = V.simulate(jt["arrival_s"], jt["demand"], jt["vdur_s"], mix.capacity, policy,
                         prio=jt["priority"])
        assert ref["t_admit"][blk] == ref["t_end"][long_i]
        out[policy] = ref
    fifo, mmu = out[S.FIFO], out[S.MMU]
    # FIFO: no small job passes the blocker
    assert np.all(fifo["t_admit"][small] >= fifo["t_admit"][blk])
    # MMU: every small job that arrives while the long job runs is admitted
    # on arrival (the free memory around it holds each of them)
    during = small & (jt["arrival_s"] < mmu["t_end"][long_i])
    assert during.sum() > 30
    assert np.array_equal(mmu["t_admit"][during], jt["arrival_s"][during])
    # and FIFO's small jobs that arrived during the long job waited for it
    assert np.all(fifo["t_admit"][during] >= fifo["t_end"][long_i])
