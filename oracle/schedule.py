"""Virtual-clock replay of a job mix through the scheduler -- CPU oracle.

Paper: Sec. II (four-stage life cycle: initialise, pre-allocate, post-free,
shut down) and Sec. V (waiting clients are served by the policy when memory
is freed).  Each job arrives, declares its demand (pre-allocation), runs for
a fixed virtual duration once admitted, then posts a full release.

Ordering (a reading; the paper does not fix it): events are processed one
at a time in the order (time, releases before arrivals, job index), and one
admission pass runs after every event.  A job's virtual duration is an input
(a function of its footprint supplied by the workload generator), so the
whole schedule is deterministic and a device-driven run must reproduce it
exactly.
"""
from __future__ import annotations

import heapq

import numpy as np

from . import sched as S

EV_RELEASE = 0
EV_ARRIVE = 1


def simulate(arrival_s, demand, vdur_s, capacity: int, policy: int = S.MMU, prio=None):
    """Returns dict of float64 arrays t_admit, t_end (seconds) and the pass
    count.  A job whose demand exceeds the capacity is rejected at arrival
    (t_admit = t_end = nan)."""
    arrival = np.asarray(arrival_s, dtype=np.float64)
    d = np.asarray(demand, dtype=np.int64)
    dur = np.asarray(vdur_s, dtype=np.float64)
    n = d.size
    prio = np.zeros(n, np.int64) if prio is None else np.asarray(prio, np.int64)
    t_admit = np.full(n, np.nan)
    t_end = np.full(n, np.nan)

    heap = [(float(arrival[j]), EV_ARRIVE, j) for j in range(n)]
    heapq.heapify(heap)
    pend = []          # job ids waiting, arrival order
    used = 0
    passes = 0
    while heap:
        t, ev, j = heapq.heappop(heap)
        if ev == EV_RELEASE:
            used -= int(d[j])
        else:
            if d[j] > capacity:
                continue
            pend.append(j)
        passes += 1
        if not pend:
            continue
        pd = d[pend]
        admit, R2 = S.policy_pass(policy, pd, capacity - used, prio[pend])
        used = capacity - R2
        keep = []
        for k, jj in enumerate(pend):
            if admit[k]:
                t_admit[jj] = t
                t_end[jj] = t + dur[jj]
                heapq.heappush(heap, (float(t_end[jj]), EV_RELEASE, jj))
            else:
                keep.append(jj)
        pend = keep
        assert 0 <= used <= capacity
    return {"t_admit": t_admit, "t_end": t_end, "passes": passes}


def percentile(x, p: float) -> float:
    """Nearest-rank percentile: the ceil(p n / 100)-th smallest value."""
    v = np.sort(np.asarray(x, dtype=np.float64))
    if v.size == 0:
        return float("nan")
    k = int(np.ceil(p * v.size / 100.0))
    return float(v[max(k, 1) - 1])
