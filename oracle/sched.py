"""Admission passes and scheduler state -- CPU oracle (test infrastructure only).

Paper: Sec. III-B "Shared Memory Data" (total memory, total used, itemised
use per client, queue of waiting clients with optional priority), Sec. IV
(pre-allocation and post-free checks) and Sec. V (the four notification
policies).  All arithmetic is exact integer byte accounting; nothing is
rounded anywhere in admission.

Conventions shared with the C-ABI contract (stated, not imported):
* a queue is an int64 array of declared demands in arrival order; an entry
  with a negative demand is a withdrawn request (a hole): it is neither
  admitted nor does it block anything;
* ``R`` is the free memory seen by the pass, capacity minus the sum of the
  reservations of running jobs (Sec. III-B: total minus total used).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

FIFO = 0
MMU = 1
PRIO_FIFO = 2
PRIO_MMU = 3

OK = 0
NOT_READY = 1
TIMEOUT = 2
E_INVALID = -1
E_TOOBIG = -2


# ---------------------------------------------------------------------------
# Single passes over an ordered queue
# ---------------------------------------------------------------------------
def fifo_pass(demand, R: int):
    """Policy 1, FIFO (Sec. V, and its recursive definition): the first waiting
    client is served if its demand fits the free memory; while memory remains,
    the next one is served; the first client that does not fit stops the pass.

    The admitted set is therefore the longest prefix of present entries whose
    demand sum is <= R.  Returns (admit: bool[n], R_after).

    The prefix sums are exact for any int64 demands: numpy's int64 cumsum is
    used only when no sum can leave the int64 range, Python integers
    otherwise."""
    d = np.asarray(demand, dtype=np.int64)
    present = d >= 0
    if d.size == 0 or int(d.max()) * d.size < 2**63:
        S = np.cumsum(np.where(present, d, 0))
    else:
        S = np.fromiter(itertools.accumulate(v if v >= 0 else 0 for v in d.tolist()),
                        dtype=object, count=d.size)
    over = np.nonzero(present & (S > R))[0]
    k = int(over[0]) if over.size else d.size
    admit = present.copy()
    admit[k:] = False
    used = int(S[k - 1]) if k > 0 else 0
    return admit, int(R) - used


def mmu_pass(demand, R: int):
    """Policy 2, Maximum Memory Utilisation (Sec. V, and its recursive
    definition): walking the queue in order, every client whose demand fits
    the memory that is still free is served; a client that does not fit keeps
    waiting while the walk continues with the next one.  This is greedy
    first-fit in queue order.  The walk may stop once R == 0 because every
    present demand is >= 1.  Returns (admit: bool[n], R_after)."""
    d = np.asarray(demand, dtype=np.int64)
    admit = np.zeros(d.size, dtype=bool)
    R = int(R)
    for i in range(d.size):
        if R == 0:
            break
        di = int(d[i])
        if 0 <= di <= R:
            admit[i] = True
            R -= di
    return admit, R


def mmu_pass_rounds(demand, R: int):
    """MMU computed as iterative rounds (the formulation the device kernels
    use): each round takes the present entries after the last break whose
    demand is <= R, admits the longest prefix of them whose sum is <= R,
    subtracts that sum, and restarts after the first candidate that did not
    fit (its demand now exceeds R, and R never grows within a pass, so it can
    never fit later).  Equal to ``mmu_pass``; kept as a second statement so
    the tests can show the equivalence.  Returns (admit, R_after, rounds)."""
    d = np.asarray(demand, dtype=np.int64)
    admit = np.zeros(d.size, dtype=bool)
    R = int(R)
    start = 0
    rounds = 0
    while start < d.size and R > 0:
        rounds += 1
        seg = d[start:]
        cand = (seg >= 0) & (seg <= R)
        S = np.cumsum(np.where(cand, seg, 0))
        brk = np.nonzero(cand & (S > R))[0]
        if brk.size == 0:
            admit[start:] = cand
            R -= int(S[-1])
            break
        b = int(brk[0])
        admit[start:start + b] = cand[:b]
        R -= int(S[b - 1]) if b > 0 else 0
        start += b + 1
    return admit, R, rounds


def priority_order(prio, seq=None):
    """Queue order for the priority policies (Sec. V, Policies 3 and 4): a
    lower ``priority`` value is a higher priority (Sec. IV, initialisation
    parameters); equal priorities keep arrival order."""
    prio = np.asarray(prio, dtype=np.int64)
    seq = np.arange(prio.size) if seq is None else np.asarray(seq, dtype=np.int64)
    return np.lexsort((seq, prio))


def policy_pass(policy: int, demand, R: int, prio=None):
    """One pass of any of the four policies.  Policy 3 (Priority FIFO) is FIFO
    over the queue ordered by (priority, arrival); Policy 4 (Priority MMU) is
    first-fit over the same order.  Returns (admit in original order, R_after)."""
    d = np.asarray(demand, dtype=np.int64)
    if policy in (FIFO, MMU):
        return (fifo_pass if policy == FIFO else mmu_pass)(d, R)
    order = priority_order(prio if prio is not None else np.zeros(d.size, np.int64))
    a, R2 = (fifo_pass if policy == PRIO_FIFO else mmu_pass)(d[order], R)
    admit = np.zeros(d.size, dtype=bool)
    admit[order] = a
    return admit, R2


def first_fit_fixed_point(demand, R: int, admit) -> bool:
    """Characterisation of the first-fit (MMU) result: the admitted set A is
    the only subset with  i in A  <=>  d_i <= R - sum_{j<i, j in A} d_j  for
    every present entry i (withdrawn entries never in A).  Checked with one
    exclusive prefix sum, so it verifies a pass of any size."""
    d = np.asarray(demand, dtype=np.int64)
    a = np.asarray(admit, dtype=bool)
    if np.any(a & (d < 0)):
        return False
    taken = np.where(a, d, 0)
    excl = np.cumsum(taken) - taken
    fits = (d >= 0) & (d <= int(R) - excl)
    return bool(np.array_equal(fits, a))


def fifo_prefix_check(demand, R: int, admit) -> bool:
    """Characterisation of the FIFO result: admitted entries are exactly the
    present entries before the first present entry whose inclusive prefix sum
    of present demands exceeds R."""
    ref, _ = fifo_pass(demand, R)
    return bool(np.array_equal(ref, np.asarray(admit, dtype=bool)))


# ---------------------------------------------------------------------------
# Scheduler state (Sec. III-B) with the life-cycle calls of Sec. IV
# ---------------------------------------------------------------------------
@dataclass
class Request:
    rid: int          # unique arrival sequence number
    job: int
    prio: int
    demand: int
    state: str = "PENDING"   # PENDING / ADMITTED / WITHDRAWN


@dataclass
class PassRecord:
    pending_rids: list
    demands: list
    prios: list
    R_before: int
    admitted_rids: list
    R_after: int


@dataclass
class Scheduler:
    """Total memory, total used, itemised use per client and the queue of
    waiting requests (Sec. III-B).  ``admit`` is pre-allocation, ``release`` is
    post-free (Sec. IV).  A pass runs after every arrival and every release."""

    capacity: int
    policy: int = MMU
    used: int = 0
    jobs: dict = field(default_factory=dict)        # job -> {"prio", "timeout_ms", "res", "owner"}
    alive: object = None                            # pid -> bool, for the sanity checks
    requests: list = field(default_factory=list)    # all requests by rid
    log: list = field(default_factory=list)

    def register(self, prio: int = 0, timeout_ms: int = 60000) -> int:
        j = len(self.jobs)
        self.jobs[j] = {"prio": int(prio), "timeout_ms": int(timeout_ms), "res": 0, "owner": 0}
        return j

    def set_owner(self, job: int, pid: int) -> int:
        """The process that holds the job's memory (0: none, never reclaimed)."""
        if job not in self.jobs or pid < 0:
            return E_INVALID
        self.jobs[job]["owner"] = int(pid)
        return OK

    def sanity(self, alive) -> tuple:
        """Sanity check (Sec. III-B, third robustness feature; Sec. IV): every
        job whose owner process is no longer alive loses its waiting requests
        and its whole reservation, which then serves the waiters (one pass,
        when anything was reclaimed).  ``alive(pid)`` answers for a process.
        Returns (jobs reclaimed, bytes reclaimed)."""
        jobs, nbytes = 0, 0
        for j, info in self.jobs.items():
            if info["owner"] > 0 and not alive(info["owner"]):
                self.withdraw(j)
                nbytes += info["res"]
                self.used -= info["res"]
                info["res"] = 0
                info["owner"] = 0
                jobs += 1
        if jobs:
            self.run_pass()
        return jobs, nbytes

    def pending(self):
        return [r for r in self.requests if r.state == "PENDING"]

    def run_pass(self):
        """Apply the policy to the waiting requests in arrival order."""
        pend = self.pending()
        R = self.capacity - self.used
        d = np.array([r.demand for r in pend], dtype=np.int64)
        p = np.array([r.prio for r in pend], dtype=np.int64)
        admit, R2 = policy_pass(self.policy, d, R, p)
        got = []
        for r, a in zip(pend, admit):
            if a:
                r.state = "ADMITTED"
                self.jobs[r.job]["res"] += r.demand
                self.used += r.demand
                got.append(r.rid)
        assert self.used == self.capacity - R2
        self.log.append(PassRecord([r.rid for r in pend], d.tolist(), p.tolist(), R, got, R2))
        return got

    def admit(self, job: int, device: int, nbytes: int) -> int:
        """Pre-allocation (Sec. IV): validate the device and the request, queue
        it behind the waiting requests, run a pass.  Returns OK if admitted in
        that pass, NOT_READY if it waits (the caller may withdraw it later)."""
        if job not in self.jobs or device != 0 or nbytes <= 0:
            return E_INVALID
        if nbytes > self.capacity:
            return E_TOOBIG
        r = Request(len(self.requests), job, self.jobs[job]["prio"], int(nbytes))
        self.requests.append(r)
        got = self.run_pass()
        if r.rid in got:
            return OK
        # memory is insufficient: check whether holders are still alive
        if self.alive is not None and self.sanity(self.alive)[0]:
            return OK if r.state == "ADMITTED" else NOT_READY
        return NOT_READY

    def withdraw(self, job: int) -> int:
        """A blocking pre-allocation whose timeout expired: its waiting requests
        leave the queue and are never admitted later."""
        n = 0
        for r in self.requests:
            if r.job == job and r.state == "PENDING":
                r.state = "WITHDRAWN"
                n += 1
        return n

    def release(self, job: int, device: int, nbytes: int) -> int:
        """Post-free (Sec. IV): the released bytes must not exceed what the job
        holds; 0 bytes means all of it, a negative device means every device.
        Frees the accounting, then serves waiters with a pass."""
        if job not in self.jobs or device > 0:
            return E_INVALID
        res = self.jobs[job]["res"]
        if nbytes < 0 or nbytes > res:
            return E_INVALID
        amount = res if nbytes == 0 else int(nbytes)
        self.jobs[job]["res"] -= amount
        self.used -= amount
        self.run_pass()
        # releasing everything is the client's shutdown (Sec. IV): it also
        # checks that the other holders are alive
        if nbytes == 0 and self.alive is not None:
            self.sanity(self.alive)
        return OK

    def check_invariants(self):
        assert 0 <= self.used <= self.capacity
        assert self.used == sum(j["res"] for j in self.jobs.values())
        return True


# ---------------------------------------------------------------------------
# The admission microbenchmark: rounds of "release a coin-chosen subset of
# the running jobs, then one pass" over one large queue
# ---------------------------------------------------------------------------
@dataclass
class RoundResult:
    admitted: np.ndarray      # int64 job ids admitted in this pass, queue order
    R_after: int
    used_after: int
    released: np.ndarray      # int64 job ids released before the pass


def release_rounds(demand, capacity: int, coins, rounds: int, policy: int = MMU):
    """Round 0 is one pass over the whole queue (job j = queue position j).
    In every later round r, each running job j with coins[r-1, j] == 1 posts a
    full release (Sec. IV post-free with bytes = 0), then one pass runs over
    the waiting requests in arrival order.  Returns one RoundResult per round."""
    d = np.asarray(demand, dtype=np.int64)
    pend = np.arange(d.size, dtype=np.int64)
    running = np.zeros(d.size, dtype=bool)
    used = 0
    out = []
    for r in range(rounds):
        rel = np.zeros(0, np.int64)
        if r > 0:
            rel_mask = running & (np.asarray(coins[r - 1]) != 0)
            rel = np.nonzero(rel_mask)[0]
            used -= int(d[rel].sum())
            running[rel] = False
        R = capacity - used
        if policy == FIFO:
            admit, R2 = fifo_pass(d[pend], R)
        else:
            admit, R2 = mmu_pass(d[pend], R)
        got = pend[admit]
        running[got] = True
        used = capacity - R2
        pend = pend[~admit]
        out.append(RoundResult(got, R2, used, rel))
    return out
