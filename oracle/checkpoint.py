"""Checkpoint, integrity check and recovery of the scheduler state -- CPU
oracle (test infrastructure only).

Paper: Sec. III-B, the first two robustness features of the shared-memory
design: each client keeps a backup of the shared structure, and a starting
client checks the structure for corruption and recovers it from the backup,
falling back to a fresh structure when the backup is missing or corrupt;
Sec. IV (initialisation) places that check in the client's start-up.

The record is the one the C ABI documents for sched_checkpoint, restated here
from that contract (nothing is imported from the HIP side), little-endian:

* header, 64 bytes: magic ``SCHEDCK1``; version 1 (u32); policy (i32);
  capacity, used (i64); n_jobs (i32); 0 (i32); n_pending (i64); checksum
  (u64); 0 (u64);
* per registered job, 24 bytes: priority, timeout_ms, owner pid, 0 (i32);
  reservation (i64);
* per waiting request, 16 bytes: demand (i64); job, priority (i32), in the
  order the policy serves them (arrival order; (priority, arrival) under the
  priority policies).  Withdrawn requests are not waiting and are left out.

The checksum is FNV-1a 64 (Fowler-Noll-Vo, the "1a" variant: xor the byte,
then multiply by the prime) over the whole record with the checksum field
set to zero.
"""
from __future__ import annotations

import struct

from .sched import PRIO_FIFO, PRIO_MMU, Request, Scheduler

FNV64_OFFSET = 0xCBF29CE484222325
FNV64_PRIME = 0x100000001B3
MAGIC = b"SCHEDCK1"
HEADER = struct.Struct("<8sIiqqiiqQQ")
JOB = struct.Struct("<iiiiq")
REQ = struct.Struct("<qii")
CHECKSUM_AT = 48          # byte offset of the checksum field in the header


def fnv1a64(data: bytes, h: int = FNV64_OFFSET) -> int:
    """FNV-1a, 64-bit: for every byte, h = (h xor byte) * prime mod 2^64."""
    for b in data:
        h = ((h ^ b) * FNV64_PRIME) & 0xFFFFFFFFFFFFFFFF
    return h


def checksum(record: bytes) -> int:
    """The record's checksum: FNV-1a 64 with the checksum field zeroed."""
    body = bytearray(record)
    body[CHECKSUM_AT:CHECKSUM_AT + 8] = bytes(8)
    return fnv1a64(bytes(body))


def waiting_in_service_order(s: Scheduler):
    """The waiting requests in the order the policy considers them (Sec. V):
    arrival order, or (priority, arrival) for Policies 3 and 4."""
    pend = s.pending()
    if s.policy in (PRIO_FIFO, PRIO_MMU):
        pend = sorted(pend, key=lambda r: (r.prio, r.rid))
    return pend


def encode(s: Scheduler) -> bytes:
    """The backup of a scheduler's state (first robustness feature)."""
    pend = waiting_in_service_order(s)
    jobs = [s.jobs[j] for j in range(len(s.jobs))]
    body = b"".join(JOB.pack(j["prio"], j["timeout_ms"], j["owner"], 0, j["res"]) for j in jobs)
    body += b"".join(REQ.pack(r.demand, r.job, r.prio) for r in pend)
    head = HEADER.pack(MAGIC, 1, s.policy, s.capacity, s.used, len(jobs), 0, len(pend), 0, 0)
    rec = head + body
    return rec[:CHECKSUM_AT] + struct.pack("<Q", checksum(rec)) + rec[CHECKSUM_AT + 8:]


def decode(record: bytes, max_jobs: int):
    """Integrity check (second robustness feature).  Returns
    (header dict, jobs, requests) for an intact record whose accounting is
    consistent, else None.  Consistent means: every reservation in
    [0, capacity], their sum equal to the used total (Sec. III-B: total used
    is the sum of the itemised uses), used within the capacity, and every
    waiting request naming a job of the record, carrying that job's priority
    and a demand in [1, capacity]."""
    if len(record) < HEADER.size:
        return None
    (magic, version, policy, capacity, used, n_jobs, zero, n_pending, csum,
     _pad) = HEADER.unpack_from(record, 0)
    if magic != MAGIC or version != 1:
        return None
    if not (0 <= n_jobs <= max_jobs) or n_pending < 0:
        return None
    if len(record) != HEADER.size + JOB.size * n_jobs + REQ.size * n_pending:
        return None
    if checksum(record) != csum:
        return None
    if capacity <= 0 or not (0 <= used <= capacity):
        return None
    jobs = [JOB.unpack_from(record, HEADER.size + JOB.size * k) for k in range(n_jobs)]
    base = HEADER.size + JOB.size * n_jobs
    reqs = [REQ.unpack_from(record, base + REQ.size * k) for k in range(n_pending)]
    if any(r < 0 or r > capacity or owner < 0 or z != 0 for (_p, _t, owner, z, r) in jobs):
        return None
    if sum(r for (*_x, r) in jobs) != used:
        return None
    for demand, job, prio in reqs:
        if not (0 <= job < n_jobs) or not (1 <= demand <= capacity) or prio != jobs[job][0]:
            return None
    head = {"policy": policy, "capacity": capacity, "used": used, "n_jobs": n_jobs,
            "n_pending": n_pending, "reserved": zero}
    return head, jobs, reqs


def restore(record: bytes, policy: int, capacity: int, max_jobs: int):
    """Recovery (Sec. III-B; Sec. IV initialisation): a scheduler rebuilt from
    an intact record of the same pool and policy, its jobs numbered as in the
    record and its waiting requests re-queued in the record's order.  None
    when the record fails the integrity check or belongs to another pool --
    the caller then keeps a freshly initialised scheduler."""
    got = decode(record, max_jobs)
    if got is None:
        return None
    head, jobs, reqs = got
    if head["policy"] != policy or head["capacity"] != capacity:
        return None
    s = Scheduler(capacity, policy)
    for prio, timeout_ms, owner, _z, res in jobs:
        j = s.register(prio, timeout_ms)
        s.jobs[j]["owner"] = owner
        s.jobs[j]["res"] = res
    s.used = head["used"]
    for demand, job, prio in reqs:
        s.requests.append(Request(len(s.requests), job, prio, demand))
    return s
