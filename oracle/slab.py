"""Quota-checked slab sub-allocator -- CPU oracle (test infrastructure only).

The paper keeps an itemised record of the memory each client uses next to
the total in use (Sec. III-B, "Shared Memory Data"), and post-free only
accepts memory the client actually holds (Sec. IV).  The sub-allocator that
serves co-scheduled tenants extends that accounting to individual blocks:

* sizes are rounded up to a power-of-two class, 256 B .. 1 MiB (13 classes);
* an allocation charges its class size to the tenant (must stay <= quota)
  and to the pool (must stay <= pool size), then takes a free block of its
  class; any failure leaves no charge behind;
* a free returns a block the tenant holds and removes both charges; a free
  of anything else is invalid and changes nothing.

``simulate`` runs an op stream sequentially.  ``check_log`` validates a log
produced by concurrent execution, phase by phase, where the ops of one phase
may run in any order.  The number of blocks a class can hold is a parameter
(the device design states it).
"""
from __future__ import annotations

import numpy as np

MIN_LOG2 = 8          # 256 B
N_CLASSES = 13        # .. 1 MiB

ST_OK = 0
ST_QUOTA = 1          # tenant quota would be exceeded
ST_NOMEM_POOL = 2     # pool would be exceeded
ST_NOMEM_CLASS = 3    # no free block of the class
ST_INVALID = 4        # bad size, or free of a block not held

OP_ALLOC = 0
OP_FREE = 1


def size_class(size):
    """Smallest c with 256 * 2**c >= size (sizes 1 .. 1 MiB); -1 if invalid."""
    s = np.asarray(size, dtype=np.int64)
    c = np.zeros(s.shape, dtype=np.int64)
    for k in range(N_CLASSES):
        c += (s > (np.int64(1) << (MIN_LOG2 + k))).astype(np.int64)
    return np.where((s >= 1) & (s <= (1 << (MIN_LOG2 + N_CLASSES - 1))), c, -1)


def class_bytes(c):
    return np.int64(1) << (MIN_LOG2 + np.asarray(c, dtype=np.int64))


def simulate(kind, tenant, size, ref, quotas, pool: int, class_cap):
    """Sequential execution of an op stream.  Returns int8 status per op."""
    n = len(kind)
    quotas = np.asarray(quotas, dtype=np.int64)
    charged = np.zeros(quotas.size, dtype=np.int64)
    pool_used = 0
    live = np.zeros(N_CLASSES, dtype=np.int64)
    cls = size_class(size)
    status = np.zeros(n, dtype=np.int8)
    held = np.zeros(n, dtype=bool)          # alloc op i currently holds a block
    for i in range(n):
        t = int(tenant[i])
        if kind[i] == OP_ALLOC:
            c = int(cls[i])
            if c < 0:
                status[i] = ST_INVALID
                continue
            cs = 1 << (MIN_LOG2 + c)
            if charged[t] + cs > quotas[t]:
                status[i] = ST_QUOTA
            elif pool_used + cs > pool:
                status[i] = ST_NOMEM_POOL
            elif live[c] >= class_cap[c]:
                status[i] = ST_NOMEM_CLASS
            else:
                charged[t] += cs
                pool_used += cs
                live[c] += 1
                held[i] = True
                status[i] = ST_OK
        else:
            r = int(ref[i])
            if r < 0 or r >= i or kind[r] != OP_ALLOC or not held[r] or int(tenant[r]) != t:
                status[i] = ST_INVALID
                continue
            c = int(cls[r])
            cs = 1 << (MIN_LOG2 + c)
            charged[t] -= cs
            pool_used -= cs
            live[c] -= 1
            held[r] = False
            status[i] = ST_OK
    return status


def check_log(kind, tenant, size, ref, quotas, pool: int, class_cap, phase_len: int,
              status, ptr, pool_base: int, final_charged=None, final_pool=None, span=None):
    """Validate a concurrent allocator log.  Raises AssertionError naming the
    first violated invariant; returns a dict of counts otherwise.

    Per phase (ops of one phase are concurrent, phases are ordered):
    * frees: a free can succeed only when it names an alloc of the same
      tenant from an earlier phase that succeeded and is not yet freed; of
      the frees of one phase that name the same such alloc exactly one
      succeeds (a block is returned once, Sec. IV), every other free is
      invalid;
    * successful allocs: inside [pool_base, pool_base + span) (span defaults
      to the pool size) and aligned to their class size;
    * after the phase: live blocks do not overlap, each tenant's charge is
      <= its quota, the pool charge is <= the pool, a class holds at most
      its stated number of blocks;
    * no spurious reject: an alloc may fail on the quota only if the tenant's
      charge at phase start plus every other alloc of that tenant in the
      phase that got past its quota check, plus its own size, exceeds the
      quota (some order of the phase then makes it fail); likewise for the
      pool (allocs past the pool check) and for a class (allocs that took a
      block of that class).
    """
    kind = np.asarray(kind)
    tenant = np.asarray(tenant, dtype=np.int64)
    size = np.asarray(size, dtype=np.int64)
    ref = np.asarray(ref, dtype=np.int64)
    status = np.asarray(status, dtype=np.int64)
    ptr = np.asarray(ptr, dtype=np.uint64).astype(np.int64)  # device VAs are < 2**63
    quotas = np.asarray(quotas, dtype=np.int64)
    class_cap = np.asarray(class_cap, dtype=np.int64)
    T = quotas.size
    n = kind.size
    span = pool if span is None else int(span)
    cls = size_class(size)
    cs_all = np.where(cls >= 0, class_bytes(np.maximum(cls, 0)), 0)

    held = np.zeros(n, dtype=bool)
    charged = np.zeros(T, dtype=np.int64)
    pool_used = 0
    live = np.zeros(N_CLASSES, dtype=np.int64)
    counts = {"alloc_ok": 0, "free_ok": 0, "quota": 0, "nomem_pool": 0, "nomem_class": 0,
              "invalid": 0}
    for p0 in range(0, n, phase_len):
        p1 = min(p0 + phase_len, n)
        idx = np.arange(p0, p1)
        k = kind[p0:p1]
        st = status[p0:p1]
        is_alloc = k == OP_ALLOC
        # --- frees -----------------------------------------------------------
        fi = idx[~is_alloc]
        r = ref[fi]
        valid_ref = (r >= 0) & (r < p0)
        rr = np.where(valid_ref, r, 0)
        can_ok = valid_ref & (kind[rr] == OP_ALLOC) & held[rr] & (tenant[rr] == tenant[fi])
        got_ok = status[fi] == ST_OK
        bad = np.nonzero(got_ok & ~can_ok)[0]
        assert bad.size == 0, f"free status wrong at op {int(fi[bad[0]])}"
        # every held alloc named in the phase is freed exactly once
        named, inv = np.unique(rr[can_ok], return_inverse=True)
        wins = np.bincount(inv, weights=got_ok[can_ok].astype(np.int64), minlength=named.size)
        bad = np.nonzero(wins != 1)[0]
        assert bad.size == 0, (f"free status wrong: alloc op {int(named[bad[0]])} freed "
                               f"{int(wins[bad[0]])} times in one phase")
        assert np.all(status[fi][~got_ok] == ST_INVALID), "failed free not reported invalid"
        expect_ok = got_ok
        # --- allocs ----------------------------------------------------------
        ai = idx[is_alloc]
        a_st = status[ai]
        a_c = cls[ai]
        a_cs = cs_all[ai]
        a_t = tenant[ai]
        assert np.all((a_c >= 0) | (a_st == ST_INVALID)), "bad size not rejected"
        assert np.all((a_c < 0) | (a_st != ST_INVALID)), "valid size rejected as invalid"
        ok = a_st == ST_OK
        p_ok = ptr[ai][ok]
        cs_ok = a_cs[ok]
        assert np.all(p_ok >= pool_base) and np.all(p_ok + cs_ok <= pool_base + span), \
            "block outside the pool"
        assert np.all((p_ok - pool_base) % cs_ok == 0), "block not aligned to its class"
        # spurious-reject bounds
        past_quota = (a_st == ST_OK) | (a_st == ST_NOMEM_POOL) | (a_st == ST_NOMEM_CLASS)
        past_pool = (a_st == ST_OK) | (a_st == ST_NOMEM_CLASS)
        tq = np.bincount(a_t, weights=np.where(past_quota, a_cs, 0), minlength=T).astype(np.int64)
        pool_past = int(np.where(past_pool, a_cs, 0).sum())
        cl_took = np.bincount(np.maximum(a_c, 0), weights=ok.astype(np.int64),
                              minlength=N_CLASSES).astype(np.int64)
        q = a_st == ST_QUOTA
        if q.any():
            lhs = charged[a_t[q]] + tq[a_t[q]] + a_cs[q]
            assert np.all(lhs > quotas[a_t[q]]), "spurious quota reject"
        pr = a_st == ST_NOMEM_POOL
        if pr.any():
            assert np.all(pool_used + pool_past + a_cs[pr] > pool), "spurious pool reject"
        cr = a_st == ST_NOMEM_CLASS
        if cr.any():
            cc = a_c[cr]
            assert np.all(live[cc] + cl_took[cc] + 1 > class_cap[cc]), "spurious class reject"
        counts["alloc_ok"] += int(ok.sum())
        counts["quota"] += int(q.sum())
        counts["nomem_pool"] += int(pr.sum())
        counts["nomem_class"] += int(cr.sum())
        counts["invalid"] += int((a_st == ST_INVALID).sum()) + int((status[fi] == ST_INVALID).sum())
        counts["free_ok"] += int(got_ok.sum())
        # --- apply the phase --------------------------------------------------
        fr = rr[expect_ok]
        held[fr] = False
        np.subtract.at(charged, tenant[fr], cs_all[fr])
        pool_used -= int(cs_all[fr].sum())
        np.subtract.at(live, cls[fr], 1)
        aok = ai[ok]
        held[aok] = True
        np.add.at(charged, tenant[aok], cs_all[aok])
        pool_used += int(cs_all[aok].sum())
        np.add.at(live, cls[aok], 1)
        # --- state invariants at the phase boundary --------------------------
        assert np.all(charged <= quotas), "tenant over quota"
        assert pool_used <= pool, "pool exceeded"
        assert np.all(live <= class_cap), "class over capacity"
        h = np.nonzero(held)[0]
        order = np.argsort(ptr[h], kind="stable")
        ps = ptr[h][order]
        ce = ps + cs_all[h][order]
        assert np.all(ce[:-1] <= ps[1:]), "overlapping live blocks"
    if final_charged is not None:
        assert np.array_equal(np.asarray(final_charged, dtype=np.int64), charged), \
            "device tenant counters disagree with the log"
    if final_pool is not None:
        assert int(final_pool) == pool_used, "device pool counter disagrees with the log"
    counts["charged"] = charged
    counts["pool_used"] = pool_used
    counts["live"] = live
    return counts
