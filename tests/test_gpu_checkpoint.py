"""Checkpoint / integrity check / recovery (Sec. III-B, first and second
robustness features): the library's record against the oracle's, byte for
byte, and recovered contexts against recovered oracle schedulers."""
import ctypes as C
import os
import struct

import numpy as np
import pytest
import torch

from oracle import checkpoint as CK
from oracle import sched as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_04495_amd import cosched
    cosched.lib()
    return cosched


def _dead_pid():
    """A process id no process can have: above the kernel's pid_max."""
    try:
        with open("/proc/sys/kernel/pid_max") as f:
            return int(f.read()) + 1
    except OSError:
        return (1 << 22) + 1


def _step(cs, ctxs, refs, rng, pend_cap):
    """One random life-cycle call applied to every context and every oracle
    scheduler; all must answer alike.  Withdrawal is the timeout of a wait."""
    ref = refs[0]
    j = int(rng.integers(len(ref.jobs)))
    u = rng.random()
    if u < 0.5 and len(ref.pending()) < pend_cap:
        b = int(rng.integers(1, 4000))
        exp = [r.admit(j, 0, b) for r in refs]
        got = [cs.sched_admit(c, j, 0, b, cs.SCHED_NONBLOCK) for c in ctxs]
    elif u < 0.6:
        waiting = any(p.job == j for p in ref.pending())
        exp = [cs.SCHED_TIMEOUT if waiting else cs.SCHED_OK] * len(refs)
        for r in refs:
            r.withdraw(j)
        got = [cs.sched_wait(c, j, 1) for c in ctxs]
    else:
        res = ref.jobs[j]["res"]
        b = 0 if rng.random() < 0.5 else int(rng.integers(0, res + 2))
        exp = [r.release(j, -1, b) for r in refs]
        got = [cs.sched_release(c, j, -1, b) for c in ctxs]
    assert len(set(exp)) == 1 and got == exp, (j, u, got, exp)


def _check_res(cs, ctx, ref):
    for j in ref.jobs:
        assert cs.sched_reservation(ctx, j) == (0, ref.jobs[j]["res"]), j
    rc, st = cs.sched_stats(ctx)
    assert rc == 0 and st["used"] == ref.used


@pytest.mark.parametrize("policy", [0, 1, 2, 3])
def test_checkpoint_equals_oracle_then_restore_continues(cs, policy):
    """Random life cycle on a small ring (the live range wraps around it);
    every 20 calls the record equals the oracle's byte for byte.  The last
    record is restored into a fresh context, after which the original, the
    restored context and the restored oracle answer every call alike."""
    C_ = 10_000
    me = os.getpid()
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=C_, max_jobs=32, queue_capacity=64)
    assert rc == 0
    ctx2 = None
    ref = S.Scheduler(C_, policy)
    rng = np.random.default_rng(500 + policy)
    try:
        for k in range(12):
            pr = int(rng.integers(0, 3)) if policy >= 2 else 0
            assert cs.sched_register(ctx, pr, 100 + k)[0] == 0
            ref.register(pr, 100 + k)
            if k % 4 == 1:
                assert cs.sched_set_owner(ctx, k, me) == 0 and ref.set_owner(k, me) == S.OK
        for step in range(240):
            _step(cs, [ctx], [ref], rng, pend_cap=40)
            if step % 20 == 19:
                rc, rec = cs.sched_checkpoint(ctx)
                assert rc == 0 and rec == CK.encode(ref), step
                rc, bound = cs.sched_checkpoint_size(ctx)
                assert rc == 0 and bound >= len(rec)
        _check_res(cs, ctx, ref)
        assert len(ref.pending()) > 0
        rc, rec = cs.sched_checkpoint(ctx)
        assert rc == 0 and rec == CK.encode(ref)
        rc, ctx2 = cs.sched_create(policy=policy, capacity_bytes=C_, max_jobs=32,
                                   queue_capacity=64)
        assert rc == 0
        assert cs.sched_restore(ctx2, rec) == 0
        ref2 = CK.restore(rec, policy, C_, 32)
        assert ref2 is not None
        rc, rec2 = cs.sched_checkpoint(ctx2)
        assert rc == 0 and rec2 == rec
        _check_res(cs, ctx2, ref2)
        for step in range(160):
            _step(cs, [ctx, ctx2], [ref, ref2], rng, pend_cap=40)
        _check_res(cs, ctx, ref)
        _check_res(cs, ctx2, ref2)
        assert cs.sched_checkpoint(ctx)[1] == cs.sched_checkpoint(ctx2)[1] == CK.encode(ref2)
    finally:
        cs.sched_destroy(ctx)
        if ctx2 is not None:
            cs.sched_destroy(ctx2)


def _small_record(cs, ctx, ref):
    a = cs.sched_register(ctx, 0, 50)[1]
    b = cs.sched_register(ctx, 0, 50)[1]
    ref.register(0, 50)
    ref.register(0, 50)
    assert cs.sched_admit(ctx, a, 0, 600, cs.SCHED_NONBLOCK) == ref.admit(a, 0, 600) == 0
    assert cs.sched_admit(ctx, b, 0, 700, cs.SCHED_NONBLOCK) == ref.admit(b, 0, 700) == 1
    assert cs.sched_admit(ctx, a, 0, 500, cs.SCHED_NONBLOCK) == ref.admit(a, 0, 500) == 1
    rc, rec = cs.sched_checkpoint(ctx)
    assert rc == 0 and rec == CK.encode(ref)
    return rec


def _reseal(rec):
    return rec[:48] + struct.pack("<Q", CK.checksum(rec)) + rec[56:]


def test_restore_rejects_corruption_and_keeps_the_fresh_state(cs):
    """Every single-byte change of the record, and records whose accounting
    is inconsistent under a valid checksum, are refused with the target left
    fresh; the intact record then restores."""
    rc, ctx = cs.sched_create(policy=1, capacity_bytes=1000, max_jobs=8, queue_capacity=64)
    assert rc == 0
    rc, ctx2 = cs.sched_create(policy=1, capacity_bytes=1000, max_jobs=8, queue_capacity=64)
    assert rc == 0
    try:
        ref = S.Scheduler(1000, S.MMU)
        rec = _small_record(cs, ctx, ref)
        assert len(rec) == 64 + 2 * 24 + 2 * 16
        for i in range(len(rec)):
            for x in (0x01, 0x80):
                bad = bytearray(rec)
                bad[i] ^= x
                assert CK.decode(bytes(bad), 8) is None
                assert cs.sched_restore(ctx2, bytes(bad)) == cs.SCHED_E_INVALID, (i, x)
        J0, R0 = 64, 64 + 48
        sealed = {
            "used != sum": bytearray(rec), "request job": bytearray(rec),
            "request prio": bytearray(rec), "demand": bytearray(rec),
        }
        struct.pack_into("<q", sealed["used != sum"], 24, 500)
        struct.pack_into("<i", sealed["request job"], R0 + 8, 2)
        struct.pack_into("<i", sealed["request prio"], R0 + 12, 1)
        struct.pack_into("<q", sealed["demand"], R0, 0)
        for name, b in sealed.items():
            bad = _reseal(bytes(b))
            assert CK.decode(bad, 8) is None
            assert cs.sched_restore(ctx2, bad) == cs.SCHED_E_INVALID, name
        assert cs.sched_restore(ctx2, rec[:-1]) == cs.SCHED_E_INVALID
        assert cs.sched_restore(ctx2, b"") == cs.SCHED_E_INVALID
        # still fresh: its record is the empty scheduler's
        assert cs.sched_checkpoint(ctx2) == (0, CK.encode(S.Scheduler(1000, S.MMU)))
        assert cs.sched_restore(ctx2, rec) == 0
        ref2 = CK.restore(rec, S.MMU, 1000, 8)
        _check_res(cs, ctx2, ref2)
        # the restored requests wait like ours: once a frees 300, b's 700 is
        # served; a's own 500 waits until b frees its memory
        assert cs.sched_release(ctx2, 0, -1, 300) == ref2.release(0, -1, 300) == 0
        assert cs.sched_wait(ctx2, 1, 1000) == cs.SCHED_OK
        _check_res(cs, ctx2, ref2)
        assert ref2.jobs[0]["res"] == 300 and ref2.jobs[1]["res"] == 700
        assert cs.sched_release(ctx2, 1, -1, 0) == ref2.release(1, -1, 0) == 0
        assert cs.sched_wait(ctx2, 0, 1000) == cs.SCHED_OK
        _check_res(cs, ctx2, ref2)
        assert ref2.jobs[0]["res"] == 800 and ref2.used == 800
    finally:
        cs.sched_destroy(ctx)
        cs.sched_destroy(ctx2)


def test_restore_requires_a_fresh_matching_context(cs):
    rc, ctx = cs.sched_create(policy=1, capacity_bytes=1000, max_jobs=8, queue_capacity=64)
    assert rc == 0
    made = [ctx]
    try:
        rec = _small_record(cs, ctx, S.Scheduler(1000, S.MMU))
        for kw in (dict(policy=0, capacity_bytes=1000), dict(policy=1, capacity_bytes=999),
                   dict(policy=1, capacity_bytes=1000, max_jobs=1)):
            rc, c2 = cs.sched_create(queue_capacity=64, **kw)
            assert rc == 0
            made.append(c2)
            assert cs.sched_restore(c2, rec) == cs.SCHED_E_INVALID, kw
        rc, c3 = cs.sched_create(policy=1, capacity_bytes=1000, max_jobs=8, queue_capacity=64)
        made.append(c3)
        assert cs.sched_register(c3)[0] == 0
        assert cs.sched_restore(c3, rec) == cs.SCHED_E_INVALID          # not fresh
        assert cs.sched_restore(ctx, rec) == cs.SCHED_E_INVALID         # itself
        # a buffer smaller than the record
        buf = C.create_string_buffer(len(rec))
        n = C.c_size_t()
        assert cs.lib().sched_checkpoint(ctx, buf, len(rec) - 1, C.byref(n)) == cs.SCHED_E_INVALID
        assert cs.lib().sched_checkpoint(ctx, buf, len(rec), C.byref(n)) == 0
        assert n.value == len(rec) and buf.raw == rec
        assert cs.lib().sched_checkpoint(ctx, buf, len(rec), None) == cs.SCHED_E_INVALID
    finally:
        for c in made:
            cs.sched_destroy(c)


def test_recovered_dead_holder_is_reclaimed(cs):
    """The record keeps the owner processes: after recovery, the sanity check
    reclaims a holder whose process is gone and serves the recovered waiter,
    as the oracle does."""
    dead = _dead_pid()
    rc, ctx = cs.sched_create(policy=3, capacity_bytes=1000, max_jobs=8, queue_capacity=64)
    assert rc == 0
    rc, ctx2 = cs.sched_create(policy=3, capacity_bytes=1000, max_jobs=8, queue_capacity=64)
    assert rc == 0
    try:
        ref = S.Scheduler(1000, S.PRIO_MMU)
        a = cs.sched_register(ctx, 1, 50)[1]
        b = cs.sched_register(ctx, 0, 50)[1]
        ref.register(1, 50)
        ref.register(0, 50)
        assert cs.sched_set_owner(ctx, a, os.getpid()) == 0 and ref.set_owner(a, os.getpid()) == 0
        assert cs.sched_admit(ctx, a, 0, 800, cs.SCHED_NONBLOCK) == ref.admit(a, 0, 800) == 0
        assert cs.sched_admit(ctx, b, 0, 500, cs.SCHED_NONBLOCK) == ref.admit(b, 0, 500) == 1
        assert cs.sched_set_owner(ctx, a, dead) == 0 and ref.set_owner(a, dead) == 0
        rc, rec = cs.sched_checkpoint(ctx)
        assert rc == 0 and rec == CK.encode(ref)
        assert cs.sched_restore(ctx2, rec) == 0
        ref2 = CK.restore(rec, S.PRIO_MMU, 1000, 8)
        assert cs.sched_sanity_check(ctx2) == (0, 1, 800)
        assert ref2.sanity(lambda pid: pid != dead) == (1, 800)
        _check_res(cs, ctx2, ref2)
        assert cs.sched_wait(ctx2, b, 1000) == cs.SCHED_OK
        rc, st = cs.sched_stats(ctx2)
        assert st["used"] == 500 and st["pending"] == 0
    finally:
        cs.sched_destroy(ctx)
        cs.sched_destroy(ctx2)


def test_restore_needs_room_for_the_waiting_requests(cs):
    """A record with more waiting requests than the target's queue holds is
    refused (the target stays fresh); a large enough queue takes it."""
    rc, ctx = cs.sched_create(policy=0, capacity_bytes=1000, max_jobs=4, queue_capacity=1024)
    assert rc == 0
    made = [ctx]
    try:
        ref = S.Scheduler(1000, S.FIFO)
        a = cs.sched_register(ctx, 0, 50)[1]
        b = cs.sched_register(ctx, 0, 50)[1]
        ref.register(0, 50)
        ref.register(0, 50)
        assert cs.sched_admit(ctx, a, 0, 1000, cs.SCHED_NONBLOCK) == ref.admit(a, 0, 1000) == 0
        for _ in range(300):
            assert cs.sched_admit(ctx, b, 0, 1, cs.SCHED_NONBLOCK) == ref.admit(b, 0, 1) == 1
        rc, rec = cs.sched_checkpoint(ctx)
        assert rc == 0 and rec == CK.encode(ref) and len(rec) == 64 + 2 * 24 + 300 * 16
        rc, small = cs.sched_create(policy=0, capacity_bytes=1000, max_jobs=4, queue_capacity=256)
        assert rc == 0
        made.append(small)
        assert cs.sched_restore(small, rec) == cs.SCHED_E_INVALID
        assert cs.sched_checkpoint(small) == (0, CK.encode(S.Scheduler(1000, S.FIFO)))
        rc, big = cs.sched_create(policy=0, capacity_bytes=1000, max_jobs=4, queue_capacity=512)
        assert rc == 0
        made.append(big)
        assert cs.sched_restore(big, rec) == 0
        assert cs.sched_checkpoint(big) == (0, rec)
        # the restored waiters are served once a frees its memory (FIFO, in order)
        ref2 = CK.restore(rec, S.FIFO, 1000, 4)
        assert cs.sched_release(big, a, -1, 0) == ref2.release(a, -1, 0) == 0
        assert cs.sched_reservation(big, b) == (0, ref2.jobs[b]["res"]) and ref2.jobs[b]["res"] == 300
    finally:
        for c in made:
            cs.sched_destroy(c)
