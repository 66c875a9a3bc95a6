"""Pins of the checkpoint / integrity-check / recovery oracle (Sec. III-B,
first and second robustness features; Sec. IV initialisation)."""
import struct

import numpy as np
import pytest

from oracle import checkpoint as CK
from oracle import sched as S


# Published FNV-1a 64 test vectors (Fowler-Noll-Vo reference test suite).
@pytest.mark.parametrize("data,expect", [
    (b"", 0xCBF29CE484222325),
    (b"a", 0xAF63DC4C8601EC8C),
    (b"foobar", 0x85944171F73967E8),
])
def test_fnv1a64_published_vectors(data, expect):
    assert CK.fnv1a64(data) == expect


def test_record_layout_sizes_and_offsets():
    """Header 64 bytes with the checksum at byte 48; 24 bytes per job; 16 per
    request; all little-endian."""
    assert (CK.HEADER.size, CK.JOB.size, CK.REQ.size) == (64, 24, 16)
    s = S.Scheduler(1000, S.MMU)
    rec = CK.encode(s)
    assert len(rec) == 64 and rec[:8] == b"SCHEDCK1"
    assert struct.unpack_from("<I", rec, 8)[0] == 1
    assert struct.unpack_from("<q", rec, 16)[0] == 1000
    assert struct.unpack_from("<Q", rec, 48)[0] == CK.checksum(rec)
    # the checksum covers the record with its own field zero
    z = rec[:48] + bytes(8) + rec[56:]
    assert CK.fnv1a64(z) == struct.unpack_from("<Q", rec, 48)[0]


def _random_life(policy, seed, steps=200, C=10_000, n_jobs=12):
    """A scheduler after a random sequence of pre-allocations, post-frees and
    withdrawals; returns it and the generator for continuing."""
    rng = np.random.default_rng(seed)
    s = S.Scheduler(C, policy)
    for k in range(n_jobs):
        s.register(int(rng.integers(0, 3)) if policy >= 2 else 0, 100 + k)
        if k % 3 == 0:
            s.set_owner(k, 1000 + k)
    for _ in range(steps):
        _step(s, rng)
    return s, rng


def _step(s, rng):
    j = int(rng.integers(len(s.jobs)))
    u = rng.random()
    if u < 0.5:
        return ("admit", j, s.admit(j, 0, int(rng.integers(1, 4000))))
    if u < 0.6:
        return ("withdraw", j, s.withdraw(j))
    res = s.jobs[j]["res"]
    b = 0 if rng.random() < 0.5 else int(rng.integers(0, res + 1))
    return ("release", j, s.release(j, -1, b))


@pytest.mark.parametrize("policy", [S.FIFO, S.MMU, S.PRIO_FIFO, S.PRIO_MMU])
def test_restore_is_equivalent_state(policy):
    """A recovered scheduler is the same scheduler: its record equals the
    original's, and the same later calls give the same results, passes and
    reservations on both (the record carries everything admission depends
    on)."""
    s, rng = _random_life(policy, seed=40 + policy)
    assert len(s.pending()) > 0           # the record holds waiting requests
    rec = CK.encode(s)
    t = CK.restore(rec, policy, s.capacity, max_jobs=64)
    assert t is not None and CK.encode(t) == rec
    seed = int(rng.integers(1 << 30))
    ra, rb = np.random.default_rng(seed), np.random.default_rng(seed)
    for _ in range(200):
        assert _step(s, ra) == _step(t, rb)
        assert [j["res"] for j in s.jobs.values()] == [j["res"] for j in t.jobs.values()]
        assert s.used == t.used
        assert [p.demand for p in CK.waiting_in_service_order(s)] == \
            [p.demand for p in CK.waiting_in_service_order(t)]
    assert CK.encode(s) == CK.encode(t)


def test_priority_record_order_and_withdrawn_left_out():
    s = S.Scheduler(100, S.PRIO_FIFO)
    a, b, c = s.register(2), s.register(0), s.register(1)
    assert s.admit(a, 0, 90) == S.OK
    assert s.admit(a, 0, 50) == S.NOT_READY
    assert s.admit(c, 0, 40) == S.NOT_READY
    assert s.admit(b, 0, 30) == S.NOT_READY
    assert s.admit(c, 0, 20) == S.NOT_READY
    s.withdraw(a)
    got = CK.decode(CK.encode(s), 8)
    assert got is not None
    head, jobs, reqs = got
    # (priority, arrival): b's 30, then c's 40 and 20; a's 50 was withdrawn
    assert reqs == [(30, b, 0), (40, c, 1), (20, c, 1)]
    assert head["used"] == 90 and [j[4] for j in jobs] == [90, 0, 0]


def test_every_single_byte_corruption_is_detected():
    """FNV-1a maps its state through a bijection for each fixed byte (xor,
    then multiplication by an odd prime mod 2^64), so a record that differs in
    one byte always has a different hash; a changed checksum field no longer
    matches the recomputed one.  Hence every single-byte change fails the
    integrity check."""
    s, _ = _random_life(S.MMU, seed=7, steps=60, n_jobs=5)
    rec = CK.encode(s)
    assert CK.decode(rec, 64) is not None
    for i in range(len(rec)):
        for x in (0x01, 0x80, 0xFF):
            bad = bytearray(rec)
            bad[i] ^= x
            assert CK.decode(bytes(bad), 64) is None, (i, x)


def _reseal(rec: bytes) -> bytes:
    return rec[:48] + struct.pack("<Q", CK.checksum(rec)) + rec[56:]


def _patch(rec, off, fmt, value):
    b = bytearray(rec)
    struct.pack_into(fmt, b, off, value)
    return _reseal(bytes(b))


def test_inconsistent_accounting_rejected_even_with_valid_checksum():
    s = S.Scheduler(1000, S.MMU)
    a, b = s.register(), s.register()
    assert s.admit(a, 0, 600) == S.OK
    assert s.admit(b, 0, 700) == S.NOT_READY
    rec = CK.encode(s)
    assert CK.decode(rec, 8) is not None
    J0, R0 = 64, 64 + 2 * 24
    cases = {
        "used != sum": _patch(rec, 24, "<q", 500),
        "used > capacity": _patch(_patch(rec, 24, "<q", 1200), J0 + 16, "<q", 1200),
        "negative reservation": _patch(rec, J0 + 24 + 16, "<q", -1),
        "negative owner": _patch(rec, J0 + 8, "<i", -5),
        "nonzero job pad": _patch(rec, J0 + 12, "<i", 1),
        "request job out of range": _patch(rec, R0 + 8, "<i", 2),
        "request demand 0": _patch(rec, R0, "<q", 0),
        "request demand > capacity": _patch(rec, R0, "<q", 1001),
        "request priority differs": _patch(rec, R0 + 12, "<i", 3),
        "wrong version": _patch(rec, 8, "<I", 2),
        "count too large": _patch(rec, 40, "<q", 2),
    }
    for name, bad in cases.items():
        assert CK.decode(bad, 8) is None, name
    assert CK.decode(rec[:-1], 8) is None and CK.decode(rec + b"\0", 8) is None
    assert CK.decode(rec, 1) is None                      # more jobs than allowed


def test_recovery_falls_back_to_fresh_state():
    """A missing or corrupt backup, or one of another pool, gives no
    scheduler: the caller keeps the fresh one (Sec. III-B)."""
    s = S.Scheduler(1000, S.FIFO)
    s.register()
    s.admit(0, 0, 10)
    rec = CK.encode(s)
    assert CK.restore(rec, S.FIFO, 1000, 8) is not None
    assert CK.restore(rec, S.MMU, 1000, 8) is None
    assert CK.restore(rec, S.FIFO, 999, 8) is None
    assert CK.restore(b"", S.FIFO, 1000, 8) is None
    assert CK.restore(rec[:10], S.FIFO, 1000, 8) is None


def test_recovered_dead_holder_is_reclaimed_by_sanity_check():
    """The backup keeps the owner processes; after recovery the sanity check
    (third robustness feature) reclaims a holder whose process is gone, and
    the recovered waiter is served."""
    s = S.Scheduler(1000, S.MMU)
    a, b = s.register(), s.register()
    s.set_owner(a, 4242)
    assert s.admit(a, 0, 800) == S.OK
    assert s.admit(b, 0, 500) == S.NOT_READY
    t = CK.restore(CK.encode(s), S.MMU, 1000, 8)
    assert t.jobs[a]["owner"] == 4242
    assert t.sanity(lambda pid: pid != 4242) == (1, 800)
    assert t.jobs[b]["res"] == 500 and t.used == 500 and not t.pending()
