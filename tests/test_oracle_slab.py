"""Pins for the slab allocator oracle (oracle/slab.py)."""
import numpy as np
import pytest

from oracle import slab as A
from workloads import OP_ALLOC, OP_FREE, c3_ops


def test_size_class_brute_force():
    for s in list(range(1, 1100)) + [2**k + d for k in range(8, 21) for d in (-1, 0, 1)]:
        if s > 2**20:
            assert A.size_class(s) == -1
            continue
        c = next(c for c in range(13) if 256 * 2**c >= s)
        assert int(A.size_class(s)) == c
    assert int(A.size_class(0)) == -1


def _ops(lst):
    """lst of ('a', tenant, size) / ('f', tenant, ref)"""
    kind = np.array([OP_ALLOC if o[0] == "a" else OP_FREE for o in lst], np.uint8)
    ten = np.array([o[1] for o in lst], np.int32)
    size = np.array([o[2] if o[0] == "a" else 0 for o in lst], np.int64)
    ref = np.array([o[2] if o[0] == "f" else -1 for o in lst], np.int64)
    return kind, ten, size, ref


def test_simulate_hand_example():
    # tenant 0 quota 1024 B; tenant 1 quota 4096 B; pool 2048 B; class 0 holds 3 blocks
    cap = np.full(13, 100)
    cap[0] = 3
    k, t, s, r = _ops([
        ("a", 0, 512),   # 0 OK            t0 512,  pool 512
        ("a", 0, 300),   # 1 OK (512 B)    t0 1024, pool 1024
        ("a", 0, 1),     # 2 QUOTA         t0 1024 + 256 > 1024
        ("f", 0, 0),     # 3 OK            t0 512,  pool 512
        ("a", 0, 256),   # 4 OK class 0    t0 768,  pool 768,  class0 live 1
        ("a", 1, 1024),  # 5 OK            t1 1024, pool 1792
        ("a", 1, 512),   # 6 NOMEM_POOL    1792 + 512 > 2048
        ("a", 1, 200),   # 7 OK class 0    t1 1280, pool 2048, live 2
        ("f", 1, 0),     # 8 INVALID       op 0 already freed, other tenant
        ("f", 0, 2),     # 9 INVALID       op 2 failed
        ("f", 1, 7),     # 10 OK           t1 1024, pool 1792, live 1
        ("f", 1, 5),     # 11 OK           t1 0,    pool 768
        ("a", 1, 10),    # 12 OK class 0   t1 256,  pool 1024, live 2
        ("a", 0, 10),    # 13 OK class 0   t0 1024, pool 1280, live 3
        ("a", 1, 10),    # 14 NOMEM_CLASS  class 0 holds 3 blocks
        ("f", 0, 13),    # 15 OK
        ("f", 0, 13),    # 16 INVALID      double free
        ("a", 0, 2**20 + 1),  # 17 INVALID size
    ])
    st = A.simulate(k, t, s, r, [1024, 4096], 2048, cap)
    E = [A.ST_OK, A.ST_OK, A.ST_QUOTA, A.ST_OK, A.ST_OK, A.ST_OK, A.ST_NOMEM_POOL, A.ST_OK,
         A.ST_INVALID, A.ST_INVALID, A.ST_OK, A.ST_OK, A.ST_OK, A.ST_OK, A.ST_NOMEM_CLASS,
         A.ST_OK, A.ST_INVALID, A.ST_INVALID]
    assert list(st) == E


def _valid_log(ops, cap, base=1 << 40):
    """A correct log built by hand: sequential statuses, blocks placed at the
    lowest free index of per-class regions laid out back to back."""
    st = A.simulate(ops.kind, ops.tenant, ops.size, ops.ref, ops.quotas, ops.pool, cap)
    cls = A.size_class(ops.size)
    region = [0]
    for c in range(13):
        region.append(region[-1] + int(cap[c]) * (256 << c))
    free = [list(range(int(cap[c]) - 1, -1, -1)) for c in range(13)]
    ptr = np.zeros(ops.n, np.uint64)
    blk = {}
    for i in range(ops.n):
        if ops.kind[i] == OP_ALLOC and st[i] == A.ST_OK:
            c = int(cls[i])
            b = free[c].pop()
            blk[i] = (c, b)
            ptr[i] = base + region[c] + b * (256 << c)
        elif ops.kind[i] == OP_FREE and st[i] == A.ST_OK:
            c, b = blk.pop(int(ops.ref[i]))
            free[c].append(b)
    return st, ptr, base, region[-1]


@pytest.fixture(scope="module")
def small_ops():
    return c3_ops(seed=5, n_tenants=8, n_ops=1 << 13, phase_len=1 << 10, pool=1 << 30)


def test_generator_frees_name_earlier_phases(small_ops):
    o = small_ops
    fr = np.nonzero(o.kind == OP_FREE)[0]
    assert fr.size > 0.25 * o.n
    assert np.all(o.ref[fr] // o.phase_len < fr // o.phase_len)
    assert np.all(o.kind[o.ref[fr]] == OP_ALLOC)
    assert np.all(o.tenant[o.ref[fr]] == o.tenant[fr])
    assert np.unique(o.ref[fr]).size == fr.size


def test_checker_accepts_valid_log(small_ops):
    cap = np.full(13, 1 << 12)
    st, ptr, base, span = _valid_log(small_ops, cap)
    o = small_ops
    res = A.check_log(o.kind, o.tenant, o.size, o.ref, o.quotas, o.pool, cap, o.phase_len, st,
                      ptr, base, span=span)
    assert res["alloc_ok"] > 0 and res["free_ok"] > 0


@pytest.mark.parametrize("mistake", ["overlap", "misalign", "outside", "spurious_quota",
                                     "over_quota", "free_status", "spurious_class"])
def test_checker_catches_planted_mistakes(small_ops, mistake):
    o = small_ops
    cap = np.full(13, 1 << 12)
    quotas = o.quotas.copy()
    st, ptr, base, span = _valid_log(o, cap)
    st = st.astype(np.int64).copy()
    ptr = ptr.copy()
    ok_allocs = np.nonzero((o.kind == OP_ALLOC) & (st == A.ST_OK))[0]
    i, j = ok_allocs[5], ok_allocs[6]
    if mistake == "overlap":
        ptr[j] = ptr[i]
        # keep both live: make sure neither is freed afterwards
        frees = np.nonzero((o.kind == OP_FREE) & np.isin(o.ref, [i, j]))[0]
        st[frees] = A.ST_INVALID
    elif mistake == "misalign":
        ptr[i] += 128
    elif mistake == "outside":
        ptr[i] = base - 4096
    elif mistake == "spurious_quota":
        st[i] = A.ST_QUOTA
    elif mistake == "over_quota":
        quotas[o.tenant[i]] = 256
    elif mistake == "free_status":
        f = np.nonzero((o.kind == OP_FREE) & (st == A.ST_OK))[0][3]
        st[f] = A.ST_INVALID
    elif mistake == "spurious_class":
        st[i] = A.ST_NOMEM_CLASS
    with pytest.raises(AssertionError):
        A.check_log(o.kind, o.tenant, o.size, o.ref, quotas, o.pool, cap, o.phase_len, st, ptr,
                    base, span=span)


def test_checker_allows_justified_rejects():
    # tenant 0: quota 1024, two concurrent 1024 B allocs in one phase: one may win
    k, t, s, r = _ops([("a", 0, 1024), ("a", 0, 1024)])
    cap = np.full(13, 10)
    st = np.array([A.ST_QUOTA, A.ST_OK])
    ptr = np.array([0, 1 << 40], np.uint64)
    A.check_log(k, t, s, r, [1024], 1 << 20, cap, 2, st, ptr, 1 << 40)
    # both failing would be spurious
    with pytest.raises(AssertionError):
        A.check_log(k, t, s, r, [1024], 1 << 20, cap, 2, np.array([A.ST_QUOTA, A.ST_QUOTA]),
                    np.zeros(2, np.uint64), 1 << 40)


def test_checker_two_frees_of_one_block_in_a_phase():
    """Two frees naming one allocation in the same phase (plus a concurrent
    allocation of the same class that may reuse the block): exactly one free
    succeeds and the other is invalid, whichever of the two wins.  Both
    succeeding, or neither, is a mistake the checker reports."""
    # phase 0: three allocations; phase 1: two frees of op 0 and a new one
    k, t, s, r = _ops([("a", 0, 256), ("a", 1, 256), ("a", 1, 256),
                       ("f", 0, 0), ("f", 0, 0), ("a", 0, 256)])
    cap = np.full(13, 10)
    base = 1 << 40
    ptr = np.array([base, base + 256, base + 512, 0, 0, base], np.uint64)
    for st in ([A.ST_OK] * 3 + [A.ST_OK, A.ST_INVALID, A.ST_OK],
               [A.ST_OK] * 3 + [A.ST_INVALID, A.ST_OK, A.ST_OK]):
        # the new allocation took the freed block's address: no overlap,
        # since the first block is no longer held
        res = A.check_log(k, t, s, r, [1024, 1024], 1 << 20, cap, 3, np.array(st), ptr, base)
        assert res["free_ok"] == 1 and list(res["charged"]) == [256, 512]
    for st in ([A.ST_OK] * 3 + [A.ST_OK, A.ST_OK, A.ST_OK],
               [A.ST_OK] * 3 + [A.ST_INVALID, A.ST_INVALID, A.ST_OK]):
        with pytest.raises(AssertionError):
            A.check_log(k, t, s, r, [1024, 1024], 1 << 20, cap, 3, np.array(st),
                        np.array([base, base + 256, base + 512, 0, 0, base + 768], np.uint64),
                        base)
    # the sequential simulator: the second free is invalid
    st = A.simulate(k, t, s, r, [1024, 1024], 1 << 20, cap)
    assert list(st) == [A.ST_OK] * 3 + [A.ST_OK, A.ST_INVALID, A.ST_OK]
