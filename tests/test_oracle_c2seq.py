"""The compiled sequential oracle of the release/admit rounds (oracle/c2seq.c)
against the pinned numpy statement of the same rounds and against first
principles: every pass's result is the first-fit fixed point (MMU) or the
longest fitting prefix (FIFO) of the waiting requests, and the accounting
closes (Sec. III-B, Sec. IV, Sec. V Policies 1 and 2)."""
import numpy as np
import pytest

from oracle import c2seq
from oracle import sched as S
from workloads import c2_queue, random_queue


def _same(a, b):
    assert len(a) == len(b)
    for (ids, R, rel), rr in zip(a, b):
        assert np.array_equal(ids, rr.admitted)
        assert R == rr.R_after
        assert rel == rr.released.size


@pytest.mark.parametrize("policy", [S.FIFO, S.MMU])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_c2seq_equals_numpy_rounds(policy, seed):
    q = c2_queue(seed=seed, n=1 << 14, capacity=280 * 10**9 // 64)
    a = c2seq.release_rounds(q.demand, q.capacity, q.coins, q.rounds, policy)
    b = S.release_rounds(q.demand, q.capacity, q.coins, q.rounds, policy)
    _same(a, b)


def test_c2seq_full_c2_step():
    q = c2_queue(seed=2)
    a = c2seq.release_rounds(q.demand, q.capacity, q.coins, q.rounds, S.MMU)
    b = S.release_rounds(q.demand, q.capacity, q.coins, q.rounds, S.MMU)
    _same(a, b)


@pytest.mark.parametrize("policy", [S.FIFO, S.MMU])
def test_c2seq_passes_are_fixed_points(policy):
    """Each pass, rebuilt from the waiting list it saw, is the policy's own
    characterisation; holes (withdrawn requests) neither admit nor block."""
    rng = np.random.default_rng(11)
    for case in range(40):
        n = int(rng.integers(0, 60))
        d = random_queue(case, n, 1 << 12, holes=0.2)
        R = int(rng.integers(0, 1 << 14))
        coins = rng.integers(0, 2, (3, n)).astype(np.uint8)
        res = c2seq.release_rounds(d, R, coins, 4, policy)
        pend = np.arange(n)
        running = np.zeros(n, bool)
        used = 0
        for r, (ids, Ra, rel) in enumerate(res):
            if r > 0:
                m = running & (coins[r - 1] != 0)
                assert rel == int(m.sum())
                used -= int(d[m].sum())
                running[m] = False
            Rb = R - used
            adm = np.isin(pend, ids)
            if policy == S.MMU:
                assert S.first_fit_fixed_point(d[pend], Rb, adm)
            else:
                assert S.fifo_prefix_check(d[pend], Rb, adm)
            assert Ra == Rb - int(d[ids].sum())
            running[ids] = True
            used = R - Ra
            pend = pend[~adm]


def test_c2seq_edge_cases():
    r = c2seq.release_rounds(np.zeros(0, np.int64), 10, np.zeros((0, 0), np.uint8), 1)
    assert r[0][0].size == 0 and r[0][1] == 10
    # R = 0: nothing admitted under either policy
    for pol in (S.FIFO, S.MMU):
        r = c2seq.release_rounds(np.array([1, 2, 3]), 0, np.zeros((0, 3), np.uint8), 1, pol)
        assert r[0][0].size == 0 and r[0][1] == 0
    # FIFO stops at the first misfit, MMU backfills past it
    d = np.array([4, 10, 3, 2])
    assert c2seq.release_rounds(d, 9, np.zeros((0, 4), np.uint8), 1, S.FIFO)[0][0].tolist() == [0]
    assert c2seq.release_rounds(d, 9, np.zeros((0, 4), np.uint8), 1, S.MMU)[0][0].tolist() == [0, 2, 3]
