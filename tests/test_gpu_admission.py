"""Admission parity: the HIP kernels vs the CPU oracle, bit-exact."""
import numpy as np
import pytest
import torch

from oracle import sched as S
from workloads import c2_queue, c2d_fifo_queue, c2d_queue, random_queue

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_04495_amd import cosched
    cosched.lib()
    return cosched


def _scan(cs, pol, d_np, R, window_limit, write_all=1, ws=False):
    """ws: run in a workspace of the caller's (always k_round) instead of the
    library's own (where FIFO scans take the split round)."""
    d = torch.from_numpy(np.ascontiguousarray(d_np, dtype=np.int64)).to(DEV)
    dec = torch.full((max(d_np.size, 1),), 7, dtype=torch.uint8, device=DEV)[: d_np.size]
    w, wb = None, 0
    if ws:
        wb = cs.sched_scan_workspace_size(d_np.size)
        w = torch.empty(wb, dtype=torch.uint8, device=DEV)
    rc, r = cs.sched_scan(pol, d, R, dec, write_all=write_all, window_limit=window_limit,
                          d_ws=w, ws_bytes=wb)
    assert rc == 0
    return dec.cpu().numpy(), r


def _check(cs, pol, d_np, R, wl, ws=False):
    dec, r = _scan(cs, pol, d_np, R, wl, ws=ws)
    ref, R2 = (S.fifo_pass if pol == cs.SCHED_POLICY_FIFO else S.mmu_pass)(d_np, R)
    print(f"  pol={pol} n={d_np.size} R={R} wl={wl} admitted={int(ref.sum())}", flush=True)
    assert set(np.unique(dec)) <= {0, 1}
    bad = np.nonzero(dec.astype(bool) != ref)[0]
    assert bad.size == 0, f"first mismatch at {bad[:5]}"
    assert r["free_after"] == R2
    assert r["admitted"] == int(ref.sum())
    assert r["admitted_bytes"] == R - R2
    last = int(np.nonzero(ref)[0][-1]) if ref.any() else -1
    assert r["last_admitted"] == last


SIZES = [0, 1, 2, 255, 4095, 4096, 4097, 3 * 4096 + 17, 50_000]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("wl", [0, 1, 16])
@pytest.mark.parametrize("pol", [0, 1])
def test_scan_random(cs, n, wl, pol):
    rng = np.random.default_rng(n * 7 + wl)
    d = random_queue(int(rng.integers(1 << 30)), n, 1000, holes=0.05)
    tot = int(d[d >= 0].sum()) if n else 0
    for R in sorted({0, 1, 999, tot // 3, max(tot - 1, 0), tot, tot + 5}):
        _check(cs, pol, d, R, wl)


def _huge_queue(seed, n):
    """Small demands with entries near 2^62 mixed in (a few per tile): the
    int64 sums of such a queue wrap unless candidates are clamped."""
    rng = np.random.default_rng(seed)
    d = random_queue(int(rng.integers(1 << 30)), n, 1000, holes=0.05)
    big = rng.random(n) < 0.01
    d[big] = (1 << 62) - rng.integers(0, 1 << 20, int(big.sum()))
    return d


@pytest.mark.parametrize("n", [5, 4097, 3 * 4096 + 17, 50_000])
@pytest.mark.parametrize("wl", [0, 1])
@pytest.mark.parametrize("pol", [0, 1])
def test_scan_huge_demands(cs, n, wl, pol):
    """Demands near 2^62 (any non-negative int64 is a valid demand): under
    FIFO no candidate is filtered, so the grid round's tile sums, its break
    scan and its look-back self-sums must not wrap.  The first case is
    [1, 2^62, 2^62, 2^62, 2^62] at R = 10: only the first entry fits."""
    if n == 5:
        d = np.array([1] + [1 << 62] * 4, np.int64)
        Rs = [10]
    else:
        d = _huge_queue(n + wl, n)
        small = d[(d >= 0) & (d < (1 << 40))]
        Rs = [10, int(small.sum()) // 2, int(small.sum()) + 5]
    for R in Rs:
        _check(cs, pol, d, R, wl)
    assert cs.sched_set_lookback_polls(0) == 0     # every look-back sums its predecessors
    try:
        for R in Rs:
            _check(cs, pol, d, R, 0)
    finally:
        assert cs.sched_set_lookback_polls(256) == 0


@pytest.mark.parametrize("wl", [0, 4])
def test_scan_adversarial_rounds(cs, wl):
    # [1, R, 1, R-1, ...]: every round admits one entry and breaks on the next
    R = 100_000
    d = np.array([x for k in range(600) for x in (1, R - k)], np.int64)
    _check(cs, cs.SCHED_POLICY_MMU, d, R, wl)


@pytest.mark.parametrize("pol", [0, 1])
def test_scan_lookback_computes_missing_sums(cs, pol):
    """With no polling at all, a look-back that meets a predecessor tile which
    has not published its sum yet computes that sum from the tile's demands
    itself.  Decisions stay equal to the oracle's (1 to 80 tiles, grid rounds
    from the start, breaks in many tiles).  Each case runs in the caller's
    workspace (k_round, whatever the policy) and in the library's (a FIFO
    scan there takes the split round)."""
    assert cs.sched_set_lookback_polls(-1) == cs.SCHED_E_INVALID
    assert cs.sched_set_lookback_polls(0) == 0
    try:
        for n in (4097, 3 * 4096 + 17, 50_000, 80 * 4096 - 3):
            rng = np.random.default_rng(n + pol)
            d = random_queue(int(rng.integers(1 << 30)), n, 1000, holes=0.05)
            tot = int(d[d >= 0].sum())
            for R in sorted({999, tot // 3, max(tot - 1, 0), tot + 5}):
                _check(cs, pol, d, R, 0, ws=True)
                _check(cs, pol, d, R, 0)
    finally:
        assert cs.sched_set_lookback_polls(256) == 0      # the library default


def test_scan_grid_rounds_beside_a_busy_device(cs):
    """Grid rounds (many breaks, so tiles look back) while a long triad on
    another stream holds compute units: some round workgroups start late, and
    look-backs that outwait the poll bound sum the missing tiles themselves.
    Decisions equal those of the same scan on an idle device and form the
    first-fit fixed point."""
    n = 1 << 21
    d = random_queue(77, n, 1000, holes=0.05)
    R = int(d[d >= 0].sum()) // 3
    ref_dec, ref_r = _scan(cs, cs.SCHED_POLICY_MMU, d, R, 0)
    assert S.first_fit_fixed_point(d, R, ref_dec.astype(bool)) and ref_r["rounds"] >= 3
    m = 1 << 27
    a = torch.empty(m, dtype=torch.float32, device=DEV)
    b, c = torch.empty_like(a), torch.empty_like(a)
    assert cs.sched_triad_fill(b, c, 3) == 0
    torch.cuda.synchronize()
    busy, scan_s = torch.cuda.Stream(), torch.cuda.Stream()
    dd = torch.from_numpy(d).to(DEV)
    dec = torch.full((n,), 7, dtype=torch.uint8, device=DEV)
    torch.cuda.synchronize()
    assert cs.sched_triad(a, b, c, 3.0, 40, stream=busy) == 0
    rc, r = cs.sched_scan(cs.SCHED_POLICY_MMU, dd, R, dec, write_all=1, window_limit=0,
                          stream=scan_s)
    assert rc == 0
    torch.cuda.synchronize()
    got = dec.cpu().numpy()
    assert np.array_equal(got, ref_dec)
    assert r["free_after"] == ref_r["free_after"] and r["rounds"] == ref_r["rounds"]


@pytest.mark.parametrize("wl", [0, 16])
def test_scan_c2_pass0(cs, wl):
    q = c2_queue(seed=2)
    for pol in (0, 1):
        _check(cs, pol, q.demand, q.capacity, wl)


@pytest.mark.parametrize("wl", [0, 1])
def test_scan_dense_fixed_point(cs, wl):
    """Dense queue (2^22): the final round reads every entry.  The result must
    be the unique first-fit fixed point, checked over every entry."""
    q = c2d_queue(seed=3, n=1 << 22)
    dec, r = _scan(cs, cs.SCHED_POLICY_MMU, q.demand, q.capacity, wl)
    a = dec.astype(bool)
    assert S.first_fit_fixed_point(q.demand, q.capacity, a)
    assert r["free_after"] == q.capacity - int(q.demand[a].sum())
    # FIFO decide-every-entry on the same queue
    dec, r = _scan(cs, cs.SCHED_POLICY_FIFO, q.demand, q.capacity, wl)
    assert S.fifo_prefix_check(q.demand, q.capacity, dec.astype(bool))


@pytest.mark.slow
@pytest.mark.parametrize("wl", [1, 64])
def test_scan_dense_full_size(cs, wl):
    """The dense first-fit pass at 2^26 entries, with the window walk the
    benchmark times (64 windows) and with a single window.  Every decision is
    checked by the first-fit fixed point, which is unique, so this equals the
    sequential result entry for entry."""
    q = c2d_queue(seed=2, n=1 << 26)
    dec, r = _scan(cs, cs.SCHED_POLICY_MMU, q.demand, q.capacity, wl)
    assert set(np.unique(dec)) <= {0, 1}
    a = dec.astype(bool)
    assert S.first_fit_fixed_point(q.demand, q.capacity, a)
    assert r["admitted"] == int(a.sum())
    assert r["free_after"] == q.capacity - int(q.demand[a].sum())


@pytest.mark.slow
def test_scan_dense_largest_size(cs):
    """The largest dense pass the benchmark sweeps, 2^28 entries (2 GiB of
    demands), with its 64-window walk, checked over every entry."""
    q = c2d_queue(seed=5, n=1 << 28)
    dec, r = _scan(cs, cs.SCHED_POLICY_MMU, q.demand, q.capacity, 64)
    a = dec.astype(bool)
    assert S.first_fit_fixed_point(q.demand, q.capacity, a)
    assert r["admitted"] == int(a.sum())
    assert r["free_after"] == q.capacity - int(q.demand[a].sum())


@pytest.mark.slow
def test_scan_fifo_whole_queue_full_size(cs):
    """FIFO over 2^26 entries whose demands sum to the capacity: the whole
    queue is the admitted prefix and no memory is left (the FIFO case of the
    dense sweep, with the window limit the benchmark passes, which a FIFO scan
    caps at two windows, so every tile of the grid round looks back)."""
    q = c2d_fifo_queue(seed=2, n=1 << 26)
    dec, r = _scan(cs, cs.SCHED_POLICY_FIFO, q.demand, q.capacity, 64)
    assert np.all(dec == 1)
    assert r["admitted"] == q.n and r["free_after"] == 0
    assert r["last_admitted"] == q.n - 1


def test_scan_rejects_bad_args(cs):
    d = torch.ones(4, dtype=torch.int64, device=DEV)
    dec = torch.zeros(4, dtype=torch.uint8, device=DEV)
    assert cs.sched_scan(7, d, 10, dec)[0] == cs.SCHED_E_INVALID
    assert cs.sched_scan(1, d, -1, dec)[0] == cs.SCHED_E_INVALID
    assert cs.sched_scan(1, d, 1 << 46, dec)[0] == cs.SCHED_E_INVALID


# --------------------------------------------------------------------------
# Context path: intake, passes, compaction, batched release (C2 rounds)
# --------------------------------------------------------------------------
def _c2_ctx_run(cs, q, policy, window_limit=0):
    n = q.n
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=q.capacity, max_jobs=n,
                              queue_capacity=n, window_limit=window_limit)
    assert rc == 0
    try:
        rc, j0 = cs.sched_register_batch(ctx, n)
        assert rc == 0 and j0 == 0
        d_job = torch.arange(n, dtype=torch.int32, device=DEV)
        d_dem = torch.from_numpy(q.demand).to(DEV)
        assert cs.sched_enqueue_batch(ctx, d_job, d_dem) == 0
        coins = torch.from_numpy(q.coins).to(DEV)
        out = torch.empty(n, dtype=torch.int32, device=DEV)
        got = []
        for r in range(q.rounds):
            if r > 0:
                assert cs.sched_release_masked(ctx, coins[r - 1]) == 0
            rc, res = cs.sched_pass(ctx)
            assert rc == 0
            rc, na = cs.sched_last_admitted(ctx, out)
            assert rc == 0 and na == res["admitted"]
            torch.cuda.synchronize()
            got.append((out[:na].cpu().numpy().astype(np.int64), res))
        rc, st = cs.sched_stats(ctx)
        return got, st
    finally:
        cs.sched_destroy(ctx)


@pytest.mark.parametrize("policy", [0, 1])
@pytest.mark.parametrize("wl", [0, 16])
def test_ctx_c2_rounds_small(cs, policy, wl):
    q = c2_queue(seed=5, n=1 << 14, capacity=2 * 10**11)
    got, st = _c2_ctx_run(cs, q, policy, wl)
    ref = S.release_rounds(q.demand, q.capacity, q.coins, q.rounds, policy)
    for r, ((adm, res), rr) in enumerate(zip(got, ref)):
        print(f"  round {r}: admitted {adm.size}", flush=True)
        assert np.array_equal(adm, rr.admitted), f"round {r}"
        assert res["free_after"] == rr.R_after
    assert st["used"] == ref[-1].used_after


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_ctx_c2_full(cs, seed):
    q = c2_queue(seed=seed)
    got, st = _c2_ctx_run(cs, q, 1, 16)
    ref = S.release_rounds(q.demand, q.capacity, q.coins, q.rounds, S.MMU)
    for r, ((adm, res), rr) in enumerate(zip(got, ref)):
        assert np.array_equal(adm, rr.admitted), f"round {r}"
        assert res["free_after"] == rr.R_after
    assert st["used"] == ref[-1].used_after <= q.capacity


@pytest.mark.parametrize("policy", [0, 1])
@pytest.mark.parametrize("seed,n", [(5, 1 << 14), (2, 1 << 20)])
def test_ctx_chain_equals_oracle(cs, policy, seed, n):
    """The device-chained release/admit rounds reproduce every round of the
    oracle: admitted ids (concatenated in round order) and free memory."""
    q = c2_queue(seed=seed, n=n, capacity=280 * 10**9 if n > 1 << 16 else 2 * 10**11)
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=q.capacity, max_jobs=n,
                              queue_capacity=n, window_limit=16)
    assert rc == 0
    try:
        assert cs.sched_register_batch(ctx, n)[0] == 0
        d_job = torch.arange(n, dtype=torch.int32, device=DEV)
        d_dem = torch.from_numpy(q.demand).to(DEV)
        coins = torch.from_numpy(q.coins).to(DEV)
        adm = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        for rep in range(2):            # the same context twice: reset must restore it
            assert cs.sched_reset(ctx) == 0
            assert cs.sched_enqueue_batch(ctx, d_job, d_dem) == 0
            rc, res = cs.sched_pass_chain(ctx, q.rounds, coins, adm)
            assert rc == 0
            torch.cuda.synchronize()
            ref = S.release_rounds(q.demand, q.capacity, q.coins, q.rounds, policy)
            got = adm.cpu().numpy().astype(np.int64)
            off = 0
            for r, (rr, pr) in enumerate(zip(ref, res)):
                k = rr.admitted.size
                assert pr["admitted"] == k, f"round {r}"
                assert np.array_equal(got[off:off + k], rr.admitted), f"round {r}"
                assert pr["free_after"] == rr.R_after
                # the round's release step (Sec. IV post-free of whole jobs)
                assert pr["released"] == rr.released.size, f"round {r}"
                assert pr["released_bytes"] == int(q.demand[rr.released].sum()), f"round {r}"
                off += k
            rc, st = cs.sched_stats(ctx)
            assert st["used"] == ref[-1].used_after
    finally:
        cs.sched_destroy(ctx)


# (jobs, requests, rounds, capacity, demand bound): "few" repeats jobs often
# (a job holds several entries of the running list); "many" admits tens of
# thousands of requests per pass; "grow" (4000 large requests, then 26000
# small ones, one per job) runs ~2500 jobs for two rounds and then up to
# ~18500, so the running list grows sevenfold within one chain
CHAIN_SHAPES = {"few": (300, 2000, 12, 10**6, 10**6 // 40),
                "many": (60_000, 60_000, 6, 2 * 10**7, 1000),
                "grow": (30_000, 30_000, 10, 10**6, 600)}


@pytest.mark.parametrize("policy", [0, 1])
@pytest.mark.parametrize("seed,shape", [(11, "few"), (12, "few"), (13, "many"), (14, "grow")])
def test_ctx_chain_repeated_jobs(cs, policy, seed, shape):
    """Chain rounds where jobs have several requests in the queue: a job can be
    released and admitted again within one chain, and several of its requests
    can be admitted by one pass.  Reference: per round, every masked job that
    holds a reservation releases all of it (Sec. IV post-free, 0 bytes), then
    one oracle pass (Sec. V) runs over the waiting requests in order."""
    rng = np.random.default_rng(seed)
    n_jobs, n_req, rounds, C, dmax = CHAIN_SHAPES[shape]
    if shape == "grow":
        job = np.arange(n_req, dtype=np.int32)
        dem = np.concatenate([rng.integers(200, dmax, 4000),
                              rng.integers(10, 60, n_req - 4000)]).astype(np.int64)
    else:
        job = rng.integers(0, n_jobs, n_req).astype(np.int32)
        dem = rng.integers(1, dmax, n_req).astype(np.int64)
    masks = (rng.random((rounds - 1, n_jobs)) < 0.4).astype(np.uint8)
    # reference
    res = np.zeros(n_jobs, np.int64)
    pend = np.arange(n_req)
    used = 0
    ref = []
    for r in range(rounds):
        rel_jobs = 0
        rel_bytes = 0
        if r > 0:
            hit = (masks[r - 1] != 0) & (res > 0)
            rel_jobs = int(hit.sum())
            rel_bytes = int(res[hit].sum())
            used -= rel_bytes
            res[hit] = 0
        R = C - used
        if policy == S.FIFO:
            adm, R2 = S.fifo_pass(dem[pend], R)
        else:
            adm, R2 = S.mmu_pass(dem[pend], R)
        got = pend[adm]
        np.add.at(res, job[got], dem[got])
        used = C - R2
        pend = pend[~adm]
        ref.append((job[got].astype(np.int64), R2, rel_jobs, rel_bytes))
    if shape == "many":
        assert ref[0][0].size > 12288 and max(x[0].size for x in ref[1:]) > 1536
    if shape == "grow":
        running = np.cumsum([x[0].size - x[2] for x in ref])
        assert running[0] < 4096 and running[1] < 4096 and running.max() > 16384, running
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=C, max_jobs=n_jobs,
                              queue_capacity=1 << int(np.ceil(np.log2(max(n_req, 4096)))))
    assert rc == 0
    try:
        assert cs.sched_register_batch(ctx, n_jobs)[0] == 0
        d_job = torch.from_numpy(job).to(DEV)
        d_dem = torch.from_numpy(dem).to(DEV)
        d_masks = torch.from_numpy(masks).to(DEV)
        adm = torch.full((n_req,), -1, dtype=torch.int32, device=DEV)
        assert cs.sched_enqueue_batch(ctx, d_job, d_dem) == 0
        rc, out = cs.sched_pass_chain(ctx, rounds, d_masks, adm)
        assert rc == 0
        torch.cuda.synchronize()
        got = adm.cpu().numpy().astype(np.int64)
        off = 0
        for r, ((jobs_r, R2, rj, rb), o) in enumerate(zip(ref, out)):
            k = jobs_r.size
            assert o["admitted"] == k, f"round {r}"
            assert np.array_equal(got[off:off + k], jobs_r), f"round {r}"
            assert o["free_after"] == R2, f"round {r}"
            assert o["released"] == rj and o["released_bytes"] == rb, f"round {r}"
            off += k
        rc, st = cs.sched_stats(ctx)
        assert st["used"] == C - ref[-1][1]
    finally:
        cs.sched_destroy(ctx)


def test_enqueue_batch_rejects_invalid(cs):
    """A batch with any invalid request (unknown job, demand < 1 or above the
    capacity) is refused as a whole and leaves the queue as it was; valid
    batches before and after it are admitted exactly as the oracle says."""
    C, n_jobs = 10_000, 16
    rng = np.random.default_rng(5)
    rc, ctx = cs.sched_create(policy=cs.SCHED_POLICY_MMU, capacity_bytes=C, max_jobs=n_jobs,
                              queue_capacity=4096)
    assert rc == 0
    try:
        assert cs.sched_register_batch(ctx, n_jobs)[0] == 0
        def batch(k):
            j = rng.integers(0, n_jobs, k).astype(np.int32)
            d = rng.integers(1, C // 20, k).astype(np.int64)
            return j, d
        j1, d1 = batch(300)
        assert cs.sched_enqueue_batch(ctx, torch.from_numpy(j1).to(DEV),
                                      torch.from_numpy(d1).to(DEV)) == 0
        for bad in ("demand0", "job", "toobig"):
            jb, db = batch(500)
            if bad == "demand0":
                db[250] = 0
            elif bad == "job":
                jb[499] = n_jobs
            else:
                db[0] = C + 1
            assert cs.sched_enqueue_batch(ctx, torch.from_numpy(jb).to(DEV),
                                          torch.from_numpy(db).to(DEV)) == cs.SCHED_E_INVALID
        j2, d2 = batch(200)
        assert cs.sched_enqueue_batch(ctx, torch.from_numpy(j2).to(DEV),
                                      torch.from_numpy(d2).to(DEV)) == 0
        rc, st = cs.sched_stats(ctx)
        assert st["pending"] == 500
        rc, res = cs.sched_pass(ctx)
        assert rc == 0
        d = np.concatenate([d1, d2])
        admit, R2 = S.mmu_pass(d, C)
        assert res["admitted"] == int(admit.sum()) and res["free_after"] == R2
        out = torch.full((600,), -1, dtype=torch.int32, device=DEV)
        rc, n = cs.sched_last_admitted(ctx, out)
        assert rc == 0 and n == int(admit.sum())
        jobs = np.concatenate([j1, j2])
        assert np.array_equal(out[:n].cpu().numpy(), jobs[admit])
    finally:
        cs.sched_destroy(ctx)


def test_scan_caller_workspace_equals_library_workspace(cs):
    """sched_scan with the caller's workspace (filled with garbage, reused by
    two calls in a row, the second smaller) decides exactly as with the
    library's own workspace and as the oracle."""
    for n, R, pol, wl in ((3 * 4096 + 17, 10**6, 1, 0), (5000, 3 * 10**5, 0, 4),
                          (70_000, 10**7, 1, 2), (257, 4000, 1, 0)):
        q = random_queue(n, n, 1000, holes=0.05)
        d = torch.from_numpy(q).to(DEV)
        ws_n = cs.sched_scan_workspace_size(70_000)
        ws = torch.full((ws_n,), 0xA5, dtype=torch.uint8, device=DEV)
        dec_a = torch.full((n,), 7, dtype=torch.uint8, device=DEV)
        dec_b = torch.full((n,), 7, dtype=torch.uint8, device=DEV)
        rc, ra = cs.sched_scan(pol, d, R, dec_a, write_all=1, window_limit=wl)
        assert rc == 0
        rc, rb = cs.sched_scan(pol, d, R, dec_b, write_all=1, window_limit=wl, d_ws=ws,
                               ws_bytes=ws_n)
        assert rc == 0
        assert ra == rb
        assert torch.equal(dec_a, dec_b)
        ref, R2 = (S.fifo_pass if pol == 0 else S.mmu_pass)(q, R)
        assert np.array_equal(dec_b.cpu().numpy().astype(bool), ref) and rb["free_after"] == R2
    # too small a workspace is refused
    d = torch.ones(10_000, dtype=torch.int64, device=DEV)
    dec = torch.zeros(10_000, dtype=torch.uint8, device=DEV)
    small = torch.zeros(256, dtype=torch.uint8, device=DEV)
    assert cs.sched_scan(1, d, 100, dec, d_ws=small, ws_bytes=256)[0] == cs.SCHED_E_INVALID


# --------------------------------------------------------------------------
# Life-cycle API vs the oracle state machine
# --------------------------------------------------------------------------
@pytest.mark.parametrize("policy", [0, 1, 2, 3])
def test_lifecycle_random_vs_oracle(cs, policy):
    C = 10_000
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=C, max_jobs=64, queue_capacity=4096)
    assert rc == 0
    ref = S.Scheduler(C, policy)
    rng = np.random.default_rng(policy + 100)
    try:
        jobs = []
        for _ in range(24):
            pr = int(rng.integers(0, 3)) if policy >= 2 else 0
            rc, j = cs.sched_register(ctx, pr, 10)
            assert rc == 0
            jobs.append(j)
            ref.register(pr, 10)
        for step in range(300):
            j = jobs[int(rng.integers(len(jobs)))]
            if rng.random() < 0.55:
                b = int(rng.integers(1, 4000))
                got = cs.sched_admit(ctx, j, 0, b, cs.SCHED_NONBLOCK)
                exp = ref.admit(j, 0, b)
                assert got == exp, f"step {step} admit"
            else:
                res = ref.jobs[j]["res"]
                b = 0 if rng.random() < 0.5 else int(rng.integers(0, res + 2))
                got = cs.sched_release(ctx, j, -1, b)
                exp = ref.release(j, -1, b)
                assert got == exp, f"step {step} release"
            for jj in jobs:
                assert cs.sched_reservation(ctx, jj) == (0, ref.jobs[jj]["res"])
        rc, st = cs.sched_stats(ctx)
        assert st["used"] == ref.used
    finally:
        cs.sched_destroy(ctx)


@pytest.mark.parametrize("policy", [2, 3])
@pytest.mark.parametrize("span", [3, 140_001])
def test_priority_order_large_queue(cs, policy, span):
    """Policies 3/4 over queues of several 4096-entry tiles with ragged tails:
    the device orders the live queue by (priority, arrival) -- one digit pass
    for three priorities, five for a span of 140 001 -- and every pass admits
    exactly what the oracle's pass over the (priority, arrival) order admits,
    in that order.  A second batch appended behind the leftovers of the first
    pass is ordered together with them."""
    rng = np.random.default_rng(span + policy)
    n_jobs = 300
    prio_of = rng.integers(-(span // 2), span - span // 2, n_jobs).astype(np.int64)
    for n1, n2 in ((1, 1), (4095, 4097), (3 * 4096 + 17, 5000)):
        d1 = rng.integers(1, 1000, n1).astype(np.int64)
        d2 = rng.integers(1, 1000, n2).astype(np.int64)
        C = max(int(d1.sum() * 2 // 5), 1000) + 1   # every demand (< 1000) fits alone
        rc, ctx = cs.sched_create(policy=policy, capacity_bytes=C, max_jobs=n_jobs,
                                  queue_capacity=1 << 15)
        assert rc == 0
        try:
            for p in prio_of:
                assert cs.sched_register(ctx, int(p), 60000)[0] == 0
            pend_job = np.zeros(0, np.int32)
            pend_dem = np.zeros(0, np.int64)
            used = 0
            for d in (d1, d2):
                j = rng.integers(0, n_jobs, d.size).astype(np.int32)
                assert cs.sched_enqueue_batch(ctx, torch.from_numpy(j).to(DEV),
                                              torch.from_numpy(d).to(DEV)) == 0
                pend_job = np.concatenate([pend_job, j])
                pend_dem = np.concatenate([pend_dem, d])
                rc, res = cs.sched_pass(ctx)
                assert rc == 0
                order = S.priority_order(prio_of[pend_job])
                a, R2 = (S.fifo_pass if policy == 2 else S.mmu_pass)(pend_dem[order], C - used)
                print(f"  policy={policy} span={span} n={pend_job.size} admitted={int(a.sum())}",
                      flush=True)
                assert res["admitted"] == int(a.sum()) and res["free_after"] == R2
                k = int(a.sum())
                out = torch.full((max(k, 1),), -1, dtype=torch.int32, device=DEV)
                rc, n = cs.sched_last_admitted(ctx, out)
                assert rc == 0 and n == k
                assert np.array_equal(out.cpu().numpy()[:k], pend_job[order][a])
                keep = np.ones(pend_job.size, bool)
                keep[order[a]] = False
                pend_job, pend_dem = pend_job[keep], pend_dem[keep]
                used = C - R2
        finally:
            cs.sched_destroy(ctx)


def test_lifecycle_errors_and_timeout(cs):
    rc, ctx = cs.sched_create(policy=1, capacity_bytes=1000, max_jobs=4, queue_capacity=64)
    assert rc == 0
    try:
        _, a = cs.sched_register(ctx, 0, 50)
        _, b = cs.sched_register(ctx, 0, 50)
        assert cs.sched_admit(ctx, a, 1, 10) == cs.SCHED_E_INVALID      # wrong device
        assert cs.sched_admit(ctx, a, 0, 0) == cs.SCHED_E_INVALID       # no bytes
        assert cs.sched_admit(ctx, 9, 0, 10) == cs.SCHED_E_INVALID      # unknown job
        assert cs.sched_admit(ctx, a, 0, 1001) == cs.SCHED_E_TOOBIG
        assert cs.sched_admit(ctx, a, 0, 800) == cs.SCHED_OK
        # blocking admit of b times out after 50 ms and is withdrawn
        assert cs.sched_admit(ctx, b, 0, 300) == cs.SCHED_TIMEOUT
        assert cs.sched_release(ctx, a, 0, 801) == cs.SCHED_E_INVALID
        assert cs.sched_release(ctx, a, -1, 0) == cs.SCHED_OK
        # the withdrawn request is never admitted later
        assert cs.sched_reservation(ctx, b) == (0, 0)
        rc, st = cs.sched_stats(ctx)
        assert st["withdrawn"] == 1 and st["used"] == 0
        # non-blocking wait path
        assert cs.sched_admit(ctx, a, 0, 900) == cs.SCHED_OK
        assert cs.sched_admit(ctx, b, 0, 200, cs.SCHED_NONBLOCK) == cs.SCHED_NOT_READY
        assert cs.sched_release(ctx, a, 0, 100) == cs.SCHED_OK           # 200 free now
        assert cs.sched_wait(ctx, b, 10) == cs.SCHED_OK
        assert cs.sched_reservation(ctx, b) == (0, 200)
    finally:
        cs.sched_destroy(ctx)


def test_ctx_reset_then_other_stream_and_host_reads(cs):
    """sched_reset only orders its kernels on the context stream: a chain run
    on another stream right after it, and host-side reads (stats, a
    reservation), must still see the reset state; the array form of the chain
    results equals the per-round dictionaries."""
    q = c2_queue(seed=5, n=1 << 14, capacity=2 * 10**11)
    n = q.demand.size
    rc, ctx = cs.sched_create(policy=1, capacity_bytes=q.capacity, max_jobs=n,
                              queue_capacity=n, window_limit=16)
    assert rc == 0
    try:
        assert cs.sched_register_batch(ctx, n)[0] == 0
        d_job = torch.arange(n, dtype=torch.int32, device=DEV)
        d_dem = torch.from_numpy(q.demand).to(DEV)
        coins = torch.from_numpy(q.coins).to(DEV)
        ref = S.release_rounds(q.demand, q.capacity, q.coins, q.rounds, S.MMU)
        # leave the context busy, then reset and read it from the host at once
        assert cs.sched_enqueue_batch(ctx, d_job, d_dem) == 0
        rc, _ = cs.sched_pass_chain(ctx, q.rounds, coins)
        assert rc == 0
        assert cs.sched_reset(ctx) == 0
        rc, st = cs.sched_stats(ctx)
        assert rc == 0 and st["used"] == 0
        rc, v = cs.sched_reservation(ctx, int(ref[0].admitted[0]))
        assert rc == 0 and v == 0
        # reset again, then intake and chain on a stream of the caller's
        assert cs.sched_reset(ctx) == 0
        side = torch.cuda.Stream()
        assert cs.sched_enqueue_batch(ctx, d_job, d_dem, stream=side) == 0
        rc, arr = cs.sched_pass_chain_array(ctx, q.rounds, coins, stream=side)
        assert rc == 0
        col = {k: i for i, k in enumerate(cs.PASS_FIELDS)}
        for r, rr in enumerate(ref):
            assert arr[r, col["admitted"]] == rr.admitted.size, f"round {r}"
            assert arr[r, col["free_after"]] == rr.R_after, f"round {r}"
            assert arr[r, col["released"]] == rr.released.size, f"round {r}"
        # and once more through the dictionary form, on the context stream
        assert cs.sched_reset(ctx) == 0
        assert cs.sched_enqueue_batch(ctx, d_job, d_dem) == 0
        rc, res = cs.sched_pass_chain(ctx, q.rounds, coins)
        assert rc == 0
        for r, pr in enumerate(res):
            assert [pr[k] for k in cs.PASS_FIELDS] == [int(v) for v in arr[r]], f"round {r}"
    finally:
        cs.sched_destroy(ctx)


def test_enqueue_batch_alignment_and_wrap(cs):
    """Batched intake at ring positions that are and are not multiples of 4,
    across the ring's end, and from an input that is not 16-B aligned: each
    pass admits the batch exactly as the oracle does."""
    C, n_jobs = 10**9, 64
    rng = np.random.default_rng(9)
    rc, ctx = cs.sched_create(policy=cs.SCHED_POLICY_MMU, capacity_bytes=C, max_jobs=n_jobs,
                              queue_capacity=1024)
    assert rc == 0
    try:
        assert cs.sched_register_batch(ctx, n_jobs)[0] == 0
        used = 0
        for k, offset in ((5, 0), (1003, 0), (3, 0), (257, 0), (1000, 0), (6, 1), (401, 1)):
            j = rng.integers(0, n_jobs, k + offset).astype(np.int32)
            d = rng.integers(1, 100, k + offset).astype(np.int64)
            dj = torch.from_numpy(j).to(DEV)[offset:]   # offset 1: a 4-B shifted view
            dd = torch.from_numpy(d).to(DEV)[offset:]
            assert cs.sched_enqueue_batch(ctx, dj, dd) == 0
            rc, res = cs.sched_pass(ctx)
            assert rc == 0
            admit, R2 = S.mmu_pass(d[offset:], C - used)
            assert admit.all() and res["admitted"] == k and res["free_after"] == R2
            used += int(d[offset:].sum())
            out = torch.full((k,), -1, dtype=torch.int32, device=DEV)
            rc, n = cs.sched_last_admitted(ctx, out)
            assert rc == 0 and n == k
            assert np.array_equal(out.cpu().numpy(), j[offset:]), (k, offset)
        rc, st = cs.sched_stats(ctx)
        assert rc == 0 and st["used"] == used and st["pending"] == 0
    finally:
        cs.sched_destroy(ctx)


# --------------------------------------------------------------------------
# Sanity check (Sec. III-B third robustness feature, Sec. IV)
# --------------------------------------------------------------------------
def _dead_pid():
    """A process id no process can have: above the kernel's pid_max."""
    try:
        with open("/proc/sys/kernel/pid_max") as f:
            return int(f.read()) + 1
    except OSError:
        return (1 << 22) + 1


def test_sanity_reclaims_dead_owner_on_admit_and_shutdown(cs):
    import os
    dead = _dead_pid()
    alive = lambda pid: pid != dead
    rc, ctx = cs.sched_create(policy=cs.SCHED_POLICY_MMU, capacity_bytes=10_000, max_jobs=8,
                              queue_capacity=256)
    assert rc == 0
    sc = S.Scheduler(capacity=10_000, policy=S.MMU)
    sc.alive = alive
    try:
        jobs = [cs.sched_register(ctx)[1] for _ in range(5)]
        for _ in range(5):
            sc.register()
        a, b, c, d, e = jobs
        assert cs.sched_set_owner(ctx, a, dead) == 0 and sc.set_owner(a, dead) == S.OK
        assert cs.sched_set_owner(ctx, b, os.getpid()) == 0 and sc.set_owner(b, os.getpid()) == S.OK
        assert cs.sched_set_owner(ctx, a, -1) == cs.SCHED_E_INVALID
        # a and b fit; c does not beside them, so the admission checks the
        # holders: a's process is gone, its 6000 bytes serve c at once
        for j, nb in ((a, 6000), (b, 3000), (c, 2000)):
            assert cs.sched_admit(ctx, j, 0, nb, cs.SCHED_NONBLOCK) == sc.admit(j, 0, nb) == 0
        for j in jobs:
            assert cs.sched_reservation(ctx, j)[1] == sc.jobs[j]["res"]
        # a second dead holder, found at another job's shutdown
        assert cs.sched_set_owner(ctx, d, os.getpid()) == 0 and sc.set_owner(d, os.getpid()) == 0
        assert cs.sched_admit(ctx, d, 0, 4000, cs.SCHED_NONBLOCK) == sc.admit(d, 0, 4000) == 0
        assert cs.sched_admit(ctx, e, 0, 5000, cs.SCHED_NONBLOCK) == sc.admit(e, 0, 5000) \
            == cs.SCHED_NOT_READY
        assert cs.sched_set_owner(ctx, d, dead) == 0 and sc.set_owner(d, dead) == 0
        assert cs.sched_release(ctx, c, 0, 0) == sc.release(c, 0, 0) == 0
        for j in jobs:
            assert cs.sched_reservation(ctx, j)[1] == sc.jobs[j]["res"], j
        rc, st = cs.sched_stats(ctx)
        assert st["used"] == sc.used == 8000 and st["pending"] == 0
        # nothing left to reclaim; an explicit check finds nothing
        assert cs.sched_sanity_check(ctx) == (0, 0, 0)
    finally:
        cs.sched_destroy(ctx)


def test_sanity_while_waiting_and_explicit(cs):
    """A blocked admission checks the holders while it waits: once the
    holder's process is gone (here: its owner becomes a pid no process has)
    the waiter is admitted; an explicit check reports what it reclaimed and
    withdraws the dead job's own waiting requests."""
    import os
    import threading
    rc, ctx = cs.sched_create(policy=cs.SCHED_POLICY_FIFO, capacity_bytes=10_000, max_jobs=8,
                              queue_capacity=256)
    assert rc == 0
    try:
        a = cs.sched_register(ctx)[1]
        b = cs.sched_register(ctx, timeout_ms=20_000)[1]
        c = cs.sched_register(ctx)[1]
        assert cs.sched_set_owner(ctx, a, os.getpid()) == 0
        assert cs.sched_admit(ctx, a, 0, 9000, cs.SCHED_NONBLOCK) == 0
        out = {}
        t = threading.Thread(target=lambda: out.update(rc=cs.sched_admit(ctx, b, 0, 5000, 0)))
        t.start()
        t.join(0.3)
        assert t.is_alive()                       # b waits: a holds 9000 and is alive
        assert cs.sched_set_owner(ctx, a, _dead_pid()) == 0
        t.join(10.0)
        assert not t.is_alive() and out["rc"] == 0
        assert cs.sched_reservation(ctx, a)[1] == 0 and cs.sched_reservation(ctx, b)[1] == 5000
        # the explicit form: c holds memory and waits for more, then dies
        assert cs.sched_set_owner(ctx, c, os.getpid()) == 0
        assert cs.sched_admit(ctx, c, 0, 4000, cs.SCHED_NONBLOCK) == 0
        assert cs.sched_admit(ctx, c, 0, 3000, cs.SCHED_NONBLOCK) == cs.SCHED_NOT_READY
        assert cs.sched_set_owner(ctx, c, _dead_pid()) == 0
        assert cs.sched_sanity_check(ctx) == (0, 1, 4000)
        rc, st = cs.sched_stats(ctx)
        assert st["used"] == 5000
        # c's waiting request was withdrawn: with the whole pool free it is
        # still never admitted
        assert cs.sched_release(ctx, b, 0, 0) == 0
        assert cs.sched_reservation(ctx, c)[1] == 0
        rc, st = cs.sched_stats(ctx)
        assert st["used"] == 0
    finally:
        cs.sched_destroy(ctx)


@pytest.mark.parametrize("policy", [0, 1])
def test_enqueue_chain_equals_separate_calls(cs, policy):
    """The fused intake + chain gives what sched_enqueue_batch followed by
    sched_pass_chain gives, round by round, and both equal the oracle's
    release/admit rounds (Sec. IV post-free, Sec. V passes)."""
    n = 1 << 14
    q = c2_queue(seed=7, n=n, capacity=2 * 10**11)
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=q.capacity, max_jobs=n,
                              queue_capacity=n, window_limit=16)
    assert rc == 0
    try:
        assert cs.sched_register_batch(ctx, n)[0] == 0
        d_job = torch.arange(n, dtype=torch.int32, device=DEV)
        d_dem = torch.from_numpy(q.demand).to(DEV)
        coins = torch.from_numpy(q.coins).to(DEV)
        adm1 = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        adm2 = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        assert cs.sched_reset(ctx) == 0
        assert cs.sched_enqueue_batch(ctx, d_job, d_dem) == 0
        rc, r1 = cs.sched_pass_chain_array(ctx, q.rounds, coins, adm1)
        assert rc == 0
        st1 = cs.sched_stats(ctx)[1]
        assert cs.sched_reset(ctx) == 0
        rc, r2 = cs.sched_enqueue_chain_array(ctx, d_job, d_dem, q.rounds, coins, adm2)
        assert rc == 0
        st2 = cs.sched_stats(ctx)[1]
        torch.cuda.synchronize()
        assert np.array_equal(r1, r2)
        assert torch.equal(adm1, adm2)
        assert st1["used"] == st2["used"] and st1["pending"] == st2["pending"]
        ref = S.release_rounds(q.demand, q.capacity, q.coins, q.rounds, policy)
        got = adm2.cpu().numpy().astype(np.int64)
        col = {k: i for i, k in enumerate(cs.PASS_FIELDS)}
        off = 0
        for r, rr in enumerate(ref):
            k = rr.admitted.size
            assert r2[r, col["admitted"]] == k and np.array_equal(got[off:off + k], rr.admitted)
            assert r2[r, col["free_after"]] == rr.R_after
            off += k
    finally:
        cs.sched_destroy(ctx)


@pytest.mark.parametrize("policy", [0, 1])
def test_chain_after_per_pass_calls_releases_their_jobs(cs, policy):
    """After a reset, a chain whose running list may start empty (nothing
    admitted yet) skips the list scan; once a per-pass call has admitted
    jobs, a later chain must find them running.  Round 0 by sched_pass, the
    release of round 1 by sched_release_masked, the remaining rounds by one
    chain: every round equals the oracle's release/admit rounds."""
    n = 1 << 14
    q = c2_queue(seed=9, n=n, capacity=2 * 10**11)
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=q.capacity, max_jobs=n,
                              queue_capacity=n, window_limit=16)
    assert rc == 0
    try:
        assert cs.sched_register_batch(ctx, n)[0] == 0
        d_job = torch.arange(n, dtype=torch.int32, device=DEV)
        d_dem = torch.from_numpy(q.demand).to(DEV)
        coins = torch.from_numpy(q.coins).to(DEV)
        adm = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        out = torch.empty(n, dtype=torch.int32, device=DEV)
        ref = S.release_rounds(q.demand, q.capacity, q.coins, q.rounds, policy)
        col = {k: i for i, k in enumerate(cs.PASS_FIELDS)}
        for rep in range(2):
            assert cs.sched_reset(ctx) == 0
            assert cs.sched_enqueue_batch(ctx, d_job, d_dem) == 0
            rc, r0 = cs.sched_pass(ctx)
            assert rc == 0 and r0["admitted"] == ref[0].admitted.size
            rc, na = cs.sched_last_admitted(ctx, out)
            assert rc == 0 and np.array_equal(out[:na].cpu().numpy(), ref[0].admitted)
            assert cs.sched_release_masked(ctx, coins[0]) == 0
            rc, rr = cs.sched_pass_chain_array(ctx, q.rounds - 1, coins[1:].contiguous(), adm)
            assert rc == 0
            torch.cuda.synchronize()
            got = adm.cpu().numpy().astype(np.int64)
            off = 0
            for r in range(1, q.rounds):
                k = ref[r].admitted.size
                assert rr[r - 1, col["admitted"]] == k, f"round {r}"
                assert np.array_equal(got[off:off + k], ref[r].admitted), f"round {r}"
                assert rr[r - 1, col["free_after"]] == ref[r].R_after
                if r > 1:
                    assert rr[r - 1, col["released"]] == ref[r].released.size, f"round {r}"
                off += k
            assert cs.sched_stats(ctx)[1]["used"] == ref[-1].used_after
    finally:
        cs.sched_destroy(ctx)


def test_enqueue_chain_refused_batch_changes_nothing(cs):
    """A fused call whose batch holds an invalid request (unknown job) is
    refused whole: SCHED_E_INVALID, nothing appended, no round run (running
    jobs keep their reservations although the masks would release them); the
    calls after it behave as if it had never been made."""
    C, n_jobs, n = 10_000, 64, 40
    rng = np.random.default_rng(3)
    rc, ctx = cs.sched_create(policy=cs.SCHED_POLICY_MMU, capacity_bytes=C, max_jobs=n_jobs,
                              queue_capacity=4096)
    assert rc == 0
    try:
        assert cs.sched_register_batch(ctx, n_jobs)[0] == 0
        job = np.arange(n, dtype=np.int32)
        dem = rng.integers(1, 800, n).astype(np.int64)
        masks = np.ones((2, n_jobs), np.uint8)
        d_masks = torch.from_numpy(masks).to(DEV)
        # a first, valid fused call: jobs 0..39 queued, round 0 admits a prefix
        rc, r0 = cs.sched_enqueue_chain_array(ctx, torch.from_numpy(job).to(DEV),
                                              torch.from_numpy(dem).to(DEV), 1)
        assert rc == 0
        st0 = cs.sched_stats(ctx)[1]
        res0 = [cs.sched_reservation(ctx, j)[1] for j in range(n_jobs)]
        adm0, R0 = S.mmu_pass(dem, C)
        assert st0["used"] == C - R0 and st0["pending"] == n - int(adm0.sum())
        # refused: job 99 does not exist
        bad = job.copy()
        bad[7] = 99
        rc, _ = cs.sched_enqueue_chain_array(ctx, torch.from_numpy(bad).to(DEV),
                                             torch.from_numpy(dem).to(DEV), 3, d_masks)
        assert rc == cs.SCHED_E_INVALID
        st1 = cs.sched_stats(ctx)[1]
        assert st1["used"] == st0["used"] and st1["pending"] == st0["pending"]
        assert [cs.sched_reservation(ctx, j)[1] for j in range(n_jobs)] == res0
        # a plain chain afterwards runs (the refused intake left nothing behind): round 1
        # releases every running job (mask 1) and admits from the waiting ones
        rc, r2 = cs.sched_pass_chain_array(ctx, 2, d_masks)
        assert rc == 0
        col = {k: i for i, k in enumerate(cs.PASS_FIELDS)}
        pend = dem[~adm0]
        a1, R1 = S.mmu_pass(pend, C - (C - R0))      # round 0 of this chain: nothing freed yet
        assert r2[0, col["admitted"]] == int(a1.sum())
        assert r2[1, col["released"]] == int(adm0.sum()) + int(a1.sum())
    finally:
        cs.sched_destroy(ctx)
