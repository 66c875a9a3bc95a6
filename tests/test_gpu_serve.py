"""Serving loop: virtual-clock schedules equal the oracle's replay; real-time
runs are memory-safe; each job's result is the same alone, in the mix and in
a batched launch."""
import numpy as np
import pytest
import torch

from oracle import sched as S
from oracle import schedule as V
from oracle import tenants as T
from workloads import (GiB, MiB, JobMix, KIND_GEMM, KIND_HIST, KIND_TRIAD, c1_jobs, c4_jobs,
                       c5_jobs, gemm_demand, hist_demand, job_table, triad_demand)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_04495_amd import cosched
    cosched.lib()
    return cosched


def _ctx(cs, policy, capacity, n):
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=capacity, max_jobs=max(n, 1),
                              queue_capacity=max(n, 4096), window_limit=16)
    assert rc == 0
    return ctx


def _virtual(cs, mix, policy, prio=None):
    jt = job_table(mix)
    if prio is not None:
        jt["priority"] = prio
    ctx = _ctx(cs, policy, mix.capacity, mix.n)
    try:
        rc, res, sm = cs.sched_serve(ctx, jt, mode=cs.SCHED_SERVE_VIRTUAL)
        assert rc == 0
    finally:
        cs.sched_destroy(ctx)
    ref = V.simulate(jt["arrival_s"], jt["demand"], jt["vdur_s"], mix.capacity, policy,
                     prio=jt["priority"])
    return res, sm, ref


@pytest.mark.parametrize("policy", [0, 1])
def test_virtual_c1_equals_oracle(cs, policy):
    res, sm, ref = _virtual(cs, c1_jobs(1), policy)
    assert np.array_equal(res["t_admit"], ref["t_admit"])
    assert np.array_equal(res["t_end"], ref["t_end"])
    assert sm["completed"] == 16 and sm["violations"] == 0


@pytest.mark.parametrize("policy", [0, 1])
def test_virtual_c4_prefix_equals_oracle(cs, policy):
    mix = c4_jobs(4, n=1500)
    mix.capacity = 64 * GiB          # contended: the queue builds up
    res, sm, ref = _virtual(cs, mix, policy)
    ok = ~np.isnan(ref["t_admit"])
    assert np.array_equal(np.isnan(res["t_admit"]) | (res["status"] != 0), ~ok)
    assert np.array_equal(res["t_admit"][ok], ref["t_admit"][ok])
    assert np.array_equal(res["t_end"][ok], ref["t_end"][ok])
    print(f"  passes={sm['passes']} p99 wait={sm['p99_wait_s']:.3f}", flush=True)


@pytest.mark.parametrize("policy", [2, 3])
def test_virtual_priority_equals_oracle(cs, policy):
    """Policies 3/4: (priority, arrival) order; a third of the jobs get a
    higher priority (value 0), the rest value 1 or 2."""
    mix = c4_jobs(6, n=800)
    mix.capacity = 48 * GiB
    prio = np.random.default_rng(9).integers(0, 3, mix.n).astype(np.int32)
    res, sm, ref = _virtual(cs, mix, policy, prio)
    ok = ~np.isnan(ref["t_admit"])
    assert np.array_equal(res["t_admit"][ok], ref["t_admit"][ok])
    assert np.array_equal(res["t_end"][ok], ref["t_end"][ok])


@pytest.mark.parametrize("policy", [0, 1])
def test_virtual_hol_equals_oracle(cs, policy):
    """The head-of-line study (a 16 GiB request that cannot fit beside a
    20 GiB job, then 200 small jobs): the device loop's schedule equals the
    oracle's entry by entry under FIFO and MMU."""
    from workloads import hol_jobs
    mix = hol_jobs()
    res, sm, ref = _virtual(cs, mix, policy)
    assert np.array_equal(res["t_admit"], ref["t_admit"])
    assert np.array_equal(res["t_end"], ref["t_end"])
    assert sm["completed"] == mix.n and sm["violations"] == 0


def test_virtual_c5_prefix_equals_oracle(cs):
    mix = c5_jobs(5, n=3000, capacity=200 * GiB)
    res, sm, ref = _virtual(cs, mix, 1)
    ok = ~np.isnan(ref["t_admit"])
    assert np.array_equal(res["t_admit"][ok], ref["t_admit"][ok])


def _small_mix(seed, n_tri=12, n_gemm=4, n_hist=4):
    rng = np.random.default_rng(seed)
    kinds, sizes = [], []
    for _ in range(n_tri):
        kinds.append(KIND_TRIAD)
        sizes.append(int(rng.integers(1 << 16, 1 << 22)))
    for _ in range(n_gemm):
        kinds.append(KIND_GEMM)
        sizes.append(int(rng.choice([256, 512, 1024])))
    for _ in range(n_hist):
        kinds.append(KIND_HIST)
        sizes.append(int(rng.integers(1 << 16, 1 << 22)))
    order = rng.permutation(len(kinds))
    kind = np.array(kinds, np.int32)[order]
    size = np.array(sizes, np.int64)[order]
    demand = np.where(kind == KIND_TRIAD, triad_demand(size),
                      np.where(kind == KIND_GEMM, gemm_demand(size), hist_demand(size)))
    arr = np.cumsum(rng.exponential(2e-4, kind.size))
    return JobMix(seed, arr, kind, size, demand.astype(np.int64), 256 * MiB, "small")


def _digest_ref(kind, size, seed):
    if kind == KIND_TRIAD:
        a = T.triad_ref(seed, np.arange(size)).astype(np.float32)
        return int(a.view(np.uint32).astype(np.uint64).sum()) & (2**64 - 1)
    if kind == KIND_HIST:
        return int(T.hist_ref(seed, size).sum()) & (2**64 - 1)
    return None


@pytest.mark.parametrize("policy", [0, 1])
def test_realtime_alone_vs_mix(cs, policy):
    mix = _small_mix(7)
    jt = job_table(mix)
    ctx = _ctx(cs, policy, mix.capacity, mix.n)
    try:
        rc, mixed, sm = cs.sched_serve(ctx, jt, n_streams=4, digest=1)
        assert rc == 0 and sm["violations"] == 0 and sm["completed"] == mix.n
        rc, alone, sm2 = cs.sched_serve(ctx, jt, serial=1, digest=1)
        assert rc == 0 and sm2["completed"] == mix.n
    finally:
        cs.sched_destroy(ctx)
    assert np.array_equal(mixed["digest"], alone["digest"])
    assert sm2["max_running"] == 1
    assert np.all(mixed["t_admit"] >= mixed["t_arrive"]) and np.all(mixed["t_end"] >= mixed["t_start"])
    for i in range(mix.n):
        ref = _digest_ref(mix.kind[i], int(mix.size[i]), int(jt["seed"][i]))
        if ref is not None:
            assert int(mixed["digest"][i]) == ref, i


def test_realtime_c1_fifo(cs):
    mix = c1_jobs(1)
    jt = job_table(mix)
    ctx = _ctx(cs, 0, mix.capacity, mix.n)
    try:
        rc, res, sm = cs.sched_serve(ctx, jt, n_streams=8)
        assert rc == 0
    finally:
        cs.sched_destroy(ctx)
    assert sm["completed"] == 16 and sm["violations"] == 0
    # FIFO: admission order is arrival order
    assert np.all(np.diff(res["t_admit"]) >= 0)
    assert sm["peak_used"] <= mix.capacity


def test_batched_equals_unbatched(cs, tmp_path):
    mix = c5_jobs(5, n=600, capacity=8 * GiB)
    small = mix.demand < 16 * MiB
    jt = job_table(mix)
    ctx = _ctx(cs, 1, mix.capacity, mix.n)
    try:
        rc, per_job, sm1 = cs.sched_serve(ctx, jt, n_streams=8, digest=1)
        assert rc == 0 and sm1["violations"] == 0
        rc, batched, sm2 = cs.sched_serve(ctx, jt, n_streams=8, digest=1, batch_small=1,
                                          use_graph=1, tune_cache=str(tmp_path / "tune.json"))
        assert rc == 0 and sm2["violations"] == 0
        assert sm2["completed"] + sm2["rejected"] == mix.n
        assert sm2["rejected"] == int((mix.demand > mix.capacity).sum())
    finally:
        cs.sched_destroy(ctx)
    print(f"  batches={sm2['batches']} batched_jobs={sm2['batched_jobs']} "
          f"tuned block={sm2['tuned_block']} chunk={sm2['tuned_chunk']}", flush=True)
    assert sm2["batches"] >= 2 and sm2["batched_jobs"] == int(small.sum())
    assert np.array_equal(batched["batched"].astype(bool), small)
    ok = batched["status"] == 0
    assert np.array_equal(per_job["status"], batched["status"])
    assert np.array_equal(per_job["digest"][ok], batched["digest"][ok])
    for i in np.nonzero(small)[0][:5]:
        assert int(batched["digest"][i]) == _digest_ref(KIND_TRIAD, int(mix.size[i]), int(jt["seed"][i]))
