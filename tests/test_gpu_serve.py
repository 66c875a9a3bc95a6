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
    assert ok.sum() > 0
    assert np.array_equal(res["t_admit"][ok], ref["t_admit"][ok])
    assert np.array_equal(res["t_end"][ok], ref["t_end"][ok])


@pytest.mark.slow
@pytest.mark.parametrize("policy", [0, 1])
def test_virtual_c4_full_equals_oracle(cs, policy):
    """The whole serving configuration: 10 000 jobs at 200/s on 280 GB;
    every job's admission and end equal the oracle's replay."""
    mix = c4_jobs(4)
    res, sm, ref = _virtual(cs, mix, policy)
    assert sm["completed"] == mix.n and sm["violations"] == 0
    assert not np.isnan(ref["t_admit"]).any()
    assert np.array_equal(res["t_admit"], ref["t_admit"])
    assert np.array_equal(res["t_end"], ref["t_end"])
    print(f"  passes={sm['passes']} p99 wait={sm['p99_wait_s']:.3f}", flush=True)


def _mix(seed, n_tri=20, n_gemm=12, n_hist=8, capacity=256 * MiB, tiny=True):
    """A C4-shaped mix (half triads, 30 % GEMM, 20 % histograms) at sizes the
    oracle recomputes in seconds; ragged sizes, and a few tiny jobs whose
    arrays are shorter than one 4 KiB unit."""
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
    if tiny:
        kinds += [KIND_TRIAD, KIND_TRIAD, KIND_HIST, KIND_HIST]
        sizes += [1, 1001, 3, 1025]
    order = rng.permutation(len(kinds))
    kind = np.array(kinds, np.int32)[order]
    size = np.array(sizes, np.int64)[order]
    demand = np.where(kind == KIND_TRIAD, triad_demand(size),
                      np.where(kind == KIND_GEMM, gemm_demand(size), hist_demand(size)))
    arr = np.cumsum(rng.exponential(2e-4, kind.size))
    return JobMix(seed, arr, kind, size, demand.astype(np.int64), capacity, "mix")


def _digest_ref(kind, size, seed):
    """The oracle's output, digested as the serving loop digests a job's
    output (position-keyed, oracle/tenants.py)."""
    if kind == KIND_TRIAD:
        return T.position_digest(T.triad_ref(seed, np.arange(size)).astype(np.float32))
    if kind == KIND_HIST:
        return T.position_digest(T.hist_ref(seed, size).astype(np.uint32))
    return None


def _check_gemm_samples(sample, N, seed):
    """Sampled entries of C against fp64 on the exact bf16 inputs: within the
    stated 2e-2 relative tolerance and within the fp32 accumulation bound."""
    rows, cols = T.gemm_sample_positions(seed, N)
    A = T.gemm_operand(2 * seed, rows, N)
    B = T.gemm_operand(2 * seed + 1, cols, N)
    ref = (A * B).sum(axis=1)
    absdot = (np.abs(A) * np.abs(B)).sum(axis=1)
    got = np.asarray(sample, np.float64)
    assert np.all(np.abs(got - ref) <= 2e-2 * np.maximum(np.abs(ref), 1.0)), (got, ref)
    u = 2.0 ** -24
    assert np.all(np.abs(got - ref) <= N * u / (1 - N * u) * absdot), (got, ref)


def _check_memory(cs, ctx, sm, n):
    """Memory safety of a real-time run: no violation, every page and every
    charge back at the end, the free list a permutation of the pool, and the
    tenants' slab counters back to zero."""
    assert sm["violations"] == 0
    assert sm["pages_left"] == 0 and sm["charged_left"] == 0 and sm["page_check"] == 0
    assert sm["peak_pages"] <= sm["pool_pages"]
    rc, charged, _ = cs.sched_slab_counters(ctx, n)
    assert rc == 0 and not any(charged)


def _check_results(mix, jt, res):
    for i in range(mix.n):
        if res["status"][i] != 0:
            continue
        if mix.kind[i] == KIND_GEMM:
            _check_gemm_samples(res["sample"][i], int(mix.size[i]), int(jt["seed"][i]))
        else:
            ref = _digest_ref(mix.kind[i], int(mix.size[i]), int(jt["seed"][i]))
            assert int(res["digest"][i]) == ref, (i, int(mix.kind[i]), int(mix.size[i]))


@pytest.mark.parametrize("policy", [0, 1])
def test_realtime_alone_vs_mix(cs, policy):
    """Every job of a contended three-kind mix, run co-scheduled and alone
    (exclusive serial execution): triad and histogram outputs equal the
    oracle's element by element (position-keyed digests), GEMM samples match
    fp64, and each GEMM's whole output is bit-identical alone and in the
    mix."""
    mix = _mix(7)
    jt = job_table(mix)
    ctx = _ctx(cs, policy, mix.capacity, mix.n)
    try:
        rc, mixed, sm = cs.sched_serve(ctx, jt, n_streams=4, digest=1)
        assert rc == 0 and sm["completed"] == mix.n, (rc, sm["completed"])
        _check_memory(cs, ctx, sm, mix.n)
        assert sm["slot_waits"] == 0 and sm["max_running"] > 1
        rc, alone, sm2 = cs.sched_serve(ctx, jt, serial=1, digest=1)
        assert rc == 0 and sm2["completed"] == mix.n
        _check_memory(cs, ctx, sm2, mix.n)
    finally:
        cs.sched_destroy(ctx)
    assert sm2["max_running"] == 1
    assert np.array_equal(mixed["digest"], alone["digest"])
    assert np.array_equal(mixed["sample"], alone["sample"])
    assert np.all(mixed["t_place"] >= mixed["t_admit"]) and np.all(mixed["t_admit"] >= mixed["t_arrive"])
    assert np.all(mixed["t_end"] >= mixed["t_start"])
    _check_results(mix, jt, mixed)


def test_realtime_slot_waits(cs):
    """With three placement slots the admitted jobs queue for slots: every
    result is still the oracle's and the pool comes back whole."""
    mix = _mix(8, n_tri=10, n_gemm=4, n_hist=4, capacity=1 << 30)
    jt = job_table(mix)
    ctx = _ctx(cs, 1, mix.capacity, mix.n)
    try:
        rc, res, sm = cs.sched_serve(ctx, jt, n_streams=2, digest=1, max_placed=3)
        assert rc == 0 and sm["completed"] == mix.n
        _check_memory(cs, ctx, sm, mix.n)
    finally:
        cs.sched_destroy(ctx)
    assert sm["placement_slots"] == 3 and sm["slot_waits"] > 0
    assert sm["pool_pages"] == -(-mix.capacity // (64 << 10)) + 3
    _check_results(mix, jt, res)


def test_paged_gemm_equals_contiguous(cs):
    """The serving loop's GEMM (operands and result in mapped pages, loaded
    through the page table) gives the same C, bit for bit, as the contiguous
    kernel on the same inputs."""
    N, seed = 1024, 21
    mix = JobMix(0, np.zeros(1), np.array([KIND_GEMM], np.int32), np.array([N], np.int64),
                 gemm_demand(np.array([N])).astype(np.int64), 64 * MiB, "one")
    jt = job_table(mix)
    jt["seed"][0] = seed
    ctx = _ctx(cs, 1, mix.capacity, 1)
    try:
        rc, res, sm = cs.sched_serve(ctx, jt, digest=1)
        assert rc == 0 and sm["completed"] == 1 and sm["violations"] == 0
    finally:
        cs.sched_destroy(ctx)
    A = torch.empty(N * N, dtype=torch.int16, device="cuda:0")
    B = torch.empty(N * N, dtype=torch.int16, device="cuda:0")
    C = torch.empty(N * N, dtype=torch.float32, device="cuda:0")
    assert cs.sched_gemm_fill(A, N, N, 2 * seed) == 0
    assert cs.sched_gemm_fill(B, N, N, 2 * seed + 1) == 0
    assert cs.sched_gemm_bf16(A, B, C, N, N, N) == 0
    torch.cuda.synchronize()
    assert int(res["digest"][0]) == T.position_digest(C.cpu().numpy())
    _check_gemm_samples(res["sample"][0], N, seed)


def test_realtime_c1_fifo(cs):
    mix = c1_jobs(1)
    jt = job_table(mix)
    ctx = _ctx(cs, 0, mix.capacity, mix.n)
    try:
        rc, res, sm = cs.sched_serve(ctx, jt, n_streams=8)
        assert rc == 0
        _check_memory(cs, ctx, sm, mix.n)
    finally:
        cs.sched_destroy(ctx)
    assert sm["completed"] == 16 and sm["slot_waits"] == 0
    # FIFO: admission order is arrival order
    assert np.all(np.diff(res["t_admit"]) >= 0)
    assert sm["peak_used"] <= mix.capacity


def test_batched_equals_unbatched(cs, tmp_path):
    """Small triads packed into one persistent, graph-replayed launch give
    the same output as per-job launches (every job, position-keyed digests)
    and as the oracle (every 4th small job and the first large ones)."""
    mix = c5_jobs(5, n=600, capacity=8 * GiB)
    small = mix.demand < 16 * MiB
    jt = job_table(mix)
    ctx = _ctx(cs, 1, mix.capacity, mix.n)
    try:
        rc, per_job, sm1 = cs.sched_serve(ctx, jt, n_streams=8, digest=1)
        assert rc == 0
        _check_memory(cs, ctx, sm1, mix.n)
        rc, batched, sm2 = cs.sched_serve(ctx, jt, n_streams=8, digest=1, batch_small=1,
                                          use_graph=1, tune_cache=str(tmp_path / "tune.json"))
        assert rc == 0
        _check_memory(cs, ctx, sm2, mix.n)
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
    check = list(np.nonzero(small)[0][::4]) + list(np.nonzero(~small & ok)[0][:3])
    for i in check:
        assert int(batched["digest"][i]) == _digest_ref(KIND_TRIAD, int(mix.size[i]),
                                                        int(jt["seed"][i])), i


def _small_mix(seed):
    """Small jobs of all three kinds (every one under 16 MiB, with ragged and
    tiny sizes) and one larger job of each kind, arriving together."""
    rng = np.random.default_rng(seed)
    kinds = ([KIND_TRIAD] * 14 + [KIND_HIST] * 10 + [KIND_GEMM] * 9
             + [KIND_TRIAD, KIND_HIST, KIND_GEMM])
    sizes = ([int(x) for x in rng.integers(1, 1 << 20, 12)] + [1, 1001]
             + [int(x) for x in rng.integers(3, 1 << 20, 8)] + [3, 4099]
             + [256, 256, 256, 512, 512, 512, 1024, 1024, 1024]
             + [1 << 22, 1 << 23, 2048])
    order = rng.permutation(len(kinds))
    kind = np.array(kinds, np.int32)[order]
    size = np.array(sizes, np.int64)[order]
    demand = np.where(kind == KIND_TRIAD, triad_demand(size),
                      np.where(kind == KIND_GEMM, gemm_demand(size), hist_demand(size)))
    return JobMix(seed, np.zeros(kind.size), kind, size, demand.astype(np.int64), 1 * GiB, "small")


def test_batched_all_kinds_equals_unbatched(cs, tmp_path):
    """Triads, histograms and GEMMs under 16 MiB packed into the persistent
    batched launch (streaming, tile and digest phases; autotuned shapes) give
    the same output as per-job launches -- every output word, through the
    position-keyed digests, and the GEMM samples bit for bit -- and as the
    oracle: triad and histogram digests exactly, GEMM samples within the
    stated tolerance and the fp32 accumulation bound."""
    mix = _small_mix(11)
    small = mix.demand < 16 * MiB
    assert small.sum() == 33 and set(mix.kind[small]) == {KIND_TRIAD, KIND_HIST, KIND_GEMM}
    jt = job_table(mix)
    ctx = _ctx(cs, 1, mix.capacity, mix.n)
    try:
        rc, per_job, sm1 = cs.sched_serve(ctx, jt, n_streams=4, digest=1)
        assert rc == 0 and sm1["completed"] == mix.n
        _check_memory(cs, ctx, sm1, mix.n)
        rc, batched, sm2 = cs.sched_serve(ctx, jt, n_streams=4, digest=1, batch_small=1,
                                          use_graph=1, tune_cache=str(tmp_path / "tune.json"))
        assert rc == 0 and sm2["completed"] == mix.n
        _check_memory(cs, ctx, sm2, mix.n)
        # the second run reads the shapes from the cache
        rc, cached, sm3 = cs.sched_serve(ctx, jt, n_streams=4, digest=1, batch_small=1,
                                         use_graph=1, tune_cache=str(tmp_path / "tune.json"))
        assert rc == 0 and sm3["completed"] == mix.n
    finally:
        cs.sched_destroy(ctx)
    print(f"  batches={sm2['batches']} batched_jobs={sm2['batched_jobs']} "
          f"gemm tile={sm2['tuned_gemm_tile']} per_cu={sm2['tuned_gemm_per_cu']}", flush=True)
    assert sm2["tuned_from_cache"] == 0 and sm3["tuned_from_cache"] == 1
    assert sm2["tuned_gemm_tile"] in (64, 128) and sm2["tuned_gemm_per_cu"] >= 1
    assert (sm3["tuned_gemm_tile"], sm3["tuned_gemm_per_cu"]) == \
        (sm2["tuned_gemm_tile"], sm2["tuned_gemm_per_cu"])
    assert sm2["batched_jobs"] == int(small.sum())
    assert np.array_equal(batched["batched"].astype(bool), small)
    assert not per_job["batched"].any()
    for r in (batched, cached):
        assert np.array_equal(per_job["digest"], r["digest"])
        g = mix.kind == KIND_GEMM
        assert np.array_equal(per_job["sample"][g].view(np.uint32), r["sample"][g].view(np.uint32))
    _check_results(mix, jt, batched)


@pytest.mark.parametrize("block,chunk,per_cu,tile,per_cu1", [
    (256, 4096, 2, 64, 1), (1024, 16384, 1, 64, 4), (512, 8192, 4, 128, 1), (256, 16384, 8, 128, 3)])
def test_batched_shapes_equal_unbatched(cs, tmp_path, block, chunk, per_cu, tile, per_cu1):
    """Every launch shape the autotuner can choose gives the same outputs:
    the shapes are forced through the tuner's cache file, and the batched
    three-kind mix must equal the per-job launches word for word (digests)
    and the GEMM samples bit for bit."""
    import json
    mix = _small_mix(13)
    small = mix.demand < 16 * MiB
    jt = job_table(mix)
    cache = tmp_path / "shape.json"
    cache.write_text(json.dumps({"block": block, "chunk": chunk, "per_cu": per_cu,
                                 "gemm_tile": tile, "gemm_per_cu": per_cu1}))
    ctx = _ctx(cs, 1, mix.capacity, mix.n)
    try:
        rc, per_job, _ = cs.sched_serve(ctx, jt, n_streams=4, digest=1)
        assert rc == 0
        rc, batched, sm = cs.sched_serve(ctx, jt, n_streams=4, digest=1, batch_small=1,
                                         use_graph=1, tune_cache=str(cache))
        assert rc == 0 and sm["completed"] == mix.n
        _check_memory(cs, ctx, sm, mix.n)
    finally:
        cs.sched_destroy(ctx)
    assert sm["tuned_from_cache"] == 1
    assert (sm["tuned_block"], sm["tuned_chunk"], sm["tuned_per_cu"], sm["tuned_gemm_tile"],
            sm["tuned_gemm_per_cu"]) == (block, chunk, per_cu, tile, per_cu1)
    assert np.array_equal(batched["batched"].astype(bool), small)
    assert np.array_equal(per_job["digest"], batched["digest"])
    g = mix.kind == KIND_GEMM
    assert np.array_equal(per_job["sample"][g].view(np.uint32), batched["sample"][g].view(np.uint32))
    _check_results(mix, jt, batched)
