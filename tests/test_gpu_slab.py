"""Slab sub-allocator parity: device phases vs the oracle's simulator and
invariant checker."""
import numpy as np
import pytest
import torch

from oracle import slab as A
from workloads import c3_ops, c3s_ops

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_04495_amd import cosched
    cosched.lib()
    return cosched


def design_capacity(pool_bytes):
    """The stated layout: 13 equal regions of whole MiB, class c holding
    region / (256 << c) blocks."""
    region = (pool_bytes // 13) // (1 << 20) * (1 << 20)
    return region, np.array([region >> (8 + c) for c in range(13)], np.int64)


def run_ops(cs, ops):
    T = ops.quotas.size
    rc, ctx = cs.sched_create(capacity_bytes=1 << 40, max_jobs=16, max_tenants=T,
                              slab_pool_bytes=ops.pool, queue_capacity=4096)
    assert rc == 0
    try:
        assert cs.sched_slab_set_quotas(ctx, ops.quotas) == 0
        rc, info = cs.sched_slab_info(ctx)
        region, cap = design_capacity(ops.pool)
        assert info["region_bytes"] == region and info["class_blocks"] == list(cap)
        kind = torch.from_numpy(ops.kind).to(DEV)
        ten = torch.from_numpy(ops.tenant).to(DEV)
        size = torch.from_numpy(ops.size).to(DEV)
        ref = torch.from_numpy(ops.ref).to(DEV)
        ptr = torch.zeros(ops.n, dtype=torch.int64, device=DEV)
        st = torch.full((ops.n,), -1, dtype=torch.int8, device=DEV)
        for p0 in range(0, ops.n, ops.phase_len):
            assert cs.sched_slab_ops(ctx, p0, min(p0 + ops.phase_len, ops.n), kind, ten, size, ref,
                                     ptr, st) == 0
        torch.cuda.synchronize()
        rc, charged, pool_used = cs.sched_slab_counters(ctx, T)
        assert rc == 0
        return (st.cpu().numpy(), ptr.cpu().numpy().view(np.uint64), info, cap, charged,
                pool_used)
    finally:
        cs.sched_destroy(ctx)


@pytest.mark.parametrize("n_ops", [1 << 14, 1 << 18])
def test_c3_small_matches_sequential(cs, n_ops):
    ops = c3_ops(seed=3, n_ops=n_ops, phase_len=1 << 12)
    st, ptr, info, cap, charged, pool_used = run_ops(cs, ops)
    print(f"  ops={ops.n} allocs ok={(st[ops.kind == 0] == 0).sum()}", flush=True)
    seq = A.simulate(ops.kind, ops.tenant, ops.size, ops.ref, ops.quotas, ops.pool, cap)
    # nothing binds at this load, so every status equals the sequential one
    assert np.array_equal(st.astype(np.int64), seq.astype(np.int64))
    A.check_log(ops.kind, ops.tenant, ops.size, ops.ref, ops.quotas, ops.pool, cap, ops.phase_len,
                st, ptr, info["pool_base"], final_charged=charged, final_pool=pool_used,
                span=13 * info["region_bytes"])


@pytest.mark.parametrize("seed", [3, 4])
def test_c3s_stressed_invariants(cs, seed):
    # 2^18 ops hold ~1/16 of the full run's live memory: tighten quotas and
    # pool by the same factor so that every limit binds
    ops = c3_ops(seed=seed, n_ops=1 << 18, phase_len=1 << 12, pool=64 << 20, quota_div=64 * 16)
    st, ptr, info, cap, charged, pool_used = run_ops(cs, ops)
    res = A.check_log(ops.kind, ops.tenant, ops.size, ops.ref, ops.quotas, ops.pool, cap,
                      ops.phase_len, st, ptr, info["pool_base"], final_charged=charged,
                      final_pool=pool_used, span=13 * info["region_bytes"])
    print("  ", {k: v for k, v in res.items() if isinstance(v, int)}, flush=True)
    assert res["quota"] > 0 and res["nomem_pool"] + res["nomem_class"] > 0   # limits bind


@pytest.mark.slow
def test_c3_full_size(cs):
    """C3 as configured: 2^22 ops in 64 phases of 2^16; nothing binds, so the
    statuses equal the sequential simulation exactly."""
    ops = c3_ops(seed=3)
    st, ptr, info, cap, charged, pool_used = run_ops(cs, ops)
    seq = A.simulate(ops.kind, ops.tenant, ops.size, ops.ref, ops.quotas, ops.pool, cap)
    assert np.array_equal(st.astype(np.int64), seq.astype(np.int64))
    A.check_log(ops.kind, ops.tenant, ops.size, ops.ref, ops.quotas, ops.pool, cap, ops.phase_len,
                st, ptr, info["pool_base"], final_charged=charged, final_pool=pool_used,
                span=13 * info["region_bytes"])


@pytest.mark.slow
def test_c3s_full_size(cs):
    """C3-S (quotas / 64, 1 GiB pool): every refusal must be justified by a
    bound at its phase (check_log).  Which bound a refused allocation meets
    depends on how the phase's atomics interleave: run sequentially only 5 of
    the 2^22 operations meet a quota (325 610 find their class full), so a
    concurrent run may refuse through the pool or the classes alone.  What
    holds in every interleaving is that the limits bind."""
    ops = c3s_ops(seed=3)
    st, ptr, info, cap, charged, pool_used = run_ops(cs, ops)
    res = A.check_log(ops.kind, ops.tenant, ops.size, ops.ref, ops.quotas, ops.pool, cap,
                      ops.phase_len, st, ptr, info["pool_base"], final_charged=charged,
                      final_pool=pool_used, span=13 * info["region_bytes"])
    print("  ", {k: v for k, v in res.items() if isinstance(v, int)}, flush=True)
    assert res["quota"] + res["nomem_pool"] + res["nomem_class"] > 0


def test_lifecycle_alloc_free_quota(cs):
    rc, ctx = cs.sched_create(capacity_bytes=1 << 30, max_jobs=8, slab_pool_bytes=64 << 20,
                              queue_capacity=4096)
    assert rc == 0
    try:
        _, a = cs.sched_register(ctx)
        _, b = cs.sched_register(ctx)
        assert cs.sched_alloc(ctx, a, 100)[0] == cs.SCHED_E_QUOTA    # nothing reserved yet
        assert cs.sched_admit(ctx, a, 0, 3 << 20) == 0
        rc, p1 = cs.sched_alloc(ctx, a, 1 << 20)
        assert rc == 0 and p1
        rc, p2 = cs.sched_alloc(ctx, a, 300)                           # 512 B class
        assert rc == 0
        rc, big = cs.sched_alloc(ctx, a, (2 << 20) - 512)              # large tier, 4 KiB pages
        assert rc == cs.SCHED_E_QUOTA                                  # 1 MiB + 512 + 2 MiB > 3 MiB
        rc, big = cs.sched_alloc(ctx, a, (1 << 20) + 4096)
        assert rc == 0
        t = torch.empty(0)  # noqa: F841
        assert cs.sched_free(ctx, b, p1) == cs.SCHED_E_INVALID          # not b's block
        assert cs.sched_free(ctx, a, p1) == 0
        assert cs.sched_free(ctx, a, p1) == cs.SCHED_E_INVALID          # double free
        assert cs.sched_free(ctx, a, big) == 0
        assert cs.sched_free(ctx, a, p2) == 0
        rc, ch, pool = cs.sched_slab_counters(ctx, 2)
        assert ch == [0, 0] and pool == 0
    finally:
        cs.sched_destroy(ctx)
