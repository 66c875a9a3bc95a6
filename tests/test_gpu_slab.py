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


def test_duplicate_frees_with_concurrent_allocs(cs):
    """Frees that name the same allocation twice in one phase, beside
    allocations of the same class that can only succeed on blocks freed in
    that phase: exactly one free of each pair succeeds, no block is handed out
    while still held, and the device counters equal the log's (check_log).
    Phase 0 fills class 0 (256 B) completely; phase 1 frees 1024 of its blocks,
    each named by two frees, while 2048 allocations compete for them; phase 2
    frees everything still held once."""
    from workloads import OP_ALLOC, OP_FREE
    pool = 13 << 20                       # 1 MiB regions: class 0 holds 4096 blocks
    region, cap = design_capacity(pool)
    T = 4
    rng = np.random.default_rng(11)
    kind, ten, size, ref = [], [], [], []

    def op(k, t, sz=0, r=-1):
        kind.append(k), ten.append(t), size.append(sz), ref.append(r)

    n0 = int(cap[0])
    for i in range(n0):                   # phase 0
        op(OP_ALLOC, i % T, 256)
    victims = rng.choice(n0, 1024, replace=False)
    ph1 = []
    for v in victims:
        ph1 += [(OP_FREE, int(v) % T, 0, int(v))] * 2
    ph1 += [(OP_ALLOC, int(t), 200, -1) for t in rng.integers(0, T, 2048)]
    for j in rng.permutation(len(ph1)):   # phase 1, interleaved
        op(*ph1[j])
    p1 = n0
    held0 = sorted(set(range(n0)) - set(int(v) for v in victims))
    ph2 = [(OP_FREE, i % T, 0, i) for i in held0]
    ph2 += [(OP_FREE, ten[p1 + j], 0, p1 + j) for j in range(len(ph1)) if kind[p1 + j] == OP_ALLOC]
    for j in rng.permutation(len(ph2)):   # phase 2
        op(*ph2[j])
    kind = np.array(kind, np.uint8)
    ten = np.array(ten, np.int32)
    size = np.array(size, np.int64)
    ref = np.array(ref, np.int64)
    quotas = np.full(T, 1 << 30, np.int64)
    bounds = [0, n0, n0 + len(ph1), kind.size]
    rc, ctx = cs.sched_create(capacity_bytes=1 << 40, max_jobs=16, max_tenants=T,
                              slab_pool_bytes=pool, queue_capacity=4096)
    assert rc == 0
    try:
        assert cs.sched_slab_set_quotas(ctx, quotas) == 0
        rc, info = cs.sched_slab_info(ctx)
        dk, dt, ds, dr = (torch.from_numpy(x).to(DEV) for x in (kind, ten, size, ref))
        ptr = torch.zeros(kind.size, dtype=torch.int64, device=DEV)
        st = torch.full((kind.size,), -1, dtype=torch.int8, device=DEV)
        for b0, b1 in zip(bounds[:-1], bounds[1:]):
            assert cs.sched_slab_ops(ctx, b0, b1, dk, dt, ds, dr, ptr, st) == 0
        torch.cuda.synchronize()
        rc, charged, pool_used = cs.sched_slab_counters(ctx, T)
        assert rc == 0
        st_h = st.cpu().numpy()
        ptr_h = ptr.cpu().numpy().view(np.uint64)
    finally:
        cs.sched_destroy(ctx)
    # phases of unequal length: check_log runs on fixed-length phases, so it
    # is given each phase's ops padded to one length with invalid frees
    L = max(b1 - b0 for b0, b1 in zip(bounds[:-1], bounds[1:]))
    pk, pt, ps, pr, pst, pp = [], [], [], [], [], []
    remap = {}
    for b0, b1 in zip(bounds[:-1], bounds[1:]):
        base = len(pk)
        for i in range(b0, b1):
            remap[i] = base + i - b0
        for i in range(b0, b1):
            pk.append(kind[i]), pt.append(ten[i]), ps.append(size[i])
            pr.append(remap[int(ref[i])] if ref[i] >= 0 else -1)
            pst.append(st_h[i]), pp.append(ptr_h[i])
        for _ in range(L - (b1 - b0)):
            pk.append(OP_FREE), pt.append(0), ps.append(0), pr.append(-1)
            pst.append(A.ST_INVALID), pp.append(0)
    res = A.check_log(np.array(pk, np.uint8), np.array(pt), np.array(ps), np.array(pr), quotas,
                      pool, cap, L, np.array(pst), np.array(pp, np.uint64), info["pool_base"],
                      final_charged=charged, final_pool=pool_used, span=13 * info["region_bytes"])
    fr1 = st_h[n0:n0 + len(ph1)][kind[n0:n0 + len(ph1)] == OP_FREE]
    print(f"  phase-1 frees ok={int((fr1 == 0).sum())} of {fr1.size}; "
          f"allocs ok={int((st_h[n0:n0 + len(ph1)][kind[n0:n0 + len(ph1)] == OP_ALLOC] == 0).sum())}",
          flush=True)
    assert int((fr1 == 0).sum()) == 1024
    assert res["pool_used"] == 0 and list(res["charged"]) == [0] * T
