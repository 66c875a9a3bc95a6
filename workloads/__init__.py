"""Seeded synthetic workload generators.

This module is the only code shared between the CPU oracle (``oracle/``) and
the HIP path (``paper_1712_04495_amd/``).  It produces job parameters and
random draws only -- demands, arrival times, job kinds, allocator op streams,
release coins -- and holds none of the scheduling or allocation arithmetic.
Every generator takes an explicit seed and uses numpy's PCG64
(``np.random.default_rng``), so both sides see identical inputs.

The shapes follow the paper's scenarios (Sec. VII-B/VII-C: many concurrent
jobs of uneven GPU-memory footprint sharing one GPU, compared with sequential
execution); the concrete sizes are the synthetic configurations C1..C5 and
the dense-scan and stressed variants listed below.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KiB = 1 << 10
MiB = 1 << 20
GiB = 1 << 30
PAGE = 4 * KiB

# Job kinds understood by the tenant kernels.
KIND_TRIAD = 0
KIND_GEMM = 1
KIND_HIST = 2

# Allocator op kinds (C3).
OP_ALLOC = 0
OP_FREE = 1


# --------------------------------------------------------------------------
# C2: admission microbenchmark queue
# --------------------------------------------------------------------------
@dataclass
class AdmissionQueue:
    """A pending queue in arrival order plus the per-round release coins."""

    seed: int
    demand: np.ndarray        # int64[n], bytes, 4 KiB aligned, arrival order
    capacity: int             # bytes
    coins: np.ndarray         # uint8[rounds-1, n]; coins[r-1, j] = release job j in round r
    rounds: int

    @property
    def n(self) -> int:
        return int(self.demand.shape[0])


def loguniform_pages(rng: np.random.Generator, n: int, lo_log2: int, hi_log2: int) -> np.ndarray:
    """Page counts floor(2**U) with U uniform on [lo_log2, hi_log2), clamped to >= 1."""
    u = rng.random(n)
    pages = np.floor(np.exp2(lo_log2 + u * (hi_log2 - lo_log2))).astype(np.int64)
    return np.clip(pages, 1, (1 << hi_log2) - 1)


def release_coins(seed: int, rounds: int, n: int) -> np.ndarray:
    """Fair coins: coins[r-1, j] == 1 releases running job j at round r (r >= 1)."""
    out = np.empty((max(rounds - 1, 0), n), dtype=np.uint8)
    for r in range(1, rounds):
        out[r - 1] = np.random.default_rng([seed, r]).integers(0, 2, size=n, dtype=np.uint8)
    return out


def c2_queue(seed: int = 2, n: int = 1 << 20, rounds: int = 8,
             capacity: int = 280 * 10**9) -> AdmissionQueue:
    """C2: n requests, demands log-uniform in [4 KiB, 4 GiB), 4 KiB aligned."""
    rng = np.random.default_rng(seed)
    demand = PAGE * loguniform_pages(rng, n, 0, 20)
    return AdmissionQueue(seed, demand, capacity, release_coins(seed, rounds, n), rounds)


def c2d_queue(seed: int = 2, n: int = 1 << 26, capacity: int = 280 * 10**9) -> AdmissionQueue:
    """C2-D (dense): demands log-uniform in [64 MiB, 4 GiB) so free memory stalls
    above zero and first-fit backfill has to inspect every entry."""
    rng = np.random.default_rng(seed)
    demand = PAGE * loguniform_pages(rng, n, 14, 20)
    return AdmissionQueue(seed, demand, capacity, np.zeros((0, n), np.uint8), 1)


def c2d_fifo_queue(seed: int = 2, n: int = 1 << 26) -> AdmissionQueue:
    """C2-D (a), a FIFO pass that decides every entry: demands 4096 * U{1..64}
    (4-256 KiB) and capacity equal to their sum, so the whole queue is the
    admitted prefix (the sum stays below 2^46 up to n = 2^28)."""
    rng = np.random.default_rng(seed + 1000)
    demand = PAGE * rng.integers(1, 65, size=n, dtype=np.int64)
    return AdmissionQueue(seed, demand, int(demand.sum()), np.zeros((0, n), np.uint8), 1)


def random_queue(seed: int, n: int, max_demand: int, holes: float = 0.0):
    """Small random queue for parity sweeps: demands uniform in [1, max_demand],
    a fraction ``holes`` of entries marked withdrawn (demand -1)."""
    rng = np.random.default_rng(seed)
    d = rng.integers(1, max_demand + 1, size=n, dtype=np.int64)
    if holes > 0:
        d[rng.random(n) < holes] = -1
    return d


# --------------------------------------------------------------------------
# C3 / C3-S: slab allocator op stream
# --------------------------------------------------------------------------
@dataclass
class SlabOps:
    seed: int
    quotas: np.ndarray        # int64[T]
    pool: int                 # bytes
    kind: np.ndarray          # uint8[n]  OP_ALLOC / OP_FREE
    tenant: np.ndarray        # int32[n]
    size: np.ndarray          # int64[n]  requested bytes (allocs); 0 for frees
    ref: np.ndarray           # int64[n]  alloc op index a free names; -1 for allocs
    phase_len: int

    @property
    def n(self) -> int:
        return int(self.kind.shape[0])

    @property
    def n_phases(self) -> int:
        return (self.n + self.phase_len - 1) // self.phase_len


def c3_ops(seed: int = 3, n_tenants: int = 64, n_ops: int = 1 << 22, phase_len: int = 1 << 16,
           pool: int = 1 << 36, quota_div: int = 1, p_alloc: float = 0.6,
           min_log2: int = 8, n_classes: int = 13) -> SlabOps:
    """C3: quotas uniform in [1, 8] GiB (4 KiB aligned, divided by ``quota_div``);
    sizes 256 B * 2**k with k = min(Geom(0.5) - 1, n_classes - 1); a free names a
    uniformly chosen not-yet-freed alloc of the same tenant from an earlier phase
    (when the tenant has none the op becomes an alloc)."""
    rng = np.random.default_rng(seed)
    q = rng.uniform(1.0, 8.0, size=n_tenants) * GiB / quota_div
    quotas = (PAGE * np.floor(q / PAGE)).astype(np.int64)
    tenant = rng.integers(0, n_tenants, size=n_ops, dtype=np.int32)
    want_free = rng.random(n_ops) >= p_alloc
    k = np.minimum(rng.geometric(0.5, size=n_ops) - 1, n_classes - 1)
    sizes = (np.int64(1) << (min_log2 + k)).astype(np.int64)
    pick = rng.random(n_ops)

    kind = np.zeros(n_ops, np.uint8)
    size = np.zeros(n_ops, np.int64)
    ref = np.full(n_ops, -1, np.int64)
    # per tenant: list of alloc op indices from earlier phases that no free names yet
    avail = [[] for _ in range(n_tenants)]
    pending_phase = [[] for _ in range(n_tenants)]
    for p0 in range(0, n_ops, phase_len):
        for t in range(n_tenants):
            avail[t].extend(pending_phase[t])
            pending_phase[t].clear()
        for i in range(p0, min(p0 + phase_len, n_ops)):
            t = tenant[i]
            pool_t = avail[t]
            if want_free[i] and pool_t:
                j = int(pick[i] * len(pool_t))
                pool_t[j], pool_t[-1] = pool_t[-1], pool_t[j]
                ref[i] = pool_t.pop()
                kind[i] = OP_FREE
            else:
                kind[i] = OP_ALLOC
                size[i] = sizes[i]
                pending_phase[t].append(i)
    return SlabOps(seed, quotas, pool, kind, tenant, size, ref, phase_len)


def c3s_ops(seed: int = 3, n_ops: int = 1 << 22) -> SlabOps:
    """C3-S: the stressed variant -- quotas divided by 64, pool of 1 GiB."""
    return c3_ops(seed=seed, n_ops=n_ops, pool=1 << 30, quota_div=64)


# --------------------------------------------------------------------------
# Job mixes for co-scheduling (C1, C4, C5)
# --------------------------------------------------------------------------
@dataclass
class JobMix:
    """Jobs in arrival order.  ``size`` is the kind's size parameter: fp32
    elements per array (triad), N (GEMM, M = N = K) or keys (histogram)."""

    seed: int
    arrival_s: np.ndarray     # float64[n], seconds from t = 0
    kind: np.ndarray          # int32[n]
    size: np.ndarray          # int64[n]
    demand: np.ndarray        # int64[n] declared bytes, 4 KiB aligned
    capacity: int
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.kind.shape[0])


def round_up(x, a):
    return ((np.asarray(x, dtype=np.int64) + a - 1) // a) * a


def triad_demand(n_elems):
    """Three fp32 arrays of n elements, each rounded to 4 KiB."""
    return 3 * round_up(np.asarray(n_elems, np.int64) * 4, PAGE)


def gemm_demand(N):
    """A and B^T in bf16 (2 N^2 B each) plus C in fp32 (4 N^2 B)."""
    N = np.asarray(N, np.int64)
    return round_up(2 * N * N, PAGE) * 2 + round_up(4 * N * N, PAGE)


HIST_BINS = 4096


def hist_demand(n_keys):
    """uint32 keys plus 4096 uint32 bins."""
    return round_up(np.asarray(n_keys, np.int64) * 4, PAGE) + round_up(HIST_BINS * 4, PAGE)


NOMINAL_BW = 5.0e12      # bytes/s, for virtual durations only
NOMINAL_FLOPS = 1.0e15   # flop/s, for virtual durations only


def nominal_vdur(kind, size):
    """Virtual duration of a job from its footprint (a job parameter, used by
    the virtual-clock schedule): streamed bytes over a nominal bandwidth,
    GEMM flops over a nominal rate."""
    kind = np.asarray(kind)
    size = np.asarray(size, dtype=np.float64)
    tri = (8.0 + 10 * 12.0) * size / NOMINAL_BW
    gem = 2.0 * size ** 3 / NOMINAL_FLOPS + 8.0 * size ** 2 / NOMINAL_BW
    his = 8.0 * size / NOMINAL_BW
    return np.where(kind == KIND_TRIAD, tri, np.where(kind == KIND_GEMM, gem, his))


def job_table(mix: "JobMix"):
    """The mix as a numpy structured array in the layout of sched_job_desc_t."""
    dt = np.dtype([("arrival_s", "<f8"), ("vdur_s", "<f8"), ("demand", "<i8"), ("size", "<i8"),
                   ("kind", "<i4"), ("priority", "<i4"), ("seed", "<u8")])
    t = np.zeros(mix.n, dtype=dt)
    t["arrival_s"] = mix.arrival_s
    t["vdur_s"] = nominal_vdur(mix.kind, mix.size)
    t["demand"] = mix.demand
    t["size"] = mix.size
    t["kind"] = mix.kind
    t["seed"] = (np.uint64(mix.seed) << np.uint64(20)) + np.arange(mix.n, dtype=np.uint64) + np.uint64(1)
    return t


def c1_jobs(seed: int = 1, n: int = 16, capacity: int = 8 * GiB, gap_s: float = 5e-3) -> JobMix:
    """C1: 16 triad jobs, footprint uniform in [64 MiB, 2 GiB] (4 KiB pages),
    Poisson arrivals with mean gap 5 ms, pool 8 GiB."""
    rng = np.random.default_rng(seed)
    pages = rng.integers(16384, 524288 + 1, size=n, dtype=np.int64)
    arrival = np.cumsum(rng.exponential(gap_s, size=n))
    n_elems = (PAGE * pages) // 12
    return JobMix(seed, arrival, np.full(n, KIND_TRIAD, np.int32), n_elems,
                  triad_demand(n_elems), capacity, "c1")


def c4_jobs(seed: int = 4, n: int = 10_000, capacity: int = 280 * 10**9,
            rate: float = 200.0) -> JobMix:
    """C4: serving mix -- 50 % triad (footprint uniform 0.5..16 GiB), 30 % bf16
    GEMM (N in {1024, 2048, 4096, 8192}), 20 % histogram (2**24..2**28 keys)."""
    rng = np.random.default_rng(seed)
    arrival = np.cumsum(rng.exponential(1.0 / rate, size=n))
    u = rng.random(n)
    kind = np.where(u < 0.5, KIND_TRIAD, np.where(u < 0.8, KIND_GEMM, KIND_HIST)).astype(np.int32)
    foot = rng.uniform(0.5 * GiB, 16.0 * GiB, size=n)
    tri_n = ((foot // (12 * PAGE)).astype(np.int64) * (12 * PAGE)) // 12
    gN = np.array([1024, 2048, 4096, 8192], np.int64)[rng.integers(0, 4, size=n)]
    hk = np.int64(1) << rng.integers(24, 29, size=n).astype(np.int64)
    size = np.where(kind == KIND_TRIAD, tri_n, np.where(kind == KIND_GEMM, gN, hk)).astype(np.int64)
    demand = np.where(kind == KIND_TRIAD, triad_demand(tri_n),
                      np.where(kind == KIND_GEMM, gemm_demand(gN), hist_demand(hk))).astype(np.int64)
    return JobMix(seed, arrival, kind, size, demand, capacity, "c4")


HOL_LONG, HOL_BLOCKER, HOL_SMALL = 0, 1, 2


def hol_jobs(seed: int = 6, n_small: int = 200, capacity: int = 32 * GiB,
             small_rate: float = 1000.0) -> JobMix:
    """HOL (head-of-line study, FIFO vs MMU): a long triad of 20 GiB footprint
    at t = 0, then at 1 ms a 16 GiB triad that cannot fit beside it, then
    ``n_small`` triads of 64-256 MiB footprint (log-uniform) arriving from 2 ms
    at a Poisson rate ``small_rate``.  Under FIFO the blocker holds every small
    job until the long one ends; under MMU they fill the free memory around
    it.  The small jobs' offered traffic (~1.4 TB/s at the default rate) stays
    well below HBM bandwidth, so their waits show the admission policy rather
    than a saturated device.  ``extra["cls"]`` labels the jobs HOL_LONG /
    HOL_BLOCKER / HOL_SMALL."""
    rng = np.random.default_rng(seed)
    small = np.exp2(rng.uniform(26.0, 28.0, size=n_small))
    foot = np.concatenate([[20.0 * GiB, 16.0 * GiB], small])
    tri_n = ((foot // (12 * PAGE)).astype(np.int64) * (12 * PAGE)) // 12
    arrival = np.concatenate([[0.0, 1e-3], 2e-3 + np.cumsum(rng.exponential(1.0 / small_rate,
                                                                             size=n_small))])
    cls = np.concatenate([[HOL_LONG, HOL_BLOCKER], np.full(n_small, HOL_SMALL)]).astype(np.int32)
    n = n_small + 2
    return JobMix(seed, arrival, np.full(n, KIND_TRIAD, np.int32), tri_n, triad_demand(tri_n),
                  capacity, "hol", {"cls": cls})


def c5_jobs(seed: int = 5, n: int = 50_000, capacity: int = 280 * 10**9,
            small_frac: float = 0.7, alpha: float = 1.2, oversub: float = 4.0) -> JobMix:
    """C5: oversubscribed batch of triads, all present at t = 0.  A fraction
    ``small_frac`` has footprints log-uniform in [1 MiB, 16 MiB); the rest is
    Pareto(alpha, x_m = 16 MiB) truncated at 64 GiB (resampled), then scaled so
    the aggregate demand is ``oversub`` x capacity, clamped to [16 MiB, 64 GiB]."""
    rng = np.random.default_rng(seed)
    n_small = int(round(small_frac * n))
    n_big = n - n_small
    small = np.exp2(rng.uniform(20.0, 24.0, size=n_small))
    big = np.empty(n_big)
    todo = np.arange(n_big)
    while todo.size:
        x = 16 * MiB * (1.0 + rng.pareto(alpha, size=todo.size))
        ok = x <= 64 * GiB
        big[todo[ok]] = x[ok]
        todo = todo[~ok]
    target = oversub * capacity
    scale = max((target - small.sum()) / big.sum(), 1e-9)
    big = np.clip(big * scale, 16 * MiB, 64 * GiB)
    foot = np.concatenate([small, big])
    order = rng.permutation(n)
    foot = foot[order]
    tri_n = (round_up(foot.astype(np.int64), PAGE) // 12).astype(np.int64)
    tri_n = np.maximum(tri_n, 1)
    return JobMix(seed, np.zeros(n), np.full(n, KIND_TRIAD, np.int32), tri_n,
                  triad_demand(tri_n), capacity, "c5", {"tail_scale": float(scale)})
