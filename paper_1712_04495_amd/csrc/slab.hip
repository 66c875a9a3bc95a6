// Quota-checked slab sub-allocator in HBM.
//
// The paper records, next to the total memory in use, the memory each client
// uses (Sec. III-B) and only accepts a post-free of memory the client holds
// (Sec. IV).  This allocator carries that itemised accounting down to the
// blocks co-scheduled tenants allocate:
//   * 13 power-of-two classes, 256 B .. 1 MiB; a request takes the smallest
//     class that holds it and is charged the class size;
//   * the pool is one device allocation split into 13 equal regions (whole
//     MiB each), region c holding blocks of class c: capacity_c =
//     region_bytes / class_bytes(c) blocks, one bit each in a bitmap;
//   * an allocation charges its tenant (<= quota) and the pool (<= pool
//     bytes), then claims a free bit with an atomic OR; a failure returns
//     every charge it took, so a counter never holds more than its value at
//     the start of a phase plus the charges of allocations that got past it;
//   * a free checks that the block lies in the pool, is aligned, belongs to
//     the freeing tenant and is live, clears its bit and returns the charges.
//     Each block's owner word holds (allocating op, tenant); a free takes the
//     block back with one compare-and-swap of that word to "empty" before it
//     clears the bit, so of two frees that name one allocation only one can
//     succeed, and a free can never take a block that a later allocation
//     (of any tenant) claimed in the meantime.
// A batch of concurrent ops (a phase) first sums, per tenant and for the
// pool, the class bytes its allocations could take.  A counter that cannot
// reach its limit even if all of them succeed needs no compare-and-swap: its
// charges are added after the fact, aggregated per workgroup in LDS.  A
// counter that may bind is charged before the claim: per lane with a
// compare-and-swap loop for a tenant, and for the single pool counter by a
// wave-wide first-fit that reserves the run of lanes that fits with one
// compare-and-swap.
// Quotas come either from an explicit table (standalone use) or from the
// jobs' admitted reservations (tenant = job).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "prof.h"
#include "runtime.h"

using namespace schedk;

namespace {

constexpr int N_CLASSES = 13;
constexpr int MIN_LOG2 = 8;
constexpr int64_t MiB = 1 << 20;

// status codes of a device op
constexpr int8_t ST_OK = 0;
constexpr int8_t ST_QUOTA = 1;
constexpr int8_t ST_NOMEM_POOL = 2;
constexpr int8_t ST_NOMEM_CLASS = 3;
constexpr int8_t ST_INVALID = 4;

constexpr uint8_t OPK_ALLOC = 0;
constexpr uint8_t OPK_FREE = 1;

struct SlabDev {
  uint8_t *base;
  int64_t pool_bytes;
  int64_t region_bytes;
  int64_t cap[N_CLASSES];        // blocks per class
  int64_t words_off[N_CLASSES];  // offset of the class bitmap in `bits`
  int64_t n_words[N_CLASSES];
  int64_t owner_off[N_CLASSES];  // offset of the class owner table in `owner`
  unsigned long long *bits;
  unsigned long long *owner;     // per block: owner_word(op, tenant), or OWNER_EMPTY
  int64_t *charged;              // per tenant
  int64_t *pool_used;            // one counter
  const int64_t *quota;          // per tenant
  int64_t *phase_sum;            // per tenant, then the pool: class bytes a phase may charge
  uint8_t *unbounded;            // per tenant, then the pool: 1 = cannot bind this phase
  int32_t n_tenants;
};

constexpr unsigned long long OWNER_EMPTY = ~0ULL;
// Owner word of a block: the low 32 bits of the allocating op's index and the
// tenant.  A phase free names its alloc op, so it must find exactly this word.
__device__ __forceinline__ unsigned long long owner_word(uint64_t op, int32_t t) {
  return ((op & 0xffffffffULL) << 32) | uint32_t(t);
}

constexpr int PH_THREADS = 256;
constexpr int PH_LDS_TENANTS = 1024;  // tenants aggregated in LDS; beyond: direct atomics

__device__ __forceinline__ int size_class(int64_t size) {
  if (size < 1 || size > (int64_t(1) << (MIN_LOG2 + N_CLASSES - 1))) return -1;
  int c = 0;
  while ((int64_t(1) << (MIN_LOG2 + c)) < size) ++c;
  return c;
}

__device__ __forceinline__ uint32_t mix32(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  return uint32_t(x);
}

// Adds v to *ctr if the result stays <= limit.  Returns false without
// touching the counter otherwise.
__device__ __forceinline__ bool charge(int64_t *ctr, int64_t v, int64_t limit) {
  int64_t cur = ld_relaxed(ctr);
  for (;;) {
    if (cur + v > limit) return false;
    if (__hip_atomic_compare_exchange_strong(ctr, &cur, cur + v, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return true;
  }
}

__device__ bool slab_claim(const SlabDev &s, int c, int32_t t, uint64_t hint, uint64_t op,
                           uint64_t *out_ptr);

// One allocation with every counter charged by compare-and-swap (the
// single-op entry point).
__device__ int8_t slab_alloc_one(const SlabDev &s, int32_t t, int64_t size, uint64_t hint,
                                 uint64_t *out_ptr) {
  const int c = size_class(size);
  if (c < 0 || t < 0 || t >= s.n_tenants) return ST_INVALID;
  const int64_t cs = int64_t(1) << (MIN_LOG2 + c);
  if (!charge(&s.charged[t], cs, s.quota[t])) return ST_QUOTA;
  if (!charge(s.pool_used, cs, s.pool_bytes)) {
    add_relaxed(&s.charged[t], -cs);
    return ST_NOMEM_POOL;
  }
  if (slab_claim(s, c, t, hint, hint, out_ptr)) return ST_OK;
  add_relaxed(s.pool_used, -cs);
  add_relaxed(&s.charged[t], -cs);
  return ST_NOMEM_CLASS;
}

// Clears the block's bit if the free is valid; the caller returns the
// charges (*cs = class bytes on ST_OK).  op >= 0: the free names the alloc op
// that returned ptr, whose owner word the block must still hold; op < 0: any
// block the tenant holds (the pointer-only single-op free).
__device__ int8_t slab_free_claim(const SlabDev &s, int32_t t, uint64_t ptr, int64_t op,
                                  int64_t *cs_out) {
  if (t < 0 || t >= s.n_tenants) return ST_INVALID;
  const uint64_t b0 = uint64_t(s.base);
  if (ptr < b0 || ptr >= b0 + uint64_t(N_CLASSES) * uint64_t(s.region_bytes)) return ST_INVALID;
  const int64_t off = int64_t(ptr - b0);
  const int c = int(off / s.region_bytes);
  const int64_t roff = off - int64_t(c) * s.region_bytes;
  const int64_t cs = int64_t(1) << (MIN_LOG2 + c);
  if (roff % cs) return ST_INVALID;
  const int64_t blk = roff / cs;
  if (blk >= s.cap[c]) return ST_INVALID;
  unsigned long long *ow = s.owner + s.owner_off[c] + blk;
  unsigned long long want = op >= 0 ? owner_word(uint64_t(op), t) : ld_relaxed(ow);
  if (want == OWNER_EMPTY || int32_t(uint32_t(want)) != t) return ST_INVALID;
  // taking the owner word first makes the free exclusive: a second free of
  // the same allocation, or one racing a new claim of the block, fails here
  if (!__hip_atomic_compare_exchange_strong(ow, &want, OWNER_EMPTY, __ATOMIC_RELAXED,
                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    return ST_INVALID;
  const unsigned long long bit = 1ULL << (blk & 63);
  const unsigned long long old = __hip_atomic_fetch_and(s.bits + s.words_off[c] + (blk >> 6), ~bit,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!(old & bit)) return ST_INVALID;  // an owner word on a free block: never written so
  *cs_out = cs;
  return ST_OK;
}

__device__ int8_t slab_free_one(const SlabDev &s, int32_t t, uint64_t ptr) {
  int64_t cs = 0;
  const int8_t st = slab_free_claim(s, t, ptr, -1, &cs);
  if (st == ST_OK) {
    add_relaxed(s.pool_used, -cs);
    add_relaxed(&s.charged[t], -cs);
  }
  return st;
}

// Claims a free block of class c (charges already settled by the caller) for
// alloc op `op` of tenant t.
__device__ bool slab_claim(const SlabDev &s, int c, int32_t t, uint64_t hint, uint64_t op,
                           uint64_t *out_ptr) {
  const int64_t cs = int64_t(1) << (MIN_LOG2 + c);
  const int64_t nw = s.n_words[c];
  unsigned long long *bits = s.bits + s.words_off[c];
  const int64_t w0 = nw > 0 ? int64_t(mix32(hint) % uint64_t(nw)) : 0;
  for (int64_t k = 0; k < nw; ++k) {
    int64_t w = w0 + k;
    if (w >= nw) w -= nw;
    unsigned long long cur = ld_relaxed(bits + w);
    while (~cur) {
      const int b = __builtin_ctzll(~cur);
      const unsigned long long bit = 1ULL << b;
      const unsigned long long old =
          __hip_atomic_fetch_or(bits + w, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!(old & bit)) {
        const int64_t blk = w * 64 + b;
        st_relaxed(s.owner + s.owner_off[c] + blk, owner_word(op, t));
        *out_ptr = uint64_t(s.base + int64_t(c) * s.region_bytes + blk * cs);
        return true;
      }
      cur = old | bit;
    }
  }
  return false;
}

// Wave-collective charge of v (> 0) for the lanes with `want` against
// *ctr <= limit; every lane of the wave calls it.  Lanes go in lane order,
// first fit: the run of pending lanes whose running sum fits above the last
// counter value read is reserved with one compare-and-swap; the lane that
// breaks the run is refused (that value plus the run plus its own v exceeds
// the limit) and the rest are tried again.  Returns whether this lane's
// charge went in.
__device__ bool charge_wave_first_fit(int64_t *ctr, int64_t v, bool want, int64_t limit) {
  const int lane = lane_id();
  uint64_t pending = __ballot(want);
  if (!pending) return false;
  bool got = false;
  int64_t cur = read_lane64(ld_relaxed(ctr), __builtin_ctzll(pending));
  while (pending) {
    const bool mine = (pending >> lane) & 1;
    const int64_t pre = wave_incl_scan(mine ? v : 0);
    const uint64_t fit = __ballot(mine && pre <= limit - cur);
    if (fit) {
      const int last = 63 - __builtin_clzll(fit);
      const int leader = __builtin_ctzll(fit);
      const int64_t tot = read_lane64(pre, last);
      int64_t seen = cur;
      int ok = 0;
      if (lane == leader)
        ok = __hip_atomic_compare_exchange_strong(ctr, &seen, cur + tot, __ATOMIC_RELAXED,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ok = __builtin_amdgcn_readlane(ok, leader);
      seen = read_lane64(seen, leader);
      if (!ok) {
        cur = seen;
        continue;
      }
      cur += tot;
      got = got || ((fit >> lane) & 1);
      pending &= ~fit;
    }
    pending &= pending - 1;  // the lane that breaks the run does not fit
  }
  return got;
}

// Class bytes each tenant's allocations in ops [begin, end) could charge,
// and their total (slot n_tenants); added into phase_sum, which is zero
// before the phase.
__global__ __launch_bounds__(PH_THREADS) void k_slab_sum(SlabDev s, int64_t begin, int64_t end,
                                                         const uint8_t *__restrict__ kind,
                                                         const int32_t *__restrict__ tenant,
                                                         const int64_t *__restrict__ size) {
  __shared__ int64_t agg[PH_LDS_TENANTS];
  __shared__ int64_t red[PH_THREADS / WAVE];
  const bool lds = s.n_tenants <= PH_LDS_TENANTS;
  if (lds)
    for (int i = threadIdx.x; i < s.n_tenants; i += PH_THREADS) agg[i] = 0;
  __syncthreads();
  int64_t total = 0;
  for (int64_t i = begin + blockIdx.x * int64_t(PH_THREADS) + threadIdx.x; i < end;
       i += int64_t(gridDim.x) * PH_THREADS) {
    if (kind[i] != OPK_ALLOC) continue;
    const int32_t t = tenant[i];
    const int c = size_class(size[i]);
    if (c < 0 || t < 0 || t >= s.n_tenants) continue;
    const int64_t cs = int64_t(1) << (MIN_LOG2 + c);
    total += cs;
    if (lds)
      atomicAdd((unsigned long long *)&agg[t], (unsigned long long)cs);
    else
      add_relaxed(&s.phase_sum[t], cs);
  }
  total = block_sum<PH_THREADS>(total, red);  // ends with a barrier after the LDS adds
  if (lds)
    for (int i = threadIdx.x; i < s.n_tenants; i += PH_THREADS)
      if (agg[i]) add_relaxed(&s.phase_sum[i], agg[i]);
  if (threadIdx.x == 0 && total) add_relaxed(&s.phase_sum[s.n_tenants], total);
}

// Per counter: can it reach its limit in this phase?  Clears phase_sum for
// the next phase.
__global__ void k_slab_bound(SlabDev s) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= s.n_tenants; i += gridDim.x * blockDim.x) {
    const int64_t sum = s.phase_sum[i];
    const bool free_run = i < s.n_tenants ? ld_relaxed(&s.charged[i]) + sum <= s.quota[i]
                                          : ld_relaxed(s.pool_used) + sum <= s.pool_bytes;
    s.unbounded[i] = free_run ? 1 : 0;
    s.phase_sum[i] = 0;
  }
}

// One phase of concurrent ops [begin, end).  Arrays are indexed by the global
// op index; a free names an alloc op of an earlier phase by index.
__global__ __launch_bounds__(PH_THREADS) void k_slab_phase(
    SlabDev s, int64_t begin, int64_t end, const uint8_t *__restrict__ kind,
    const int32_t *__restrict__ tenant, const int64_t *__restrict__ size,
    const int64_t *__restrict__ ref, uint64_t *__restrict__ ptr, int8_t *__restrict__ status) {
  __shared__ int64_t agg[PH_LDS_TENANTS];  // deferred tenant charges of this workgroup
  const bool lds = s.n_tenants <= PH_LDS_TENANTS;
  if (lds)
    for (int i = threadIdx.x; i < s.n_tenants; i += PH_THREADS) agg[i] = 0;
  __syncthreads();
  const bool pool_free_run = s.unbounded[s.n_tenants] != 0;
  // the loop bound is uniform over the workgroup: every lane reaches the
  // wave-wide pool charge together
  for (int64_t base = begin + blockIdx.x * int64_t(PH_THREADS); base < end;
       base += int64_t(gridDim.x) * PH_THREADS) {
    const int64_t i = base + threadIdx.x;
    const bool active = i < end;
    int8_t st = ST_INVALID;
    uint64_t p = 0;
    int64_t cs = 0, tenant_delta = 0, pool_delta = 0;
    int32_t t = -1;
    int c = -1;
    bool t_free_run = false, want_pool = false, is_alloc = false;
    if (active) {
      t = tenant[i];
      const uint8_t k = kind[i];
      is_alloc = k == OPK_ALLOC;
      if (is_alloc) {
        c = size_class(size[i]);
        if (c >= 0 && t >= 0 && t < s.n_tenants) {
          cs = int64_t(1) << (MIN_LOG2 + c);
          t_free_run = s.unbounded[t] != 0;
          if (t_free_run || charge(&s.charged[t], cs, s.quota[t]))
            want_pool = true;
          else
            st = ST_QUOTA;
        }
      } else {
        const int64_t r = ref[i];
        if (k == OPK_FREE && r >= 0 && r < begin && kind[r] == OPK_ALLOC && status[r] == ST_OK) {
          int64_t fcs = 0;
          st = slab_free_claim(s, t, ptr[r], r, &fcs);
          if (st == ST_OK) {
            tenant_delta = -fcs;
            pool_delta = -fcs;
          }
        }
      }
    }
    bool pooled = want_pool;
    if (!pool_free_run) pooled = charge_wave_first_fit(s.pool_used, cs, want_pool, s.pool_bytes);
    if (want_pool) {
      if (!pooled) {
        st = ST_NOMEM_POOL;
        if (!t_free_run) add_relaxed(&s.charged[t], -cs);
      } else if (slab_claim(s, c, t, uint64_t(i) * 0x9E3779B97F4A7C15ULL, uint64_t(i), &p)) {
        st = ST_OK;
        if (t_free_run) tenant_delta = cs;
        if (pool_free_run) pool_delta = cs;
      } else {
        st = ST_NOMEM_CLASS;
        if (!pool_free_run) add_relaxed(s.pool_used, -cs);
        if (!t_free_run) add_relaxed(&s.charged[t], -cs);
      }
    }
    if (tenant_delta) {
      if (lds)
        atomicAdd((unsigned long long *)&agg[t], (unsigned long long)tenant_delta);
      else
        add_relaxed(&s.charged[t], tenant_delta);
    }
    pool_delta = wave_sum(pool_delta);
    if (lane_id() == 0 && pool_delta) add_relaxed(s.pool_used, pool_delta);
    if (active) {
      status[i] = st;
      ptr[i] = st == ST_OK && is_alloc ? p : 0;
    }
  }
  __syncthreads();
  if (lds)
    for (int i = threadIdx.x; i < s.n_tenants; i += PH_THREADS)
      if (agg[i]) add_relaxed(&s.charged[i], agg[i]);
}

__global__ void k_slab_one(SlabDev s, int32_t t, int64_t size, uint64_t fptr, int is_free,
                           uint64_t hint, uint64_t *out_ptr, int8_t *out_st) {
  if (threadIdx.x || blockIdx.x) return;
  uint64_t p = 0;
  const int8_t st = is_free ? slab_free_one(s, t, fptr) : slab_alloc_one(s, t, size, hint, &p);
  *out_ptr = p;
  *out_st = st;
}

// Charges (v > 0) or uncharges (v < 0) a tenant without a block: the large
// tier.  Status ST_OK or ST_QUOTA.
__global__ void k_slab_charge(SlabDev s, int32_t t, int64_t v, int8_t *out_st) {
  if (threadIdx.x || blockIdx.x) return;
  if (v >= 0) {
    *out_st = charge(&s.charged[t], v, s.quota[t]) ? ST_OK : ST_QUOTA;
  } else {
    add_relaxed(&s.charged[t], v);
    *out_st = ST_OK;
  }
}

__global__ void k_slab_reset_bits(SlabDev s) {
  for (int c = 0; c < N_CLASSES; ++c) {
    unsigned long long *bits = s.bits + s.words_off[c];
    const int64_t nw = s.n_words[c], cap = s.cap[c];
    for (int64_t w = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; w < nw;
         w += int64_t(gridDim.x) * blockDim.x) {
      // bits beyond the class capacity are permanently taken
      const int64_t lo = w * 64;
      unsigned long long v = 0;
      if (lo + 64 > cap) {
        const int64_t valid = cap - lo;
        v = valid <= 0 ? ~0ULL : (~0ULL << valid);
      }
      bits[w] = v;
    }
    unsigned long long *ow = s.owner + s.owner_off[c];
    for (int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; b < cap;
         b += int64_t(gridDim.x) * blockDim.x)
      ow[b] = OWNER_EMPTY;
  }
}

}  // namespace

struct SlabState {
  SlabDev dev{};
  int64_t *d_quota = nullptr;       // explicit quota table
  bool explicit_quota = false;
  uint64_t *d_one_ptr = nullptr;
  int8_t *d_one_st = nullptr;
  void *h_one = nullptr;
  uint64_t hint = 1;
  hipEvent_t last_phase = nullptr;  // completion of the last batch of ops
  bool phase_recorded = false;
  std::vector<std::pair<void *, int64_t>> large;  // large-tier blocks: ptr, charged bytes
  std::vector<int32_t> large_owner;
};

static int slab_apply_quota_source(sched_ctx *c) {
  SlabState *s = c->slab;
  s->dev.quota = s->explicit_quota ? s->d_quota : c->jb.res;
  return SCHED_OK;
}

int sched_slab_init(sched_ctx *c, int64_t pool_bytes, int32_t n_tenants) {
  const int64_t region = (pool_bytes / N_CLASSES) / MiB * MiB;
  if (region <= 0) return SCHED_E_INVALID;
  SlabState *s = new SlabState();
  c->slab = s;
  SlabDev &d = s->dev;
  d.pool_bytes = pool_bytes;
  d.region_bytes = region;
  d.n_tenants = n_tenants;
  int64_t words = 0, owners = 0;
  for (int k = 0; k < N_CLASSES; ++k) {
    d.cap[k] = region >> (MIN_LOG2 + k);
    d.n_words[k] = (d.cap[k] + 63) / 64;
    d.words_off[k] = words;
    d.owner_off[k] = owners;
    words += d.n_words[k];
    owners += d.cap[k];
  }
  SCHED_HIP_TRY(hipMalloc(&d.base, size_t(region) * N_CLASSES));
  SCHED_HIP_TRY(hipMalloc(&d.bits, sizeof(unsigned long long) * words));
  SCHED_HIP_TRY(hipMalloc(&d.owner, sizeof(unsigned long long) * owners));
  SCHED_HIP_TRY(hipMalloc(&d.charged, sizeof(int64_t) * n_tenants));
  SCHED_HIP_TRY(hipMemset(d.charged, 0, sizeof(int64_t) * n_tenants));
  SCHED_HIP_TRY(hipMalloc(&d.pool_used, sizeof(int64_t)));
  SCHED_HIP_TRY(hipMemset(d.pool_used, 0, sizeof(int64_t)));
  SCHED_HIP_TRY(hipMalloc(&d.phase_sum, sizeof(int64_t) * (n_tenants + 1)));
  SCHED_HIP_TRY(hipMemset(d.phase_sum, 0, sizeof(int64_t) * (n_tenants + 1)));
  SCHED_HIP_TRY(hipMalloc(&d.unbounded, n_tenants + 1));
  SCHED_HIP_TRY(hipEventCreateWithFlags(&s->last_phase, hipEventDisableTiming));
  SCHED_HIP_TRY(hipMalloc(&s->d_quota, sizeof(int64_t) * n_tenants));
  SCHED_HIP_TRY(hipMemset(s->d_quota, 0, sizeof(int64_t) * n_tenants));
  SCHED_HIP_TRY(hipMalloc(&s->d_one_ptr, sizeof(uint64_t)));
  SCHED_HIP_TRY(hipMalloc(&s->d_one_st, sizeof(int8_t)));
  SCHED_HIP_TRY(hipHostMalloc(&s->h_one, 64, hipHostMallocDefault));
  k_slab_reset_bits<<<256, 256, 0, c->stream>>>(d);
  SCHED_HIP_TRY(hipGetLastError());
  // quotas default to the job reservations when tenants are jobs
  s->explicit_quota = n_tenants > c->jb.max_jobs;
  return slab_apply_quota_source(c);
}

void sched_slab_free(sched_ctx *c) {
  SlabState *s = c->slab;
  if (!s) return;
  for (auto &b : s->large)
    if (b.first) (void)hipFree(b.first);
  if (s->last_phase) (void)hipEventSynchronize(s->last_phase);
  void *dev[] = {s->dev.base,     s->dev.bits,      s->dev.owner,  s->dev.charged,
                 s->dev.pool_used, s->dev.phase_sum, s->dev.unbounded, s->d_quota,
                 s->d_one_ptr,    s->d_one_st};
  for (void *p : dev)
    if (p) (void)hipFree(p);
  if (s->h_one) (void)hipHostFree(s->h_one);
  if (s->last_phase) (void)hipEventDestroy(s->last_phase);
  delete s;
  c->slab = nullptr;
}

bool sched_slab_quota_is_reservation(sched_ctx *c) {
  return c->slab && !c->slab->explicit_quota && c->slab->dev.n_tenants >= c->jb.max_jobs;
}

int64_t sched_slab_pool_used(sched_ctx *c) {
  if (!c->slab) return 0;
  int64_t v = 0;
  if (c->slab->phase_recorded && hipEventSynchronize(c->slab->last_phase) != hipSuccess) return -1;
  if (hipMemcpy(&v, c->slab->dev.pool_used, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return v;
}

static int8_t to_status_code(int8_t st) {
  switch (st) {
    case ST_OK: return SCHED_OK;
    case ST_QUOTA: return SCHED_E_QUOTA;
    case ST_NOMEM_POOL:
    case ST_NOMEM_CLASS: return SCHED_E_NOMEM;
    default: return SCHED_E_INVALID;
  }
}

// Work on the context stream starts after the last batch of ops, which may
// run on another stream: a batch decides before it starts which counters can
// bind, and must not see charges from outside it.
static int slab_after_phase(sched_ctx *c, hipStream_t st) {
  SlabState *s = c->slab;
  if (s->phase_recorded) SCHED_HIP_TRY(hipStreamWaitEvent(st, s->last_phase, 0));
  return SCHED_OK;
}

static int slab_one_locked(sched_ctx *c, int32_t t, int64_t size, uint64_t fptr, int is_free,
                           uint64_t *out_ptr, int8_t *out_st) {
  SlabState *s = c->slab;
  if (int rc = slab_after_phase(c, c->stream)) return rc;
  k_slab_one<<<1, 64, 0, c->stream>>>(s->dev, t, size, fptr, is_free, s->hint++ * 0x9E3779B97F4A7C15ULL,
                                      s->d_one_ptr, s->d_one_st);
  SCHED_HIP_TRY(hipGetLastError());
  SCHED_HIP_TRY(hipMemcpyAsync(s->h_one, s->d_one_ptr, 8, hipMemcpyDeviceToHost, c->stream));
  SCHED_HIP_TRY(hipMemcpyAsync((char *)s->h_one + 8, s->d_one_st, 1, hipMemcpyDeviceToHost, c->stream));
  SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
  *out_ptr = *(uint64_t *)s->h_one;
  *out_st = *((int8_t *)s->h_one + 8);
  return SCHED_OK;
}

static int slab_charge_locked(sched_ctx *c, int32_t t, int64_t v, int8_t *st) {
  SlabState *s = c->slab;
  if (int rc = slab_after_phase(c, c->stream)) return rc;
  k_slab_charge<<<1, 64, 0, c->stream>>>(s->dev, t, v, s->d_one_st);
  SCHED_HIP_TRY(hipGetLastError());
  SCHED_HIP_TRY(hipMemcpyAsync((char *)s->h_one + 8, s->d_one_st, 1, hipMemcpyDeviceToHost, c->stream));
  SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
  *st = *((int8_t *)s->h_one + 8);
  return SCHED_OK;
}

extern "C" int sched_alloc(sched_ctx_t *c, sched_job_t job, size_t bytes, void **dev_ptr) {
  if (!c || !dev_ptr) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (!c->slab || job < 0 || job >= c->sh->n_jobs || job >= c->slab->dev.n_tenants || bytes == 0)
    return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  SlabState *s = c->slab;
  if (bytes <= size_t(MiB)) {
    uint64_t p = 0;
    int8_t st = 0;
    if (int rc = slab_one_locked(c, job, int64_t(bytes), 0, 0, &p, &st)) return rc;
    if (st == ST_NOMEM_POOL || st == ST_NOMEM_CLASS) c->sh->stats.violations += 1;
    if (st != ST_OK) return to_status_code(st);
    *dev_ptr = (void *)p;
    return SCHED_OK;
  }
  // large tier: its own device allocation, charged to the job in 4 KiB pages
  const int64_t charged = int64_t((bytes + 4095) / 4096 * 4096);
  int8_t st = 0;
  if (int rc = slab_charge_locked(c, job, charged, &st)) return rc;
  if (st != ST_OK) return SCHED_E_QUOTA;
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    int8_t st2;
    (void)slab_charge_locked(c, job, -charged, &st2);
    c->sh->stats.violations += 1;
    return SCHED_E_NOMEM;
  }
  s->large.push_back({p, charged});
  s->large_owner.push_back(job);
  *dev_ptr = p;
  return SCHED_OK;
}

extern "C" int sched_free(sched_ctx_t *c, sched_job_t job, void *dev_ptr) {
  if (!c) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (!c->slab || job < 0 || job >= c->sh->n_jobs || job >= c->slab->dev.n_tenants || !dev_ptr)
    return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  SlabState *s = c->slab;
  for (size_t i = 0; i < s->large.size(); ++i) {
    if (s->large[i].first == dev_ptr) {
      if (s->large_owner[i] != job) return SCHED_E_INVALID;
      int8_t st;
      if (int rc = slab_charge_locked(c, job, -s->large[i].second, &st)) return rc;
      SCHED_HIP_TRY(hipFree(dev_ptr));
      s->large[i] = s->large.back();
      s->large.pop_back();
      s->large_owner[i] = s->large_owner.back();
      s->large_owner.pop_back();
      return SCHED_OK;
    }
  }
  uint64_t p = 0;
  int8_t st = 0;
  if (int rc = slab_one_locked(c, job, 0, uint64_t(dev_ptr), 1, &p, &st)) return rc;
  return st == ST_OK ? SCHED_OK : SCHED_E_INVALID;
}

extern "C" int sched_slab_set_quotas(sched_ctx_t *c, int32_t n, const int64_t *h_quotas) {
  if (!c || n < 0 || (n > 0 && !h_quotas)) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (!c->slab || n > c->slab->dev.n_tenants) return SCHED_E_INVALID;
  for (int32_t i = 0; i < n; ++i)
    if (h_quotas[i] < 0) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  SlabState *s = c->slab;
  if (int rc = slab_after_phase(c, c->stream)) return rc;
  std::vector<int64_t> q(s->dev.n_tenants, 0);
  std::copy(h_quotas, h_quotas + n, q.begin());
  SCHED_HIP_TRY(hipMemcpyAsync(s->d_quota, q.data(), sizeof(int64_t) * q.size(), hipMemcpyHostToDevice,
                               c->stream));
  SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
  s->explicit_quota = true;
  return slab_apply_quota_source(c);
}

extern "C" int sched_slab_ops(sched_ctx_t *c, int64_t begin, int64_t end, const uint8_t *d_kind,
                              const int32_t *d_tenant, const int64_t *d_size, const int64_t *d_ref,
                              uint64_t *d_ptr, int8_t *d_status, sched_stream_t stream) {
  if (!c || begin < 0 || end < begin) return SCHED_E_INVALID;
  if (end > begin && (!d_kind || !d_tenant || !d_size || !d_ref || !d_ptr || !d_status))
    return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (!c->slab) return SCHED_E_INVALID;
  if (end == begin) return SCHED_OK;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = stream ? (hipStream_t)stream : c->stream;
  SlabState *st = c->slab;
  const SlabDev &d = st->dev;
  if (int rc = slab_after_phase(c, s)) return rc;
  const int64_t n = end - begin;
  const int grid = int(std::min<int64_t>((n + PH_THREADS - 1) / PH_THREADS, 1024));
  k_slab_sum<<<grid, PH_THREADS, 0, s>>>(d, begin, end, d_kind, d_tenant, d_size);
  SCHED_HIP_TRY(hipGetLastError());
  k_slab_bound<<<(d.n_tenants + 1 + 255) / 256, 256, 0, s>>>(d);
  SCHED_HIP_TRY(hipGetLastError());
  SCHED_PROF_LAUNCH("k_slab_phase", s,
                    (k_slab_phase<<<grid, PH_THREADS, 0, s>>>(d, begin, end, d_kind, d_tenant, d_size,
                                                              d_ref, d_ptr, d_status)));
  SCHED_HIP_TRY(hipGetLastError());
  SCHED_HIP_TRY(hipEventRecord(st->last_phase, s));
  st->phase_recorded = true;
  return SCHED_OK;
}

extern "C" int sched_slab_info(sched_ctx_t *c, sched_slab_info_t *out) {
  if (!c || !out) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (!c->slab) return SCHED_E_INVALID;
  const SlabDev &d = c->slab->dev;
  sched_slab_info_t r{};
  r.pool_base = uint64_t(d.base);
  r.pool_bytes = d.pool_bytes;
  r.region_bytes = d.region_bytes;
  r.n_classes = N_CLASSES;
  r.n_tenants = d.n_tenants;
  for (int k = 0; k < N_CLASSES; ++k) r.class_blocks[k] = d.cap[k];
  *out = r;
  return SCHED_OK;
}

extern "C" int sched_slab_counters(sched_ctx_t *c, int32_t n, int64_t *h_charged,
                                   int64_t *h_pool_used) {
  if (!c || n < 0 || (n > 0 && !h_charged) || !h_pool_used) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (!c->slab || n > c->slab->dev.n_tenants) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  if (c->slab->phase_recorded) SCHED_HIP_TRY(hipEventSynchronize(c->slab->last_phase));
  SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
  if (n) SCHED_HIP_TRY(hipMemcpy(h_charged, c->slab->dev.charged, sizeof(int64_t) * n, hipMemcpyDeviceToHost));
  SCHED_HIP_TRY(hipMemcpy(h_pool_used, c->slab->dev.pool_used, sizeof(int64_t), hipMemcpyDeviceToHost));
  return SCHED_OK;
}

extern "C" int sched_slab_reset(sched_ctx_t *c) {
  if (!c) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (!c->slab) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  SlabState *s = c->slab;
  if (s->phase_recorded) SCHED_HIP_TRY(hipEventSynchronize(s->last_phase));
  for (auto &b : s->large)
    if (b.first) (void)hipFree(b.first);
  s->large.clear();
  s->large_owner.clear();
  k_slab_reset_bits<<<256, 256, 0, c->stream>>>(s->dev);
  SCHED_HIP_TRY(hipGetLastError());
  SCHED_HIP_TRY(hipMemsetAsync(s->dev.charged, 0, sizeof(int64_t) * s->dev.n_tenants, c->stream));
  SCHED_HIP_TRY(hipMemsetAsync(s->dev.pool_used, 0, sizeof(int64_t), c->stream));
  SCHED_HIP_TRY(hipMemsetAsync(s->dev.phase_sum, 0, sizeof(int64_t) * (s->dev.n_tenants + 1), c->stream));
  SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
  return SCHED_OK;
}


// ======================================================================
// Page tier (see pages.h): the serving loop's tenant memory.
// ======================================================================
namespace {

constexpr int PG_THREADS = 256;
constexpr int PG_MAX_JOBS_PER_PLACEMENT = PG_THREADS * 64;  // one 64-bit mask per thread

// Control words of the page tier.
enum : int {
  PGC_PAGES = 0,     // pages in use (the free stack holds n_pages - this)
  PGC_NODES = 1,     // nodes in use
  PGC_CHARGED = 2,   // bytes charged over all live placements
  PGC_VIOL = 3,      // placements of admitted jobs that failed
  PGC_PLACED = 4,    // placements made
  PGC_RELEASED = 5,  // placements released
  PGC_INV = 6,       // charged total seen above the admitted total
  PGC_PEAK = 7,      // most pages in use at once
  PGC_N = 8
};

constexpr int32_t PG_ST_PLACED = 0, PG_ST_QUOTA = 1, PG_ST_POOL = 2, PG_ST_NODES = 3,
                  PG_ST_INVALID = 5, PG_ST_RELEASED = 6;

struct PageTierDev {
  char *pool;
  uint32_t *stack;   // free pages: entries [0, n_pages - ctl[PGC_PAGES])
  uint32_t *nstack;  // free nodes: entries [0, n_nodes - ctl[PGC_NODES])
  uint32_t *nodes;   // n_nodes * PG_NODE page numbers
  uint32_t *dirs;    // n_slots * PG_DIR entries
  PlaceRec *recs;    // n_slots
  int64_t *ctl;      // PGC_N words
  int64_t n_pages, n_nodes;
  int32_t n_slots;
};

// Like charge(), returning the counter's value before the charge.
__device__ __forceinline__ bool charge_from(int64_t *ctr, int64_t v, int64_t limit, int64_t *before) {
  int64_t cur = ld_relaxed(ctr);
  for (;;) {
    if (cur + v > limit) return false;
    if (__hip_atomic_compare_exchange_strong(ctr, &cur, cur + v, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      *before = cur;
      return true;
    }
  }
}

__global__ void k_pg_init(PageTierDev d) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < d.n_pages;
       i += int64_t(gridDim.x) * blockDim.x)
    d.stack[i] = uint32_t(i);
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < d.n_nodes;
       i += int64_t(gridDim.x) * blockDim.x)
    d.nstack[i] = uint32_t(i);
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < d.n_slots;
       i += int64_t(gridDim.x) * blockDim.x)
    d.recs[i] = PlaceRec{0, 0, 0, PG_ST_RELEASED};
  if (blockIdx.x == 0 && threadIdx.x < PGC_N) d.ctl[threadIdx.x] = 0;
}

// One workgroup per placement request.  Charges every job of the placement
// against its quota (the job's admitted reservation), takes the pages (and
// nodes) with one compare-and-swap each, and writes the page table.  Any
// failure returns what was taken, leaves the placement empty and counts a
// violation: admission guarantees that it cannot happen.
__global__ __launch_bounds__(PG_THREADS) void k_pg_place(PageTierDev d, SlabDev s,
                                                         const int64_t *__restrict__ used,
                                                         const PgReq *__restrict__ reqs,
                                                         const int32_t *__restrict__ jobs,
                                                         const int64_t *__restrict__ bytes,
                                                         int32_t *__restrict__ job_status) {
  __shared__ int s_fail;
  __shared__ int32_t s_status;
  __shared__ int64_t s_pbase, s_nbase, s_bytes;
  const PgReq r = reqs[blockIdx.x];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_fail = 0;
    s_bytes = 0;
    s_status = PG_ST_PLACED;
  }
  __syncthreads();
  const bool valid = r.slot >= 0 && r.slot < d.n_slots && r.pages >= 0 &&
                     r.pages <= PG_MAX_PAGES && r.n_jobs >= 0 &&
                     r.n_jobs <= PG_MAX_JOBS_PER_PLACEMENT;
  const int64_t k = valid ? r.pages : 0;
  const int32_t nn = k > PG_DIR ? int32_t((k + PG_NODE - 1) / PG_NODE) : 0;
  // 1. the quota of every job of the placement
  uint64_t got = 0;
  int64_t mine = 0;
  if (valid) {
    int bit = 0;
    for (int64_t i = tid; i < r.n_jobs; i += PG_THREADS, ++bit) {
      const int32_t j = jobs[r.job_off + i];
      const int64_t b = bytes[r.job_off + i];
      if (j < 0 || j >= s.n_tenants || b < 0 || !charge(&s.charged[j], b, s.quota[j])) {
        atomicOr(&s_fail, 1);
      } else {
        got |= 1ULL << bit;
        mine += b;
      }
    }
  } else if (tid == 0) {
    s_fail = 1;
  }
  if (mine) atomicAdd((unsigned long long *)&s_bytes, (unsigned long long)mine);
  __syncthreads();
  // 2. pages and nodes
  if (tid == 0) {
    if (s_fail) {
      s_status = valid ? PG_ST_QUOTA : PG_ST_INVALID;
    } else {
      int64_t before = 0;
      if (!charge_from(&d.ctl[PGC_PAGES], k, d.n_pages, &before)) {
        s_status = PG_ST_POOL;
      } else {
        s_pbase = d.n_pages - before - k;
        max_relaxed(&d.ctl[PGC_PEAK], before + k);
        if (nn) {
          int64_t nb = 0;
          if (!charge_from(&d.ctl[PGC_NODES], int64_t(nn), d.n_nodes, &nb)) {
            add_relaxed(&d.ctl[PGC_PAGES], -k);
            s_status = PG_ST_NODES;
          } else {
            s_nbase = d.n_nodes - nb - nn;
          }
        }
      }
      if (s_status != PG_ST_PLACED) s_fail = 1;
    }
  }
  __syncthreads();
  PlaceRec *rec = d.recs + (valid ? r.slot : 0);
  if (s_fail) {
    // return the quota charges this thread took
    if (valid) {
      int bit = 0;
      for (int64_t i = tid; i < r.n_jobs; i += PG_THREADS, ++bit)
        if ((got >> bit) & 1) add_relaxed(&s.charged[jobs[r.job_off + i]], -bytes[r.job_off + i]);
    }
    if (valid && job_status)
      for (int64_t i = tid; i < r.n_jobs; i += PG_THREADS) {
        const int32_t j = jobs[r.job_off + i];
        if (j >= 0 && j < s.n_tenants) job_status[j] = s_status;
      }
    if (tid == 0) {
      add_relaxed(&d.ctl[PGC_VIOL], int64_t(1));
      if (valid) *rec = PlaceRec{0, 0, 0, s_status};
    }
    return;
  }
  // 3. the page table
  uint32_t *dir = d.dirs + int64_t(r.slot) * PG_DIR;
  const int64_t pb = s_pbase, nb = s_nbase;
  for (int64_t i = tid; i < k; i += PG_THREADS) {
    const uint32_t pg = d.stack[pb + i];
    if (!nn) {
      dir[i] = pg;
    } else {
      const uint32_t node = d.nstack[nb + (i >> PG_NODE_SHIFT)];
      d.nodes[uint64_t(node) * PG_NODE + (i & (PG_NODE - 1))] = pg;
      if ((i & (PG_NODE - 1)) == 0) dir[i >> PG_NODE_SHIFT] = node;
    }
  }
  if (job_status)
    for (int64_t i = tid; i < r.n_jobs; i += PG_THREADS) job_status[jobs[r.job_off + i]] = PG_ST_PLACED;
  __syncthreads();
  if (tid == 0) {
    *rec = PlaceRec{k, s_bytes, nn, PG_ST_PLACED};
    const int64_t tot = add_relaxed(&d.ctl[PGC_CHARGED], s_bytes) + s_bytes;
    add_relaxed(&d.ctl[PGC_PLACED], int64_t(1));
    // the bytes charged over all live placements never exceed the admitted
    // reservations (every placement is released before its reservation is)
    if (tot > ld_relaxed(used)) add_relaxed(&d.ctl[PGC_INV], int64_t(1));
  }
}

// One workgroup per released slot: pushes its pages and nodes back and
// returns its jobs' charges.
__global__ __launch_bounds__(PG_THREADS) void k_pg_release(PageTierDev d, SlabDev s,
                                                           const PgReq *__restrict__ reqs,
                                                           const int32_t *__restrict__ jobs,
                                                           const int64_t *__restrict__ bytes) {
  __shared__ int64_t s_pbase, s_nbase;
  __shared__ PlaceRec s_rec;
  const PgReq r = reqs[blockIdx.x];
  const int tid = threadIdx.x;
  if (r.slot < 0 || r.slot >= d.n_slots) return;
  PlaceRec *rec = d.recs + r.slot;
  if (tid == 0) s_rec = *rec;
  __syncthreads();
  if (s_rec.status != PG_ST_PLACED) return;  // nothing mapped, no charge held
  const int64_t k = s_rec.pages;
  const int32_t nn = s_rec.nodes;
  if (tid == 0) {
    s_pbase = d.n_pages - add_relaxed(&d.ctl[PGC_PAGES], -k);
    if (nn) s_nbase = d.n_nodes - add_relaxed(&d.ctl[PGC_NODES], -int64_t(nn));
  }
  __syncthreads();
  const uint32_t *dir = d.dirs + int64_t(r.slot) * PG_DIR;
  for (int64_t i = tid; i < k; i += PG_THREADS)
    d.stack[s_pbase + i] =
        nn ? d.nodes[uint64_t(dir[i >> PG_NODE_SHIFT]) * PG_NODE + (i & (PG_NODE - 1))] : dir[i];
  for (int32_t i = tid; i < nn; i += PG_THREADS) d.nstack[s_nbase + i] = dir[i];
  if (r.n_jobs >= 0 && r.n_jobs <= PG_MAX_JOBS_PER_PLACEMENT)
    for (int64_t i = tid; i < r.n_jobs; i += PG_THREADS) {
      const int32_t j = jobs[r.job_off + i];
      if (j >= 0 && j < s.n_tenants) add_relaxed(&s.charged[j], -bytes[r.job_off + i]);
    }
  __syncthreads();
  if (tid == 0) {
    add_relaxed(&d.ctl[PGC_CHARGED], -s_rec.bytes);
    add_relaxed(&d.ctl[PGC_RELEASED], int64_t(1));
    *rec = PlaceRec{0, 0, 0, PG_ST_RELEASED};
  }
}

// Free-stack check when nothing is placed: every page (node) number appears
// exactly once.  seen[] is zero on entry; bad[0] counts duplicates and
// out-of-range entries.
__global__ void k_pg_check(const uint32_t *__restrict__ st, int64_t n, uint32_t *seen,
                           unsigned long long *bad) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const uint32_t p = st[i];
    if (p >= uint64_t(n)) {
      atomicAdd(bad, 1ULL);
      continue;
    }
    const uint32_t bit = 1u << (p & 31);
    if (atomicOr(&seen[p >> 5], bit) & bit) atomicAdd(bad, 1ULL);
  }
}

// Identity page table over a contiguous buffer of k pages (for kernels that
// run outside a placement).
__global__ void k_pg_identity(uint32_t *dir, uint32_t *nodes, int64_t k) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < k;
       i += int64_t(gridDim.x) * blockDim.x) {
    if (k <= PG_DIR) {
      dir[i] = uint32_t(i);
    } else {
      nodes[i] = uint32_t(i);
      if ((i & (PG_NODE - 1)) == 0) dir[i >> PG_NODE_SHIFT] = uint32_t(i >> PG_NODE_SHIFT);
    }
  }
}

}  // namespace

struct PageTier {
  PageTierDev dev{};
  int device = 0;
};

int pg_create(sched_ctx *c, int64_t pool_pages, int32_t n_slots, hipStream_t s, PageTier **out) {
  if (!c->slab || pool_pages <= 0 || pool_pages > (int64_t(1) << 32) || n_slots <= 0)
    return SCHED_E_INVALID;
  PageTier *t = new PageTier();
  t->device = c->device;
  PageTierDev &d = t->dev;
  d.n_pages = pool_pages;
  d.n_nodes = 2 * ((pool_pages + PG_NODE - 1) / PG_NODE) + 2;
  d.n_slots = n_slots;
  auto fail = [&](hipError_t e) {
    sched_note_hip_error(e, "page tier allocation", __FILE__, __LINE__);
    pg_destroy(t);
    return SCHED_E_INTERNAL;
  };
  hipError_t e = hipMalloc(&d.pool, size_t(pool_pages) << PG_SHIFT);
  if (e == hipSuccess) e = hipMalloc(&d.stack, sizeof(uint32_t) * pool_pages);
  if (e == hipSuccess) e = hipMalloc(&d.nstack, sizeof(uint32_t) * d.n_nodes);
  if (e == hipSuccess) e = hipMalloc(&d.nodes, sizeof(uint32_t) * d.n_nodes * PG_NODE);
  if (e == hipSuccess) e = hipMalloc(&d.dirs, sizeof(uint32_t) * int64_t(n_slots) * PG_DIR);
  if (e == hipSuccess) e = hipMalloc(&d.recs, sizeof(PlaceRec) * n_slots);
  if (e == hipSuccess) e = hipMalloc(&d.ctl, sizeof(int64_t) * PGC_N);
  if (e != hipSuccess) return fail(e);
  k_pg_init<<<1024, 256, 0, s>>>(d);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  *out = t;
  return SCHED_OK;
}

void pg_destroy(PageTier *t) {
  if (!t) return;
  PageTierDev &d = t->dev;
  void *p[] = {d.pool, d.stack, d.nstack, d.nodes, d.dirs, d.recs, d.ctl};
  for (void *q : p)
    if (q) (void)hipFree(q);
  delete t;
}

int pg_place(sched_ctx *c, PageTier *t, int32_t n, const PgReq *reqs, const int32_t *jobs,
             const int64_t *bytes, int32_t *job_status, hipStream_t s) {
  if (n <= 0) return SCHED_OK;
  SCHED_PROF_LAUNCH("k_pg_place", s,
                    (k_pg_place<<<n, PG_THREADS, 0, s>>>(t->dev, c->slab->dev, &c->eng.d_ctl->used,
                                                         reqs, jobs, bytes, job_status)));
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int pg_release(sched_ctx *c, PageTier *t, int32_t n, const PgReq *reqs, const int32_t *jobs,
               const int64_t *bytes, hipStream_t s) {
  if (n <= 0) return SCHED_OK;
  SCHED_PROF_LAUNCH("k_pg_release", s,
                    (k_pg_release<<<n, PG_THREADS, 0, s>>>(t->dev, c->slab->dev, reqs, jobs, bytes)));
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

PageMap pg_map(const PageTier *t, int32_t slot, int64_t pages) {
  PageMap m{};
  m.pool = t->dev.pool;
  m.dir = t->dev.dirs + int64_t(slot) * PG_DIR;
  m.nodes = t->dev.nodes;
  m.rec = t->dev.recs + slot;
  m.direct = pages <= PG_DIR ? 1 : 0;
  return m;
}

int pg_counters(PageTier *t, hipStream_t s, PgCounters *out) {
  int64_t v[PGC_N] = {0};
  SCHED_HIP_TRY(hipStreamSynchronize(s));
  SCHED_HIP_TRY(hipMemcpy(v, t->dev.ctl, sizeof(v), hipMemcpyDeviceToHost));
  out->pages_used = v[PGC_PAGES];
  out->nodes_used = v[PGC_NODES];
  out->charged = v[PGC_CHARGED];
  out->violations = v[PGC_VIOL];
  out->placed = v[PGC_PLACED];
  out->released = v[PGC_RELEASED];
  out->over_admitted = v[PGC_INV];
  out->peak_pages = v[PGC_PEAK];
  out->pool_pages = t->dev.n_pages;
  return SCHED_OK;
}

int pg_check_free(PageTier *t, hipStream_t s, int64_t *bad) {
  const PageTierDev &d = t->dev;
  uint32_t *seen = nullptr;
  unsigned long long *d_bad = nullptr;
  const int64_t words = (std::max(d.n_pages, d.n_nodes) + 31) / 32;
  SCHED_HIP_TRY(hipMalloc(&seen, sizeof(uint32_t) * words));
  SCHED_HIP_TRY(hipMalloc(&d_bad, sizeof(unsigned long long)));
  unsigned long long h = 0;
  hipError_t e = hipMemsetAsync(d_bad, 0, sizeof(unsigned long long), s);
  const uint32_t *stacks[2] = {d.stack, d.nstack};
  const int64_t sizes[2] = {d.n_pages, d.n_nodes};
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipMemsetAsync(seen, 0, sizeof(uint32_t) * words, s);
    if (e == hipSuccess) {
      k_pg_check<<<1024, 256, 0, s>>>(stacks[k], sizes[k], seen, d_bad);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d_bad, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(seen);
  (void)hipFree(d_bad);
  if (e != hipSuccess) {
    sched_note_hip_error(e, "page tier check", __FILE__, __LINE__);
    return SCHED_E_INTERNAL;
  }
  *bad = int64_t(h);
  return SCHED_OK;
}

namespace schedk {

int pg_identity(char *base, int64_t bytes, hipStream_t s, PgIdentity *out) {
  const int64_t k = (bytes + PG_BYTES - 1) / PG_BYTES;
  if (k <= 0 || k > PG_MAX_PAGES) return SCHED_E_INVALID;
  *out = PgIdentity{};
  SCHED_HIP_TRY(hipMalloc(&out->dir, sizeof(uint32_t) * PG_DIR));
  if (k > PG_DIR) SCHED_HIP_TRY(hipMalloc(&out->nodes, sizeof(uint32_t) * k));
  SCHED_HIP_TRY(hipMalloc(&out->rec, sizeof(PlaceRec)));
  const PlaceRec r{k, 0, k > PG_DIR ? int32_t((k + PG_NODE - 1) / PG_NODE) : 0, PG_ST_PLACED};
  SCHED_HIP_TRY(hipMemcpyAsync(out->rec, &r, sizeof(r), hipMemcpyHostToDevice, s));
  k_pg_identity<<<int(std::min<int64_t>((k + 255) / 256, 1024)), 256, 0, s>>>(out->dir, out->nodes, k);
  SCHED_HIP_TRY(hipGetLastError());
  SCHED_HIP_TRY(hipStreamSynchronize(s));
  out->map = PageMap{base, out->dir, out->nodes, out->rec, k <= PG_DIR ? 1 : 0, 0};
  return SCHED_OK;
}

void pg_identity_free(PgIdentity *m) {
  void *p[] = {m->dir, m->nodes, m->rec};
  for (void *q : p)
    if (q) (void)hipFree(q);
  *m = PgIdentity{};
}

}  // namespace schedk
