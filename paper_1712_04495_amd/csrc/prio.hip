// Queue order for the priority policies (Sec. V, Policies 3 and 4): before a
// pass, the live queue [head, tail) is stably ordered by priority (lower value
// first).  Within one priority the previous order is kept, and since older
// entries of a class always precede newer arrivals, that order is arrival
// order: the pass then walks the queue in (priority, arrival) order.
//
// The ordering is a least-significant-digit radix sort with 4-bit digits over
// key = priority - lo, where [lo, hi] bounds the priorities of every job the
// context knows (the host records them at registration), so only
// ceil(bitlen(hi - lo) / 4) digit passes run: one for up to 16 distinct
// consecutive priorities, none when every job has the same priority.  Each
// digit pass is a counting sort that keeps the order of equal digits:
//   count   -- per 4096-entry tile, the number of entries of each digit;
//   scan    -- one workgroup turns the digit-major table of tile counts into
//              global offsets (entries of smaller digits, then of the same
//              digit in earlier tiles);
//   scatter -- each tile ranks its entries within the tile (thread t owns 16
//              consecutive entries, so a rank is the count of the same digit
//              in earlier threads plus the earlier ones of its own run) and
//              writes key and source index to offset + rank.
// The queue entries are then gathered in the final order and written back.
// A pass is skipped when nothing was appended since the last ordering:
// compaction and withdrawal keep the order, so the queue is still sorted.
#include <algorithm>

#include "runtime.h"

using namespace schedk;

namespace {

constexpr int PR_THREADS = 256;
constexpr int PR_ITEMS = 16;                      // consecutive entries per thread
constexpr int PR_TILE = PR_THREADS * PR_ITEMS;    // 4096 entries per tile
constexpr int PR_BITS = 4;
constexpr int PR_BINS = 1 << PR_BITS;             // 16 digit values
constexpr int PR_SCAN_THREADS = 1024;

__global__ __launch_bounds__(PR_THREADS) void k_prio_keys(QueueArrays q, int64_t head, int64_t n,
                                                          int32_t lo, uint32_t *key,
                                                          uint32_t *idx) {
  const int64_t mask = q.capacity - 1;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    key[i] = uint32_t(int64_t(q.prio[(head + i) & mask]) - int64_t(lo));
    idx[i] = uint32_t(i);
  }
}

// Digits of thread t's 16 entries of tile `tile`; PR_BINS marks an entry
// beyond n.  Loads are 16-byte aligned: a run starts at a multiple of 16.
__device__ __forceinline__ void load_digits(const uint32_t *key, int64_t n, int64_t tile, int shift,
                                            uint32_t *dig) {
  const int64_t base = tile * PR_TILE + int64_t(threadIdx.x) * PR_ITEMS;
  if (base + PR_ITEMS <= n) {
    const uint4 *p = reinterpret_cast<const uint4 *>(key + base);
#pragma unroll
    for (int v = 0; v < PR_ITEMS / 4; ++v) {
      const uint4 w = p[v];
      dig[4 * v + 0] = (w.x >> shift) & (PR_BINS - 1);
      dig[4 * v + 1] = (w.y >> shift) & (PR_BINS - 1);
      dig[4 * v + 2] = (w.z >> shift) & (PR_BINS - 1);
      dig[4 * v + 3] = (w.w >> shift) & (PR_BINS - 1);
    }
  } else {
#pragma unroll
    for (int k = 0; k < PR_ITEMS; ++k)
      dig[k] = base + k < n ? (key[base + k] >> shift) & (PR_BINS - 1) : uint32_t(PR_BINS);
  }
}

// Fills cnt[d * PR_THREADS + t] with the exclusive prefix, in digit-major
// order, of the per-thread digit counts: the number of the tile's entries
// with a smaller digit plus those with digit d owned by threads before t.
// tot[d] receives the tile's count of digit d.  Ends with a barrier.
__device__ void tile_ranks(const uint32_t *dig, uint32_t *cnt, uint32_t *wsum, uint32_t *tot) {
  const int t = threadIdx.x;
#pragma unroll
  for (int d = 0; d < PR_BINS; ++d) cnt[d * PR_THREADS + t] = 0;
#pragma unroll
  for (int k = 0; k < PR_ITEMS; ++k)
    if (dig[k] < PR_BINS) cnt[dig[k] * PR_THREADS + t] += 1;  // own column only
  __syncthreads();
  // thread t scans the 16 consecutive counters [16t, 16t + 16) of the table
  uint32_t v[PR_ITEMS];
  uint32_t run = 0;
#pragma unroll
  for (int k = 0; k < PR_ITEMS; ++k) {
    v[k] = run;
    run += cnt[t * PR_ITEMS + k];
  }
  // exclusive scan of the 256 run totals: within the wave, then across waves
  const int lane = t & (WAVE - 1), w = t / WAVE;
  uint32_t incl = run;
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    const uint32_t u = __shfl_up(incl, off, WAVE);
    if (lane >= off) incl += u;
  }
  if (lane == WAVE - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t before = incl - run;
  for (int i = 0; i < w; ++i) before += wsum[i];
#pragma unroll
  for (int k = 0; k < PR_ITEMS; ++k) cnt[t * PR_ITEMS + k] = before + v[k];
  __syncthreads();
  if (t < PR_BINS) {
    const uint32_t end = t + 1 < PR_BINS ? cnt[(t + 1) * PR_THREADS]
                                         : wsum[0] + wsum[1] + wsum[2] + wsum[3];
    tot[t] = end - cnt[t * PR_THREADS];
  }
  __syncthreads();
}

// cnt_g[d * n_tiles + tile] = entries of digit d in tile `tile`
__global__ __launch_bounds__(PR_THREADS) void k_prio_count(const uint32_t *key, int64_t n,
                                                           int shift, int64_t n_tiles,
                                                           uint32_t *cnt_g) {
  __shared__ uint32_t cnt[PR_BINS * PR_THREADS];
  __shared__ uint32_t wsum[PR_THREADS / WAVE];
  __shared__ uint32_t tot[PR_BINS];
  uint32_t dig[PR_ITEMS];
  load_digits(key, n, blockIdx.x, shift, dig);
  tile_ranks(dig, cnt, wsum, tot);
  if (threadIdx.x < PR_BINS) cnt_g[int64_t(threadIdx.x) * n_tiles + blockIdx.x] = tot[threadIdx.x];
}

// In-place exclusive scan of m counts by one workgroup, in chunks of
// PR_SCAN_THREADS x 4 with a running carry.
__global__ __launch_bounds__(PR_SCAN_THREADS) void k_prio_scan(uint32_t *a, int64_t m) {
  __shared__ uint32_t wsum[PR_SCAN_THREADS / WAVE];
  __shared__ uint32_t carry_s;
  const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
  if (t == 0) carry_s = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < m; c0 += int64_t(PR_SCAN_THREADS) * 4) {
    const int64_t i0 = c0 + int64_t(t) * 4;
    uint32_t v[4], run = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = i0 + k < m ? a[i0 + k] : 0u;
      const uint32_t x = v[k];
      v[k] = run;
      run += x;
    }
    uint32_t incl = run;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
      const uint32_t u = __shfl_up(incl, off, WAVE);
      if (lane >= off) incl += u;
    }
    if (lane == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t before = carry_s + incl - run;
    for (int i = 0; i < w; ++i) before += wsum[i];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i0 + k < m) a[i0 + k] = before + v[k];
    __syncthreads();  // every thread has read carry_s and wsum
    if (t == PR_SCAN_THREADS - 1) carry_s = before + run;
    __syncthreads();
  }
}

__global__ __launch_bounds__(PR_THREADS) void k_prio_scatter(const uint32_t *key_in,
                                                             const uint32_t *idx_in, int64_t n,
                                                             int shift, int64_t n_tiles,
                                                             const uint32_t *ofs_g,
                                                             uint32_t *key_out,
                                                             uint32_t *idx_out) {
  __shared__ uint32_t cnt[PR_BINS * PR_THREADS];
  __shared__ uint32_t wsum[PR_THREADS / WAVE];
  __shared__ uint32_t tot[PR_BINS];
  __shared__ uint32_t dst0[PR_BINS];  // global offset of digit d's first entry of this tile
  uint32_t dig[PR_ITEMS];
  load_digits(key_in, n, blockIdx.x, shift, dig);
  tile_ranks(dig, cnt, wsum, tot);
  if (threadIdx.x < PR_BINS)
    dst0[threadIdx.x] = ofs_g[int64_t(threadIdx.x) * n_tiles + blockIdx.x] -
                        cnt[threadIdx.x * PR_THREADS];
  __syncthreads();
  const int t = threadIdx.x;
  const int64_t base = int64_t(blockIdx.x) * PR_TILE + int64_t(t) * PR_ITEMS;
#pragma unroll
  for (int k = 0; k < PR_ITEMS; ++k) {
    const uint32_t d = dig[k];
    if (d < PR_BINS) {
      uint32_t &r = cnt[d * PR_THREADS + t];  // own column only
      const uint32_t pos = dst0[d] + r;  // mod 2^32: dst0 may have wrapped
      r += 1;
      key_out[pos] = key_in[base + k];
      idx_out[pos] = idx_in[base + k];
    }
  }
}

// tmp <- queue entries in sorted order
__global__ void k_prio_permute(QueueArrays q, int64_t head, int64_t n, const uint32_t *order,
                               int64_t *t_dem, int32_t *t_job, int32_t *t_prio, int64_t *t_seq) {
  const int64_t mask = q.capacity - 1;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t src = (head + int64_t(order[i])) & mask;
    t_dem[i] = q.demand[src];
    t_job[i] = q.job[src];
    t_prio[i] = q.prio[src];
    t_seq[i] = q.seq[src];
  }
}

__global__ void k_prio_store(QueueArrays q, int64_t head, int64_t n, const int64_t *t_dem,
                             const int32_t *t_job, const int32_t *t_prio, const int64_t *t_seq) {
  const int64_t mask = q.capacity - 1;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t dst = (head + i) & mask;
    q.demand[dst] = t_dem[i];
    q.job[dst] = t_job[i];
    q.prio[dst] = t_prio[i];
    q.seq[dst] = t_seq[i];
  }
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace carve-up for a queue of Q entries.
struct PrioWs {
  uint32_t *key[2], *idx[2], *cnt;
  int64_t *t_dem, *t_seq;
  int32_t *t_job, *t_prio;
};

size_t ws_layout(int64_t Q, char *p, PrioWs *w) {
  const int64_t tiles = (Q + PR_TILE - 1) / PR_TILE;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *r = p ? p + off : nullptr;
    off += align256(bytes);
    return r;
  };
  PrioWs t;
  t.key[0] = (uint32_t *)take(4 * Q);
  t.key[1] = (uint32_t *)take(4 * Q);
  t.idx[0] = (uint32_t *)take(4 * Q);
  t.idx[1] = (uint32_t *)take(4 * Q);
  t.cnt = (uint32_t *)take(4 * size_t(PR_BINS) * tiles);
  t.t_dem = (int64_t *)take(8 * Q);
  t.t_seq = (int64_t *)take(8 * Q);
  t.t_job = (int32_t *)take(4 * Q);
  t.t_prio = (int32_t *)take(4 * Q);
  if (w) *w = t;
  return off;
}

}  // namespace

int sched_priority_alloc(sched_ctx *c) {
  const int64_t Q = c->q.capacity;
  if (Q > (int64_t(1) << 31)) return SCHED_E_INVALID;  // source indices are 32-bit
  const size_t need = ws_layout(Q, nullptr, nullptr);
  SCHED_HIP_TRY(hipMalloc(&c->prio_tmp, need));
  c->prio_tmp_bytes = need;
  return SCHED_OK;
}

void sched_priority_note(sched_ctx *c, int32_t prio) {
  c->sh->prio_lo = std::min(c->sh->prio_lo, prio);
  c->sh->prio_hi = std::max(c->sh->prio_hi, prio);
}

int sched_priority_reorder_locked(sched_ctx *c, hipStream_t s) {
  const int64_t n = c->sh->tail_h - c->sh->head_h;
  if (c->sh->prio_sorted_tail == c->sh->tail_h) return SCHED_OK;  // nothing appended since
  if (n <= 1 || c->sh->prio_hi <= c->sh->prio_lo) {
    c->sh->prio_sorted_tail = c->sh->tail_h;
    return SCHED_OK;
  }
  if (!c->prio_tmp) return SCHED_E_INTERNAL;
  PrioWs w;
  ws_layout(c->q.capacity, (char *)c->prio_tmp, &w);
  const uint64_t span = uint64_t(int64_t(c->sh->prio_hi) - int64_t(c->sh->prio_lo));
  int bits = 0;
  while (bits < 32 && (span >> bits) != 0) ++bits;
  const int passes = (bits + PR_BITS - 1) / PR_BITS;
  const int64_t tiles = (n + PR_TILE - 1) / PR_TILE;
  const int grid = int(std::min<int64_t>((n + 255) / 256, 2048));
  k_prio_keys<<<grid, PR_THREADS, 0, s>>>(c->q, c->sh->head_h, n, c->sh->prio_lo, w.key[0], w.idx[0]);
  SCHED_HIP_TRY(hipGetLastError());
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * PR_BITS;
    k_prio_count<<<unsigned(tiles), PR_THREADS, 0, s>>>(w.key[cur], n, shift, tiles, w.cnt);
    SCHED_HIP_TRY(hipGetLastError());
    k_prio_scan<<<1, PR_SCAN_THREADS, 0, s>>>(w.cnt, int64_t(PR_BINS) * tiles);
    SCHED_HIP_TRY(hipGetLastError());
    k_prio_scatter<<<unsigned(tiles), PR_THREADS, 0, s>>>(w.key[cur], w.idx[cur], n, shift, tiles,
                                                          w.cnt, w.key[cur ^ 1], w.idx[cur ^ 1]);
    SCHED_HIP_TRY(hipGetLastError());
    cur ^= 1;
  }
  k_prio_permute<<<grid, PR_THREADS, 0, s>>>(c->q, c->sh->head_h, n, w.idx[cur], w.t_dem, w.t_job,
                                             w.t_prio, w.t_seq);
  SCHED_HIP_TRY(hipGetLastError());
  k_prio_store<<<grid, PR_THREADS, 0, s>>>(c->q, c->sh->head_h, n, w.t_dem, w.t_job, w.t_prio,
                                           w.t_seq);
  SCHED_HIP_TRY(hipGetLastError());
  c->sh->prio_sorted_tail = c->sh->tail_h;
  return SCHED_OK;
}
