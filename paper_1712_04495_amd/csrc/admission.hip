// Admission kernels: FIFO prefix admission and first-fit backfill rounds over
// int64 demands (the paper's Policy 1 and Policy 2, Sec. V), plus queue
// intake, compaction/accounting and batched release (Sec. III-B state, Sec. IV
// pre-allocation and post-free).
//
// A pass is computed as rounds.  A round looks at the undecided entries from
// `start`, takes as candidates the present entries whose demand is <= R (every
// present entry under FIFO), and admits the longest prefix of candidates whose
// sum is <= R.  The first candidate past that prefix (the break) can never fit
// again in this pass because R only shrinks, so the next round starts right
// after it.  Under FIFO the first round is the whole pass.  Rounds reproduce
// sequential first-fit exactly; all arithmetic is exact int64.
//
// Two kernels compute rounds:
//  * k_window: one workgroup of 1024 threads walks the queue in windows of
//    4096 entries and runs all rounds of a window in LDS.  This is the
//    latency regime: when free memory runs out after a few thousand entries
//    the whole pass is one launch.
//  * k_round: a persistent grid that computes one round over the whole
//    remaining queue with a single-pass decoupled look-back scan.  Tiles are
//    taken from an atomic ticket in queue order; each tile publishes its
//    candidate sum (saturated at R + 1) and then its inclusive prefix in one
//    64-bit word (epoch:16 | status:2 | value:46).  Only the tile that holds
//    the break runs an ordered scan; every other tile either admits all of
//    its candidates or, lying past the break, admits nothing.  This is the
//    HBM-bound regime (the final round of a pass that never exhausts memory
//    reads every remaining demand once).
#include <climits>
#include <cstring>

#include "admission.h"
#include "prof.h"

namespace schedk {

constexpr uint64_t FL_AGG = 1;
constexpr uint64_t FL_INC = 2;
constexpr int64_t VMASK = (int64_t(1) << 46) - 1;

__device__ __forceinline__ unsigned long long pack_flag(uint32_t epoch, uint64_t st, int64_t v) {
  return (static_cast<unsigned long long>(epoch) << 48) | (st << 46) | uint64_t(v);
}

// The launch that follows L uses slot (L + 1) & 3: clear its ticket and break
// marker.  Launch L - 3 was the last user of that slot and has finished.
__device__ __forceinline__ void reset_next_slot(DevCtl *c, uint32_t L) {
  const int nx = (L + 1) & 3;
  c->ticket[nx] = 0;
  c->break_tile[nx] = LLONG_MAX;
  c->tiles_done[nx] = 0;
  c->round_sum[nx] = 0;
}

// Called once per tile that decided its entries.  In a round without a break
// every such tile admitted all of its candidates, so the round's admitted sum
// is the sum of the tiles' candidate sums; the tile that finishes last
// closes the round.  (With a break, the break tile closes it instead.)
__device__ __forceinline__ void tile_done(DevCtl *c, int s, int nx, int64_t a, int64_t R,
                                          int64_t end, long long n_tiles) {
  add_relaxed(&c->round_sum[s], (unsigned long long)a);
  const unsigned long long prev =
      __hip_atomic_fetch_add(&c->tiles_done[s], 1ULL, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  if (prev + 1 != (unsigned long long)n_tiles) return;
  if (__hip_atomic_load(&c->break_tile[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != LLONG_MAX)
    return;
  const int64_t sum = int64_t(ld_relaxed(&c->round_sum[s]));
  add_relaxed(&c->p_admitted_bytes, sum);
  add_relaxed(&c->p_rounds, (int64_t)1);
  c->rec[nx].R = R - sum;
  c->rec[nx].start = end;
  c->rec[nx].done = 1;
}

__device__ __forceinline__ void pass_init(DevCtl *c, uint32_t L, int filter, int from_state,
                                          int64_t R0, int64_t start, int64_t end, int append) {
  if (from_state) {
    R0 = c->capacity - c->used;
    start = c->head;
    end = c->tail;
  }
  const int s = L & 3;
  c->rec[s].R = R0;
  c->rec[s].start = start;
  c->rec[s].done = (start >= end || R0 <= 0) ? 1 : 0;
  c->ticket[s] = 0;
  c->break_tile[s] = LLONG_MAX;
  c->tiles_done[s] = 0;
  c->round_sum[s] = 0;
  c->p_admitted = 0;
  c->p_admitted_bytes = 0;
  c->p_hi = start;
  c->p_rounds = 0;
  c->p_R0 = R0;
  c->p_end = end;
  c->filter = filter;
  if (!append) c->adm_base = 0;
}

__global__ void k_prologue(DevCtl *c, uint32_t L, int filter, int from_state, int64_t R0,
                           int64_t start, int64_t end) {
  if (threadIdx.x != 0) return;
  pass_init(c, L, filter, from_state, R0, start, end, 0);
}

// Pass summary into host-mapped memory (stateless scans).
__global__ void k_summary(DevCtl *c, uint32_t L, PassSummary *out) {
  if (threadIdx.x != 0) return;
  const RoundRec &r = c->rec[L & 3];
  out->admitted = c->p_admitted;
  out->admitted_bytes = c->p_admitted_bytes;
  out->R0 = c->p_R0;
  out->R_after = r.R;
  out->rounds = c->p_rounds;
  out->start_final = r.start;
  out->hi = c->p_hi;
  out->head = c->head;
  out->tail = c->tail;
  out->used = c->used;
  out->adm_base = c->adm_base;
  out->done = r.done;
}

// ---------------------------------------------------------------------------
// Single-wave windowed rounds
// ---------------------------------------------------------------------------
// One wave walks the queue in windows of WIN entries; lane l holds the WIN_ITEMS
// consecutive entries starting at l * WIN_ITEMS, so a lane-local running sum
// plus one wave-wide exclusive scan gives every entry its prefix in queue
// order.  The break of a round is the lowest set bit of a ballot.  No LDS and
// no barriers: every round costs a few dozen wave instructions.
// init != 0: the kernel also does the prologue (pass start state from the
// arguments or, with from_state, from the control block).
__global__ __launch_bounds__(WIN_THREADS) void k_window(DevCtl *c, const int64_t *__restrict__ demand,
                                                        uint8_t *__restrict__ decision, int64_t mask,
                                                        uint32_t L, int max_windows, int init,
                                                        int filter_arg, int from_state, int64_t R0,
                                                        int64_t start0, int64_t end0, int append) {
  const int lane = threadIdx.x;
  const int s = L & 3, nx = (L + 1) & 3;
  // pass state in registers: every lane derives it from the same inputs
  int64_t R, pos, end, hi;
  int done;
  bool filter;
  if (init) {
    if (from_state) {
      R0 = c->capacity - c->used;
      start0 = c->head;
      end0 = c->tail;
    }
    R = R0;
    pos = start0;
    end = end0;
    hi = start0;
    filter = filter_arg != 0;
    done = (start0 >= end0 || R0 <= 0) ? 1 : 0;
  } else {
    const RoundRec r = c->rec[s];
    R = r.R;
    pos = r.start;
    done = r.done;
    end = c->p_end;
    filter = c->filter != 0;
    hi = c->p_hi;
  }
  if (lane == 0) reset_next_slot(c, L);
  int64_t adm_cnt = 0, adm_bytes = 0, rounds = 0;

  for (int w = 0; w < max_windows && !done; ++w) {
    if (pos >= end || R == 0) {
      done = 1;
      break;
    }
    const int64_t p0 = pos + int64_t(lane) * WIN_ITEMS;
    int64_t x[WIN_ITEMS];
#pragma unroll
    for (int k = 0; k < WIN_ITEMS; ++k) x[k] = (p0 + k < end) ? demand[(p0 + k) & mask] : -1;
    int s_loc = 0;
    for (;;) {
      const int64_t cap = R + 1;
      int64_t incl[WIN_ITEMS];
      int64_t run = 0;
#pragma unroll
      for (int k = 0; k < WIN_ITEMS; ++k) {
        const int off = lane * WIN_ITEMS + k;
        const bool cd = x[k] >= 0 && off >= s_loc && (!filter || x[k] <= R);
        run = sat_add(run, cd ? x[k] : 0, cap);
        incl[k] = cd ? run : -1;  // -1 marks a non-candidate
      }
      const int64_t wincl = wave_incl_scan_sat_dpp(run, cap);
      const int64_t ex = wave_prev_lane64(wincl);
      const int64_t total = read_lane64(wincl, WAVE - 1);
      int my_first = WIN_ITEMS;
      int64_t my_before = ex;
#pragma unroll
      for (int k = WIN_ITEMS - 1; k >= 0; --k) {
        if (incl[k] >= 0 && sat_add(ex, incl[k], cap) > R) my_first = k;
      }
      // prefix just before my_first: the last candidate before it, else ex
#pragma unroll
      for (int k = 0; k < WIN_ITEMS; ++k)
        if (k < my_first && incl[k] >= 0) my_before = sat_add(ex, incl[k], cap);
      const uint64_t ball = __ballot(my_first < WIN_ITEMS);
      int64_t first = WIN, sum = total;
      if (ball) {
        const int fl = __builtin_ctzll(ball);
        first = int64_t(fl) * WIN_ITEMS + __builtin_amdgcn_readlane(my_first, fl);
        sum = read_lane64(my_before, fl);
      }
      const int64_t lim = (first < WIN) ? first + 1 : WIN;
      int my_last = -1;  // last admitted item of this lane
      int64_t cnt = 0;
#pragma unroll
      for (int k = 0; k < WIN_ITEMS; ++k) {
        const int off = lane * WIN_ITEMS + k;
        const int64_t p = p0 + k;
        const bool in = off >= s_loc && off < lim && p < end;
        const bool a = in && incl[k] >= 0 && off < first;
        if (in) decision[p & mask] = a ? 1 : 0;
        if (a) my_last = k;
        cnt += __builtin_popcountll(__ballot(a));
      }
      adm_cnt += cnt;
      int64_t mx = -1;
      const uint64_t lb = __ballot(my_last >= 0);
      if (lb) {
        const int hl = 63 - __builtin_clzll(lb);
        mx = pos + int64_t(hl) * WIN_ITEMS + __builtin_amdgcn_readlane(my_last, hl);
      }
      adm_bytes += sum;
      if (mx + 1 > hi) hi = mx + 1;
      R -= sum;
      ++rounds;
      if (first >= WIN) {
        pos += WIN;
        break;
      }
      if (!filter || R == 0) {
        done = 1;
        pos += first + 1;
        break;
      }
      s_loc = int(first) + 1;
      if (s_loc >= WIN) {
        pos += WIN;
        break;
      }
    }
  }
  if (!done && (pos >= end || R == 0)) done = 1;
  if (lane == 0) {
    c->rec[nx].R = R;
    c->rec[nx].start = pos < end ? pos : end;
    c->rec[nx].done = done;
    if (init) {
      c->p_admitted = adm_cnt;
      c->p_admitted_bytes = adm_bytes;
      c->p_hi = hi;
      c->p_rounds = rounds;
      c->p_R0 = R0;
      c->p_end = end;
      c->filter = filter ? 1 : 0;
      if (!append) c->adm_base = 0;
    } else {
      c->p_admitted += adm_cnt;
      c->p_admitted_bytes += adm_bytes;
      c->p_hi = hi;
      c->p_rounds += rounds;
    }
  }
}

// ---------------------------------------------------------------------------
// Grid-wide round with decoupled look-back
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RND_THREADS) void k_round(DevCtl *c, const int64_t *__restrict__ demand,
                                                       uint8_t *__restrict__ decision, int64_t mask,
                                                       unsigned long long *flags, uint32_t L,
                                                       uint32_t epoch) {
  __shared__ int64_t red[RND_THREADS / WAVE];
  __shared__ long long s_t;
  __shared__ int64_t s_E;
  __shared__ int64_t s_brk_sum;
  const int tid = threadIdx.x;
  const int s = L & 3, nx = (L + 1) & 3;
  const RoundRec r = c->rec[s];
  if (blockIdx.x == 0 && tid == 0) {
    reset_next_slot(c, L);
    if (r.done) c->rec[nx] = r;
  }
  if (r.done) return;
  const int64_t R = r.R, start = r.start, end = c->p_end;
  const int64_t cap = R + 1;
  const bool filter = c->filter != 0;
  const long long n_tiles = (end - start + TILE - 1) / TILE;

  for (;;) {
    if (tid == 0) {
      const long long t = (long long)add_relaxed(&c->ticket[s], 1ULL);
      const long long bt = ld_relaxed(&c->break_tile[s]);
      s_t = (t < n_tiles && t <= bt) ? t : -1;
    }
    __syncthreads();
    const long long t = s_t;
    if (t < 0) break;
    const int64_t base = start + int64_t(t) * TILE;

    int64_t x[RND_ITEMS];
    int64_t tsum = 0;
#pragma unroll
    for (int j = 0; j < RND_ITEMS; ++j) {
      const int64_t p = base + int64_t(j) * RND_THREADS + tid;
      const int64_t v = p < end ? __builtin_nontemporal_load(demand + (p & mask)) : -1;
      const bool cd = v >= 0 && (!filter || v <= R);
      x[j] = cd ? v : -1;
      tsum += cd ? v : 0;
    }
    const int64_t Araw = block_sum<RND_THREADS>(tsum, red);
    const int64_t A = Araw < cap ? Araw : cap;

    if (Araw == 0) {
      // No candidate in this tile: every entry is rejected whatever the
      // prefix before it is, so the tile needs no look-back.  It publishes
      // its zero sum for the tiles after it (tile 0 knows its prefix is 0).
      if (tid == 0) st_relaxed(&flags[t], pack_flag(epoch, t == 0 ? FL_INC : FL_AGG, 0));
#pragma unroll
      for (int j = 0; j < RND_ITEMS; ++j) {
        const int64_t p = base + int64_t(j) * RND_THREADS + tid;
        if (p < end) decision[p & mask] = 0;
      }
      if (tid == 0) tile_done(c, s, nx, 0, R, end, n_tiles);
      continue;
    }

    if (tid < WAVE) {
      // Wave 0 looks back 64 predecessors at a time: lane l reads the flag of
      // tile p - l.  The nearest inclusive flag ends the walk once every
      // nearer predecessor has published its aggregate.
      const int lane = tid;
      int64_t E = 0;
      if (t == 0) {
        if (lane == 0) st_relaxed(&flags[t], pack_flag(epoch, FL_INC, A));
      } else {
        if (lane == 0) st_relaxed(&flags[t], pack_flag(epoch, FL_AGG, A));
        long long p = t - 1;
        for (;;) {
          const long long qq = p - lane;
          const unsigned long long f =
              qq >= 0 ? ld_relaxed(&flags[qq]) : pack_flag(epoch, FL_INC, 0);
          const uint64_t st = (f >> 46) & 3;
          const bool valid = uint32_t(f >> 48) == epoch && st != 0;
          const uint64_t inc_b = __ballot(valid && st == FL_INC);
          const uint64_t bad_b = __ballot(!valid);
          const int fi = inc_b ? __builtin_ctzll(inc_b) : WAVE;
          const uint64_t need = fi >= WAVE - 1 ? ~0ULL : ((2ULL << fi) - 1);
          if (bad_b & need) {
            // a predecessor that saw the break marker first may never publish
            if (ld_relaxed(&c->break_tile[s]) < t) {
              E = cap;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          const int64_t v = lane <= fi ? int64_t(f & VMASK) : 0;
          const int64_t w = wave_sum(v);  // <= 64 * cap, no overflow
          E = sat_add(E, w < cap ? w : cap, cap);
          if (fi < WAVE || E >= cap) break;
          p -= WAVE;
        }
        if (lane == 0) st_relaxed(&flags[t], pack_flag(epoch, FL_INC, sat_add(E, A, cap)));
      }
      if (lane == 0) {
        if (E <= R && sat_add(E, A, cap) > R) min_relaxed(&c->break_tile[s], (long long)t);
        s_E = E;
      }
    }
    __syncthreads();
    const int64_t E = s_E;
    if (E > R) continue;  // the break lies in an earlier tile, which closes the round

    int64_t tcnt = 0, tmax = -1;
    if (sat_add(E, A, cap) <= R) {
      // every candidate of this tile is admitted
#pragma unroll
      for (int j = 0; j < RND_ITEMS; ++j) {
        const int64_t p = base + int64_t(j) * RND_THREADS + tid;
        if (p < end) {
          const bool a = x[j] >= 0;
          decision[p & mask] = a ? 1 : 0;
          if (a) {
            ++tcnt;
            tmax = p;
          }
        }
      }
      const int64_t cnt = block_sum<RND_THREADS>(tcnt, red);
      const int64_t mx = block_max<RND_THREADS>(tmax, red);
      if (tid == 0) {
        if (cnt) {
          add_relaxed(&c->p_admitted, cnt);
          max_relaxed(&c->p_hi, mx + 1);
        }
        tile_done(c, s, nx, A, R, end, n_tiles);  // A is exact here: E + A <= R
      }
      continue;
    }

    // This tile holds the break: scan it row by row in queue order.
    int64_t carry = E, brk = -1, brk_sum = 0;
    for (int j = 0; j < RND_ITEMS; ++j) {
      const int64_t p = base + int64_t(j) * RND_THREADS + tid;
      const int64_t v = x[j] >= 0 ? x[j] : 0;
      int64_t rowtot;
      const int64_t ex = block_excl_scan_sat<RND_THREADS>(v, cap, red, &rowtot);
      const int64_t P = sat_add(carry, sat_add(ex, v, cap), cap);
      const bool over = x[j] >= 0 && P > R;
      const int64_t f = block_min<RND_THREADS>(over ? tid : RND_THREADS, red);
      if (f < RND_THREADS) {
        if (tid == f) s_brk_sum = sat_add(carry, ex, cap);
        if (tid <= f && p < end) {
          const bool a = x[j] >= 0 && tid < f;
          decision[p & mask] = a ? 1 : 0;
          if (a) {
            ++tcnt;
            tmax = p;
          }
        }
        __syncthreads();
        brk = base + int64_t(j) * RND_THREADS + f;
        brk_sum = s_brk_sum;
        break;
      }
      if (p < end) {
        const bool a = x[j] >= 0;
        decision[p & mask] = a ? 1 : 0;
        if (a) {
          ++tcnt;
          tmax = p;
        }
      }
      carry = sat_add(carry, rowtot, cap);
    }
    const int64_t cnt = block_sum<RND_THREADS>(tcnt, red);
    const int64_t mx = block_max<RND_THREADS>(tmax, red);
    if (tid == 0) {
      if (cnt) {
        add_relaxed(&c->p_admitted, cnt);
        max_relaxed(&c->p_hi, mx + 1);
      }
      add_relaxed(&c->p_admitted_bytes, brk_sum);
      add_relaxed(&c->p_rounds, (int64_t)1);
      const int64_t R2 = R - brk_sum;
      c->rec[nx].R = R2;
      c->rec[nx].start = brk + 1;
      c->rec[nx].done = (!filter || R2 == 0 || brk + 1 >= end) ? 1 : 0;
    }
  }
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// Compaction + accounting (single workgroup, right to left over [head, hi))
// ---------------------------------------------------------------------------
// slot >= 0: run only if the pass recorded in rec[slot] is done (lets the host
// enqueue compaction right after the window kernel without a round trip).
// The pass summary goes to `out` (host-mapped) either way.
__device__ void write_summary(DevCtl *c, const RoundRec &r, int done, PassSummary *out) {
  out->admitted = c->p_admitted;
  out->admitted_bytes = c->p_admitted_bytes;
  out->R0 = c->p_R0;
  out->R_after = r.R;
  out->rounds = c->p_rounds;
  out->start_final = r.start;
  out->hi = c->p_hi;
  out->head = c->head;
  out->tail = c->tail;
  out->used = c->used;
  out->adm_base = c->adm_base;
  out->done = done;
}

__global__ __launch_bounds__(CMP_THREADS) void k_compact(DevCtl *c, QueueArrays q, JobArrays jb,
                                                         int slot, PassSummary *out, int append) {
  if (slot >= 0 && !c->rec[slot].done) {
    if (threadIdx.x == 0 && out) write_summary(c, c->rec[slot], 0, out);
    return;
  }
  const int64_t mask = q.capacity - 1;
  __shared__ int64_t red[CMP_THREADS / WAVE];
  const int tid = threadIdx.x;
  const int64_t head = c->head, hi = c->p_hi;
  int64_t surv_hi = hi;
  const int64_t adm_base = c->adm_base;
  int64_t adm_hi = adm_base + c->p_admitted;
  for (int64_t chunk_hi = hi; chunk_hi > head; chunk_hi -= CMP_CHUNK) {
    const int64_t chunk_lo = chunk_hi - CMP_CHUNK > head ? chunk_hi - CMP_CHUNK : head;
    const int64_t p0 = chunk_lo + int64_t(tid) * CMP_ITEMS;
    int64_t d[CMP_ITEMS], sq[CMP_ITEMS];
    int32_t jo[CMP_ITEMS], pr[CMP_ITEMS];
    uint8_t adm[CMP_ITEMS], sur[CMP_ITEMS];
    int64_t a_loc = 0, s_loc = 0;
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k) {
      const int64_t p = p0 + k;
      const bool valid = p < chunk_hi;
      const int64_t pm = p & mask;
      d[k] = valid ? q.demand[pm] : -1;
      jo[k] = valid ? q.job[pm] : 0;
      pr[k] = valid ? q.prio[pm] : 0;
      sq[k] = valid ? q.seq[pm] : 0;
      const uint8_t de = valid ? q.decision[pm] : 0;
      adm[k] = valid && de == 1;
      sur[k] = valid && de != 1 && d[k] >= 0;
      a_loc += adm[k];
      s_loc += sur[k];
    }
    int64_t total;
    const int64_t ex = block_excl_scan<CMP_THREADS>((a_loc << 32) | s_loc, red, &total);
    const int64_t a_tot = total >> 32, s_tot = total & 0xffffffffLL;
    int64_t a_pos = adm_hi - a_tot + (ex >> 32);
    int64_t s_pos = surv_hi - s_tot + (ex & 0xffffffffLL);
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k) {
      const int64_t p = p0 + k;
      if (p >= chunk_hi) continue;
      q.decision[p & mask] = 0;
      if (adm[k]) {
        if (a_pos >= 0 && a_pos < q.capacity) {
          q.adm_job[a_pos] = jo[k];
          q.adm_demand[a_pos] = d[k];
          q.adm_seq[a_pos] = sq[k];
        }
        ++a_pos;
        add_relaxed(&jb.res[jo[k]], d[k]);
        jb.state[jo[k]] = 1;
      } else if (sur[k]) {
        const int64_t sm = s_pos & mask;
        q.demand[sm] = d[k];
        q.job[sm] = jo[k];
        q.prio[sm] = pr[k];
        q.seq[sm] = sq[k];
        ++s_pos;
      }
    }
    surv_hi -= s_tot;
    adm_hi -= a_tot;
  }
  __syncthreads();
  if (tid == 0) {
    c->head = surv_hi;
    c->used += c->p_admitted_bytes;
    if (out) {
      const RoundRec r = slot >= 0 ? c->rec[slot] : RoundRec{c->p_R0 - c->p_admitted_bytes, hi, 1, 0};
      write_summary(c, r, 1, out);
    }
    if (append) c->adm_base = adm_base + c->p_admitted;
  }
}

__global__ void k_release_masked(DevCtl *c, JobArrays jb, const uint8_t *__restrict__ mask,
                                 int64_t n) {
  __shared__ int64_t red[256 / WAVE];
  int64_t bytes = 0, cnt = 0;
  for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < n;
       j += int64_t(gridDim.x) * blockDim.x) {
    if (mask[j] && jb.state[j]) {
      bytes += jb.res[j];
      jb.res[j] = 0;
      jb.state[j] = 0;
      ++cnt;
    }
  }
  bytes = block_sum<256>(bytes, red);
  cnt = block_sum<256>(cnt, red);
  if (threadIdx.x == 0 && cnt) {
    add_relaxed(&c->used, -bytes);
    add_relaxed(&c->released_bytes, bytes);
    add_relaxed(&c->released_jobs, cnt);
  }
}

__global__ void k_enqueue(DevCtl *c, QueueArrays q, int64_t at, int64_t n, const int32_t *__restrict__ job,
                          const int64_t *__restrict__ demand, const int32_t *__restrict__ prio_of_job,
                          int64_t seq0) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t j = job[i];
    const int64_t pm = (at + i) & (q.capacity - 1);
    q.demand[pm] = demand[i];
    q.job[pm] = j;
    q.prio[pm] = prio_of_job[j];
    q.seq[pm] = seq0 + i;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) c->tail = at + n;
}

// ---------------------------------------------------------------------------
// Host drivers
// ---------------------------------------------------------------------------
static int grid_for(int64_t n, int threads, int cap) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  return int(g < cap ? g : cap);
}

int adm_engine_init(AdmEngine &e, int device, int64_t max_entries) {
  e.device = device;
  e.max_tiles = (max_entries + TILE - 1) / TILE + 1;
  SCHED_HIP_TRY(hipMalloc(&e.d_ctl, sizeof(DevCtl)));
  SCHED_HIP_TRY(hipMemset(e.d_ctl, 0, sizeof(DevCtl)));
  SCHED_HIP_TRY(hipHostMalloc(&e.h_ctl, sizeof(DevCtl), hipHostMallocDefault));
  memset(e.h_ctl, 0, sizeof(DevCtl));
  SCHED_HIP_TRY(hipHostMalloc(&e.h_sum, sizeof(PassSummary) * MAX_CHAIN, hipHostMallocMapped));
  memset(e.h_sum, 0, sizeof(PassSummary) * MAX_CHAIN);
  SCHED_HIP_TRY(hipHostGetDevicePointer((void **)&e.d_sum, e.h_sum, 0));
  SCHED_HIP_TRY(hipMalloc(&e.d_flags, sizeof(unsigned long long) * e.max_tiles));
  SCHED_HIP_TRY(hipMemset(e.d_flags, 0, sizeof(unsigned long long) * e.max_tiles));
  int cus = 0;
  SCHED_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  e.round_grid = cus * 8;
  e.launch = 1;
  e.epoch = 0;
  return SCHED_OK;
}

void adm_engine_free(AdmEngine &e) {
  if (e.d_ctl) (void)hipFree(e.d_ctl);
  if (e.h_ctl) (void)hipHostFree(e.h_ctl);
  if (e.d_flags) (void)hipFree(e.d_flags);
  if (e.h_sum) (void)hipHostFree(e.h_sum);
  e.h_sum = nullptr;
  e.d_sum = nullptr;
  e.d_ctl = nullptr;
  e.h_ctl = nullptr;
  e.d_flags = nullptr;
}

// Launch ids number the kernels of the pass chain consecutively: launch L
// reads slot L & 3 and prepares slot (L + 1) & 3.  Look-back flags carry a
// separate 16-bit epoch; the flag array is cleared whenever the epoch would
// repeat, so a look-back never reads a word written by an older round.
static uint32_t advance(AdmEngine &e) {
  e.launch += 1;
  return uint32_t(e.launch);
}
static int next_epoch(AdmEngine &e, hipStream_t s, uint32_t *ep) {
  if (e.epoch >= 65535) {
    k_fill_u64<<<grid_for(e.max_tiles, 256, 1024), 256, 0, s>>>(e.d_flags, e.max_tiles, 0ULL);
    SCHED_HIP_TRY(hipGetLastError());
    e.epoch = 0;
  }
  *ep = ++e.epoch;
  return SCHED_OK;
}

// Summary of the pass whose current state is in slot L & 3, into h_sum[0].
static int read_summary(AdmEngine &e, uint32_t L, hipStream_t s) {
  k_summary<<<1, 64, 0, s>>>(e.d_ctl, L, e.d_sum);
  SCHED_HIP_TRY(hipGetLastError());
  SCHED_HIP_TRY(hipStreamSynchronize(s));
  return SCHED_OK;
}

static void fill_out(const PassSummary &h, PassOut *out) {
  out->admitted = h.admitted;
  out->admitted_bytes = h.admitted_bytes;
  out->R0 = h.R0;
  out->R_after = h.R_after;
  out->rounds = h.rounds;
  out->start_final = h.start_final;
  out->hi = h.hi;
  out->head = h.head;
  out->tail = h.tail;
  out->used = h.used;
}

// Round kernels until the pass recorded in slot L & 3 is done; returns the
// launch id whose slot holds the final state.
static int run_rounds(AdmEngine &e, const int64_t *demand, uint8_t *decision, int64_t mask,
                      int64_t span_hint, hipStream_t s, uint32_t *Lio) {
  uint32_t L = *Lio;
  const int grid = grid_for(span_hint, TILE, e.round_grid);
  // every round decides at least one entry, so a pass needs at most
  // span + 1 rounds; anything beyond that is an internal error
  int64_t budget = span_hint + 2 * e.rounds_per_check + 2;
  for (;;) {
    if ((budget -= e.rounds_per_check) < 0) return SCHED_E_INTERNAL;
    for (int i = 0; i < e.rounds_per_check; ++i) {
      uint32_t ep;
      if (int rc = next_epoch(e, s, &ep)) return rc;
      SCHED_PROF_LAUNCH("k_round", s,
                        (k_round<<<grid, RND_THREADS, 0, s>>>(e.d_ctl, demand, decision, mask,
                                                              e.d_flags, L, ep)));
      SCHED_HIP_TRY(hipGetLastError());
      L = advance(e);
    }
    if (int rc = read_summary(e, L, s)) return rc;
    if (e.h_sum[0].done) break;
  }
  *Lio = L;
  return SCHED_OK;
}

static int launch_window(AdmEngine &e, const int64_t *demand, uint8_t *decision, int64_t mask,
                         int window_limit, int filter, int from_state, int64_t R0, int64_t start,
                         int64_t end, int append, hipStream_t s, uint32_t *Lio) {
  const uint32_t L = *Lio;
  SCHED_PROF_LAUNCH("k_window", s,
                    (k_window<<<1, WIN_THREADS, 0, s>>>(e.d_ctl, demand, decision, mask, L,
                                                        window_limit, 1, filter, from_state, R0,
                                                        start, end, append)));
  SCHED_HIP_TRY(hipGetLastError());
  *Lio = advance(e);
  return SCHED_OK;
}

int adm_scan(AdmEngine &e, int policy, const int64_t *demand, uint8_t *decision, int64_t start,
             int64_t end, int64_t R0, int window_limit, hipStream_t s, PassOut *out) {
  uint32_t L = uint32_t(e.launch);
  const int filter = policy == SCHED_POLICY_MMU ? 1 : 0;
  bool done = false;
  if (window_limit > 0) {
    if (int rc = launch_window(e, demand, decision, -1, window_limit, filter, 0, R0, start, end, 0,
                               s, &L))
      return rc;
    if (int rc = read_summary(e, L, s)) return rc;
    done = e.h_sum[0].done != 0;
  } else {
    k_prologue<<<1, 64, 0, s>>>(e.d_ctl, L, filter, 0, R0, start, end);
    SCHED_HIP_TRY(hipGetLastError());
  }
  if (!done)
    if (int rc = run_rounds(e, demand, decision, -1, end - start, s, &L)) return rc;
  fill_out(e.h_sum[0], out);
  return SCHED_OK;
}

int adm_pass_ctx(AdmEngine &e, int policy, const QueueArrays &q, const JobArrays &jb,
                 int window_limit, int64_t span_hint, hipStream_t s, PassOut *out) {
  uint32_t L = uint32_t(e.launch);
  const int filter = policy == SCHED_POLICY_MMU ? 1 : 0;
  const int64_t mask = q.capacity - 1;
  if (span_hint <= 0) span_hint = TILE;
  if (window_limit > 0) {
    if (int rc = launch_window(e, q.demand, q.decision, mask, window_limit, filter, 1, 0, 0, 0, 0,
                               s, &L))
      return rc;
    // compaction right behind the window kernel; it skips itself on the
    // device when the pass still needs grid rounds, and reports either way
    if (int rc = adm_compact(e, q, jb, s, int(L & 3), e.d_sum, 0)) return rc;
    SCHED_HIP_TRY(hipStreamSynchronize(s));
    if (e.h_sum[0].done) {
      fill_out(e.h_sum[0], out);
      return SCHED_OK;
    }
  } else {
    k_prologue<<<1, 64, 0, s>>>(e.d_ctl, L, filter, 1, 0, 0, 0);
    SCHED_HIP_TRY(hipGetLastError());
  }
  if (int rc = run_rounds(e, q.demand, q.decision, mask, span_hint, s, &L)) return rc;
  if (int rc = adm_compact(e, q, jb, s, int(L & 3), e.d_sum, 0)) return rc;
  SCHED_HIP_TRY(hipStreamSynchronize(s));
  fill_out(e.h_sum[0], out);
  return SCHED_OK;
}

int adm_chain(AdmEngine &e, int policy, const QueueArrays &q, const JobArrays &jb, int rounds,
              const uint8_t *masks, int64_t n_mask, hipStream_t s) {
  if (rounds <= 0 || rounds > MAX_CHAIN) return SCHED_E_INVALID;
  const int filter = policy == SCHED_POLICY_MMU ? 1 : 0;
  const int64_t mask = q.capacity - 1;
  uint32_t L = uint32_t(e.launch);
  for (int r = 0; r < rounds; ++r) {
    if (r > 0 && masks && n_mask > 0)
      if (int rc = adm_release_masked(e, jb, masks + int64_t(r - 1) * n_mask, n_mask, s)) return rc;
    // windows until the pass is done: one launch decides the whole pass
    if (int rc = launch_window(e, q.demand, q.decision, mask, 1 << 30, filter, 1, 0, 0, 0,
                               r > 0 ? 1 : 0, s, &L))
      return rc;
    if (int rc = adm_compact(e, q, jb, s, int(L & 3), e.d_sum + r, 1)) return rc;
  }
  SCHED_HIP_TRY(hipStreamSynchronize(s));
  return SCHED_OK;
}

int adm_compact(AdmEngine &e, const QueueArrays &q, const JobArrays &j, hipStream_t s, int slot,
                PassSummary *d_out, int append) {
  SCHED_PROF_LAUNCH("k_compact", s,
                    (k_compact<<<1, CMP_THREADS, 0, s>>>(e.d_ctl, q, j, slot, d_out, append)));
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int adm_release_masked(AdmEngine &e, const JobArrays &j, const uint8_t *mask, int64_t n,
                       hipStream_t s) {
  if (n <= 0) return SCHED_OK;
  SCHED_PROF_LAUNCH("k_release_masked", s,
                    (k_release_masked<<<grid_for(n, 256, 1024), 256, 0, s>>>(e.d_ctl, j, mask, n)));
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int adm_enqueue(AdmEngine &e, const QueueArrays &q, int64_t at, int64_t n, const int32_t *job,
                const int64_t *demand, const int32_t *prio_of_job, int64_t seq0, hipStream_t s) {
  k_enqueue<<<grid_for(n, 256, 4096), 256, 0, s>>>(e.d_ctl, q, at, n, job, demand, prio_of_job, seq0);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int adm_zero_decisions(uint8_t *decision, int64_t n, hipStream_t s) {
  if (n <= 0) return SCHED_OK;
  k_fill_u8<<<grid_for(n, 256, 4096), 256, 0, s>>>(decision, n, 0);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

}  // namespace schedk
