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
//  * k_window: one wave walks the queue in windows of 256 entries and runs
//    all rounds of a window in registers.  This is the latency regime: when
//    free memory runs out after a few thousand entries the whole pass is one
//    launch.
//  * k_round: a persistent grid that computes one round over the whole
//    remaining queue with a single-pass decoupled look-back scan.  Tiles are
//    dealt to the workgroups in an interleaved static order (workgroup b
//    takes tiles b, b + G, b + 2G, ...), so the grid streams one contiguous
//    stretch of the queue at a time; each tile publishes its candidate sum
//    (saturated at R + 1) and then its inclusive prefix in one 64-bit word
//    (epoch:16 | status:2 | value:46).  A look-back polls a missing
//    predecessor a bounded number of times and then sums that predecessor's
//    candidates from its demands itself, so no workgroup ever depends on
//    another one being resident.  Only the tile that holds
//    the break runs an ordered scan; every other tile either admits all of
//    its candidates or, lying past the break, admits nothing.  This is the
//    HBM-bound regime (the final round of a pass that never exhausts memory
//    reads every remaining demand once).
#include <atomic>
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

// The launch that follows L uses slot (L + 1) & 3: clear its break marker and
// counters.  Launch L - 3 was the last user of that slot and has finished.
__device__ __forceinline__ void reset_next_slot(DevCtl *c, uint32_t L) {
  const int nx = (L + 1) & 3;
  c->break_tile[nx] = LLONG_MAX;
  c->tiles_done[nx] = 0;
  c->round_sum[nx] = 0;
}

// Called once per workgroup when it leaves a round, with the candidate sum of
// the tiles it decided.  In a round without a break every decided tile
// admitted all of its candidates, so the round's admitted sum is the sum of
// those candidate sums; the workgroup that leaves last closes the round.
// (With a break, the break tile closes it instead.)  Workgroups accumulate
// over all their tiles so that these counters see one update per workgroup,
// not one per tile.
// The last workgroup only reads values other workgroups changed with device
// atomics (round_sum, break_tile); each workgroup waits for its own atomics
// to complete before it counts itself out, so those values are final when
// the count is.  No release/acquire is needed (at device scope that would
// write back the whole L2 of the workgroup's XCD once per workgroup); plain
// stores (decisions, records) are only read after the kernel ends.
// The pass summary after a round, into host-mapped memory (thread 0 of the
// workgroup that closes the round; the totals are read atomically, the
// scheduler state was written by earlier launches).
__device__ __forceinline__ void round_summary(DevCtl *c, int64_t R_after, int64_t start_final,
                                              int32_t done, PassSummary *out) {
  out->admitted = ld_relaxed(&c->p_admitted);
  out->admitted_bytes = ld_relaxed(&c->p_admitted_bytes);
  out->R0 = c->p_R0;
  out->R_after = R_after;
  out->rounds = ld_relaxed(&c->p_rounds);
  out->start_final = start_final;
  out->hi = ld_relaxed(&c->p_hi);
  out->head = c->head;
  out->tail = c->tail;
  out->used = c->used;
  out->adm_base = c->adm_base;
  out->done = done;
}

__device__ __forceinline__ void block_done(DevCtl *c, int s, int nx, int64_t a, int64_t R,
                                           int64_t end, unsigned n_blocks, PassSummary *out) {
  if (a) add_relaxed(&c->round_sum[s], (unsigned long long)a);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  const unsigned long long prev = add_relaxed(&c->tiles_done[s], 1ULL);
  if (prev + 1 != (unsigned long long)n_blocks) return;
  if (ld_relaxed(&c->break_tile[s]) != LLONG_MAX) {
    // the break tile wrote the next start state (atomically) before it
    // counted itself out
    round_summary(c, ld_relaxed(&c->rec[nx].R), ld_relaxed(&c->rec[nx].start),
                  ld_relaxed(&c->rec[nx].done), out);
    return;
  }
  const int64_t sum = int64_t(ld_relaxed(&c->round_sum[s]));
  add_relaxed(&c->p_admitted_bytes, sum);
  add_relaxed(&c->p_rounds, (int64_t)1);
  c->rec[nx].R = R - sum;
  c->rec[nx].start = end;
  c->rec[nx].done = 1;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  round_summary(c, R - sum, end, 1, out);
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


// ---------------------------------------------------------------------------
// Single-wave windowed rounds
// ---------------------------------------------------------------------------
// One wave walks the queue in windows of WIN entries; lane l holds the WIN_ITEMS
// consecutive entries starting at l * WIN_ITEMS, so a lane-local running sum
// plus one wave-wide exclusive scan gives every entry its prefix in queue
// order.  The break of a round is the lowest set bit of a ballot.  No LDS and
// no barriers.
// Sums need no saturation: a candidate's demand is clamped to R + 1 (only
// FIFO, which does not filter, sees larger ones), so a window's sum stays
// below 2^54, and a prefix exceeds R exactly when the unclamped one does.
// A round only updates a per-lane bit mask of admitted items; decisions,
// counts and the highest admitted position are written once per window, and
// the next window's demands are loaded while the current one is decided.
// init != 0: the kernel also does the prologue (pass start state from the
// arguments or, with from_state, from the control block).
__device__ __forceinline__ void window_load(const int64_t *__restrict__ demand, int64_t mask,
                                            int64_t p0, int64_t end, int64_t (&x)[WIN_ITEMS]) {
#pragma unroll
  for (int k = 0; k < WIN_ITEMS; ++k) x[k] = (p0 + k < end) ? demand[(p0 + k) & mask] : -1;
}

// Decides one window [wpos, wpos + WIN) of a pass: first-fit rounds until the
// window is exhausted or the pass ends inside it; updates the pass state.
// Returns whether the window held any candidate.
__device__ __forceinline__ bool decide_window(const int64_t (&x)[WIN_ITEMS], const int64_t wpos,
                                              const int base, const int64_t end,
                                              const int64_t mask, const bool filter,
                                              uint8_t *__restrict__ decision, int64_t &R,
                                              int &done, int64_t &hi, int64_t &adm_cnt,
                                              int64_t &adm_bytes, int64_t &rounds, int64_t &pos) {
  uint32_t abits = 0;
  int s_loc = 0, lim = WIN;
  bool any_cand = false;
  for (;;) {
    int kb = WIN_ITEMS;      // this lane's break item
    int64_t before = 0;      // prefix just before it
    int64_t total;           // the window's candidate total (exact when no lane breaks)
    uint32_t a = 0;          // this lane's items admitted by the round
    bool mine = false;       // this lane holds a candidate
    if (R < int64_t(0xffffffff)) {
      // R + 1 fits in 32 bits: candidates are clamped to it and prefixes
      // saturate at 2^32 - 1, which keeps every prefix up to R + 1 exact and
      // every larger one above R -- all the round's tests need.  After a
      // pass's first break R is below that break's demand, so this is the
      // common case.
      const uint32_t R32 = uint32_t(R), cap32 = R32 + 1;
      uint32_t v[WIN_ITEMS], rex[WIN_ITEMS];
      bool cd[WIN_ITEMS];
      uint32_t run = 0;
#pragma unroll
      for (int k = 0; k < WIN_ITEMS; ++k) {
        cd[k] = x[k] >= 0 && base + k >= s_loc && (!filter || x[k] <= R);
        v[k] = cd[k] ? (x[k] < int64_t(cap32) ? uint32_t(x[k]) : cap32) : 0u;
        rex[k] = run;
        run = add_sat_u32(run, v[k]);
        mine = mine || cd[k];
      }
      const uint32_t wincl = wave_incl_scan_sat32_dpp(run);
      const uint32_t ex = wave_prev_lane32(wincl);
      total = int64_t(uint32_t(__builtin_amdgcn_readlane(int(wincl), WAVE - 1)));
#pragma unroll
      for (int k = WIN_ITEMS - 1; k >= 0; --k) {
        const uint32_t exk = add_sat_u32(ex, rex[k]);
        const uint32_t inc = add_sat_u32(exk, v[k]);
        if (cd[k] && inc > R32) {
          kb = k;
          before = int64_t(exk);  // the break's exclusive prefix is <= R, hence exact
        }
        if (cd[k] && inc <= R32) a |= 1u << k;
      }
    } else {
      const int64_t cap = R + 1;
      int64_t v[WIN_ITEMS], r[WIN_ITEMS];
      int64_t run = 0;
#pragma unroll
      for (int k = 0; k < WIN_ITEMS; ++k) {
        const bool cd = x[k] >= 0 && base + k >= s_loc && (!filter || x[k] <= R);
        v[k] = cd ? (x[k] < cap ? x[k] : cap) : 0;
        run += v[k];
        r[k] = cd ? run : -1;  // -1 marks a non-candidate
        mine = mine || cd;
      }
      const int64_t wincl = wave_incl_scan_dpp(run);
      const int64_t ex = wave_prev_lane64(wincl);
      total = read_lane64(wincl, WAVE - 1);
#pragma unroll
      for (int k = WIN_ITEMS - 1; k >= 0; --k) {
        const int64_t inc = ex + r[k];
        if (r[k] >= 0 && inc > R) {
          kb = k;
          before = inc - v[k];
        }
        if (r[k] >= 0 && inc <= R) a |= 1u << k;
      }
    }
    if (!any_cand) any_cand = __ballot(mine) != 0;
    abits |= a;
    const uint64_t ball = __ballot(kb < WIN_ITEMS);
    int first = WIN;
    int64_t sum = total;
    if (ball) {
      const int fl = __builtin_ctzll(ball);
      first = fl * WIN_ITEMS + __builtin_amdgcn_readlane(kb, fl);
      sum = read_lane64(before, fl);
    }
    R -= sum;
    adm_bytes += sum;
    ++rounds;
    if (first >= WIN) break;
    if (!filter || R == 0) {
      done = 1;
      lim = first + 1;
      break;
    }
    s_loc = first + 1;
    if (s_loc >= WIN) break;
  }
  // the window's decided entries [0, lim)
#pragma unroll
  for (int k = 0; k < WIN_ITEMS; ++k) {
    const int64_t p = wpos + base + k;
    if (base + k < lim && p < end) decision[p & mask] = uint8_t((abits >> k) & 1u);
    adm_cnt += __builtin_popcountll(__ballot((abits >> k) & 1u));
  }
  const uint64_t lb = __ballot(abits != 0);
  if (lb) {
    const int hl = 63 - __builtin_clzll(lb);
    const uint32_t hb = uint32_t(__builtin_amdgcn_readlane(int(abits), hl));
    const int64_t mx = wpos + int64_t(hl) * WIN_ITEMS + (31 - __builtin_clz(hb));
    if (mx + 1 > hi) hi = mx + 1;
  }
  pos = done ? wpos + lim : wpos + WIN;
  return any_cand;
}

// Results of a window walk, handed to the rest of a workgroup through LDS.
struct WinResult {
  int64_t R, start, admitted, admitted_bytes, hi, rounds;
  int32_t done, pad;
};

// The window walk, run by one whole wave (lane = its lane index).
__device__ __forceinline__ void window_pass(DevCtl *c, const int64_t *__restrict__ demand,
                                            uint8_t *__restrict__ decision, int64_t mask, uint32_t L,
                                            int max_windows, int init, int filter_arg,
                                            int from_state, int64_t R0, int64_t start0,
                                            int64_t end0, int append, int lane,
                                            WinResult *wr = nullptr,
                                            const int64_t *pre = nullptr, int empty_exit = 0) {
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
  if (lane == 0 && !wr) reset_next_slot(c, L);
  int64_t adm_cnt = 0, adm_bytes = 0, rounds = 0;
  const int base = lane * WIN_ITEMS;
  // windows are contiguous (a window either completes, and the next one
  // starts WIN entries later, or ends the pass), so window w + WIN_PF can be
  // loaded as soon as window w is decided: WIN_PF - 1 windows stay in flight
  int64_t x[WIN_PF][WIN_ITEMS];
  if (pre) {
    // the caller loaded this lane's entries of the first WIN_PF windows
#pragma unroll
    for (int u = 0; u < WIN_PF; ++u)
#pragma unroll
      for (int k = 0; k < WIN_ITEMS; ++k) x[u][k] = pre[u * WIN_ITEMS + k];
  } else if (!done) {
#pragma unroll
    for (int u = 0; u < WIN_PF; ++u) window_load(demand, mask, pos + u * WIN + base, end, x[u]);
  }
  // empty_exit > 0: stop (leaving the rest to the grid rounds) after that
  // many consecutive windows without a single candidate; free memory is then
  // below every demand seen, and a candidate-free stretch is the grid
  // kernel's streaming case
  int w = 0, empty_run = 0;
  while (w < max_windows && !done) {
#pragma unroll
    for (int u = 0; u < WIN_PF; ++u) {
      if (w >= max_windows || done) break;
      if (pos >= end || R == 0) {
        done = 1;
        break;
      }
      const int64_t wpos = pos;
      const bool cand = decide_window(x[u], wpos, base, end, mask, filter, decision, R, done, hi,
                                      adm_cnt, adm_bytes, rounds, pos);
      empty_run = cand ? 0 : empty_run + 1;
      if (empty_exit > 0 && empty_run >= empty_exit) max_windows = w + 1;
      if (!done && w + WIN_PF < max_windows)
        window_load(demand, mask, wpos + WIN_PF * WIN + base, end, x[u]);
      ++w;
    }
  }
  if (!done && (pos >= end || R == 0)) done = 1;
  if (lane == 0 && !wr) {
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
  if (lane == 0 && wr) {
    wr->R = R;
    wr->start = pos < end ? pos : end;
    wr->done = done;
    wr->admitted = adm_cnt;
    wr->admitted_bytes = adm_bytes;
    wr->hi = hi;
    wr->rounds = rounds;
  }
}

__global__ __launch_bounds__(WIN_THREADS) void k_window(DevCtl *c, const int64_t *__restrict__ demand,
                                                        uint8_t *__restrict__ decision, int64_t mask,
                                                        uint32_t L, int max_windows, int init,
                                                        int filter_arg, int from_state, int64_t R0,
                                                        int64_t start0, int64_t end0, int append,
                                                        int empty_exit) {
  window_pass(c, demand, decision, mask, L, max_windows, init, filter_arg, from_state, R0, start0,
              end0, append, threadIdx.x, nullptr, nullptr, empty_exit);
}

// ---------------------------------------------------------------------------
// Grid-wide round with decoupled look-back
// ---------------------------------------------------------------------------
// Loads tile t's demands (raw; -1 past the end) without using them, so a
// prefetch does not wait for the data.
__device__ __forceinline__ void round_load(const int64_t *__restrict__ demand, int64_t mask,
                                           int64_t base, int64_t end, int64_t (&x)[RND_ITEMS]) {
#pragma unroll
  for (int j = 0; j < RND_ITEMS; ++j) {
    const int64_t p = base + int64_t(j) * RND_THREADS + threadIdx.x;
    x[j] = p < end ? __builtin_nontemporal_load(demand + (p & mask)) : -1;
  }
}

// A tile of a round is handled in two steps.  round_reduce takes its
// candidates (bit j of the returned mask: this thread's item j) and their
// sum, and publishes the sum at once for the tiles after it (tile 0, whose
// prefix is 0, publishes it as inclusive).  round_finish then looks back for
// the tile's exclusive prefix and decides it.  The round loop reduces a
// workgroup's next tile before it finishes the current one, so a tile's sum
// is out before the look-back of the tile before it has ended: the tiles
// after it find it instead of waiting for it.
// Candidates are clamped to cap = R + 1 (only FIFO, which does not filter,
// sees larger ones): a prefix exceeds R exactly when the unclamped one does,
// and every sum below stays under 2^59, so no addition can wrap whatever the
// int64 demands are.
__device__ __forceinline__ uint32_t round_reduce(unsigned long long *flags, uint32_t epoch,
                                                 long long t, int64_t R, int64_t cap, bool filter,
                                                 const int64_t (&raw)[RND_ITEMS], int64_t *red,
                                                 int64_t &Araw) {
  uint32_t cm = 0;
  int64_t tsum = 0;
#pragma unroll
  for (int j = 0; j < RND_ITEMS; ++j) {
    const int64_t v = raw[j];
    const bool cd = v >= 0 && (!filter || v <= R);
    tsum += cd ? (v < cap ? v : cap) : 0;
    cm |= uint32_t(cd) << j;
  }
  Araw = block_sum<RND_THREADS>(tsum, red);
  const int64_t A = Araw < cap ? Araw : cap;
  if (threadIdx.x == 0) st_relaxed(&flags[t], pack_flag(epoch, t == 0 ? FL_INC : FL_AGG, A));
  return cm;
}

// The second step of tile t (whole workgroup): cm and Araw from
// round_reduce.  Returns true when the tile lies past the round's break (so
// does every later tile).
__device__ __forceinline__ bool round_finish(DevCtl *c, const int64_t *__restrict__ demand,
                                             uint8_t *__restrict__ decision, int64_t mask,
                                             unsigned long long *flags, int s, int nx,
                                             uint32_t epoch, int32_t polls, int64_t R, int64_t cap,
                                             bool filter, int64_t start, int64_t end, long long t,
                                             int64_t base, uint32_t cm, int64_t Araw, int64_t *red,
                                             int64_t &s_E, int64_t &s_brk_sum, int64_t &acc_sum,
                                             int64_t &acc_cnt, int64_t &acc_hi) {
  const int tid = threadIdx.x;
  const int64_t A = Araw < cap ? Araw : cap;
  if (Araw == 0) {
    // No candidate in this tile: every entry is rejected whatever the
    // prefix before it is, so the tile needs no look-back (its zero sum is
    // published already).
#pragma unroll
    for (int j = 0; j < RND_ITEMS; ++j) {
      const int64_t p = base + int64_t(j) * RND_THREADS + tid;
      if (p < end) decision[p & mask] = 0;
    }
    return false;
  }

  if (tid < WAVE) {
    // Wave 0 looks back 64 predecessors at a time: lane l reads the flag of
    // tile p - l.  The nearest inclusive flag ends the walk once every
    // nearer predecessor has published its aggregate.  A predecessor still
    // missing after `polls` polls has its aggregate computed here from its
    // demands (lane l then holds it in `own`), so the walk never depends on
    // the workgroup that owns that tile having started.
    const int lane = tid;
    int64_t E = 0;
    if (t != 0) {
      long long p = t - 1;
      int32_t waited = 0;
      bool has_own = false;
      int64_t own = 0;
      for (;;) {
        const long long qq = p - lane;
        const unsigned long long f =
            qq >= 0 ? ld_relaxed(&flags[qq]) : pack_flag(epoch, FL_INC, 0);
        uint64_t st = (f >> 46) & 3;
        bool valid = uint32_t(f >> 48) == epoch && st != 0;
        int64_t fv = int64_t(f & VMASK);
        if (!valid && has_own) {
          valid = true;
          st = FL_AGG;
          fv = own;
        }
        const uint64_t inc_b = __ballot(valid && st == FL_INC);
        const uint64_t bad_b = __ballot(!valid);
        const int fi = inc_b ? __builtin_ctzll(inc_b) : WAVE;
        const uint64_t need = fi >= WAVE - 1 ? ~0ULL : ((2ULL << fi) - 1);
        if (bad_b & need) {
          // a predecessor that saw the break marker first may never publish
          // (the marker is read once for the whole wave)
          const long long bt = ld_relaxed(&c->break_tile[s]);
          const long long btw = (long long)(((unsigned long long)__builtin_amdgcn_readfirstlane(
                                                 int(uint64_t(bt) >> 32)) << 32) |
                                            uint32_t(__builtin_amdgcn_readfirstlane(int(bt))));
          if (btw < t) {
            E = cap;
            break;
          }
          if (waited < polls) {
            ++waited;
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          // the nearest missing predecessor: sum its candidates (every
          // lane with qq < 0 is valid, so q >= 0; q < t < n_tiles)
          const int b = __builtin_ctzll(bad_b & need);
          const int64_t qbase = start + int64_t(p - b) * TILE;
          int64_t part = 0;
          for (int k = 0; k < TILE / WAVE; ++k) {
            const int64_t pos = qbase + int64_t(k) * WAVE + lane;
            if (pos < end) {
              const int64_t v = demand[pos & mask];
              if (v >= 0 && (!filter || v <= R)) part = sat_add(part, v < cap ? v : cap, cap);
            }
          }
          const int64_t agg = wave_sum(part);  // <= 64 * cap, no overflow
          if (lane == b) {
            has_own = true;
            own = agg < cap ? agg : cap;
          }
          waited = 0;
          continue;
        }
        const int64_t v = lane <= fi ? fv : 0;
        const int64_t w = wave_sum(v);  // <= 64 * cap, no overflow
        E = sat_add(E, w < cap ? w : cap, cap);
        if (fi < WAVE || E >= cap) break;
        p -= WAVE;
        has_own = false;
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
  if (E > R) return true;  // the break lies in an earlier tile, which closes the round

  int64_t tcnt = 0, tmax = -1;
  if (sat_add(E, A, cap) <= R) {
    // every candidate of this tile is admitted
#pragma unroll
    for (int j = 0; j < RND_ITEMS; ++j) {
      const int64_t p = base + int64_t(j) * RND_THREADS + tid;
      if (p < end) {
        const bool a = (cm >> j) & 1u;
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
      acc_cnt += cnt;
      if (mx + 1 > acc_hi) acc_hi = mx + 1;
      acc_sum += A;  // exact here: E + A <= R
    }
    return false;
  }

  // The break lies in this tile (one tile per round): its demands are read
  // again, the candidates being those round_reduce took.
  int64_t x[RND_ITEMS];
#pragma unroll
  for (int j = 0; j < RND_ITEMS; ++j) {
    const int64_t p = base + int64_t(j) * RND_THREADS + tid;
    const int64_t v = ((cm >> j) & 1u) ? demand[p & mask] : int64_t(-1);
    x[j] = v >= 0 ? (v < cap ? v : cap) : -1;
  }
  // scan it row by row in queue order
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
    st_relaxed(&c->rec[nx].R, R2);
    st_relaxed(&c->rec[nx].start, brk + 1);
    st_relaxed(&c->rec[nx].done, int32_t((!filter || R2 == 0 || brk + 1 >= end) ? 1 : 0));
  }
  return false;
}

// Workgroup b of G decides tiles b, b + G, b + 2G, ... in that order.  One
// data buffer serves the whole sequence: at each step the next tile (already
// loaded) is reduced, the buffer is refilled with the tile after it, and
// only then is the current tile finished, so the refill lands while the
// current tile looks back and its decisions are written.  The sequence
// stops at the end of the queue or past the round's break (the marker is
// read by one thread before a tile is finished and shared through LDS after
// it; a marker set meanwhile is seen one tile later, and a tile past the
// break finds that out in its look-back).  Words handed over through LDS
// alternate by step parity: a word is written again only two steps on,
// after a barrier every wave has passed.
// Four workgroups per CU (at most 128 registers per lane): with one data
// buffer per workgroup, the fourth keeps as many loads in flight as three
// workgroups with two buffers did.
__global__ __launch_bounds__(RND_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_round(DevCtl *c, const int64_t *__restrict__ demand,
                                                       uint8_t *__restrict__ decision, int64_t mask,
                                                       unsigned long long *flags, uint32_t L,
                                                       uint32_t epoch, int32_t polls,
                                                       PassSummary *out) {
  __shared__ int64_t red[RND_THREADS / WAVE];
  __shared__ long long s_bt[2];
  __shared__ int64_t s_E;
  __shared__ int64_t s_brk_sum;
  const int tid = threadIdx.x;
  const int s = L & 3, nx = (L + 1) & 3;
  const RoundRec r = c->rec[s];
  if (blockIdx.x == 0 && tid == 0) {
    reset_next_slot(c, L);
    if (r.done) {
      c->rec[nx] = r;
      round_summary(c, r.R, r.start, 1, out);
    }
  }
  if (r.done) return;
  const int64_t R = r.R, start = r.start, end = c->p_end;
  const int64_t cap = R + 1;
  const bool filter = c->filter != 0;
  const long long n_tiles = (end - start + TILE - 1) / TILE;
  const long long G = gridDim.x;
  // thread 0's totals over the whole tiles this workgroup decided
  int64_t acc_sum = 0, acc_cnt = 0, acc_hi = -1;

  long long t = (long long)blockIdx.x < n_tiles ? (long long)blockIdx.x : -1;
  int64_t x[RND_ITEMS];
  uint32_t cm = 0;
  int64_t Araw = 0;
  if (t >= 0) {
    round_load(demand, mask, start + int64_t(t) * TILE, end, x);
    cm = round_reduce(flags, epoch, t, R, cap, filter, x, red, Araw);
  }
  long long tn = t >= 0 && t + G < n_tiles ? t + G : -1;
  if (tn >= 0) round_load(demand, mask, start + int64_t(tn) * TILE, end, x);
  int par = 0;
  while (t >= 0) {
    long long bt = LLONG_MAX;
    if (tid == 0) bt = ld_relaxed(&c->break_tile[s]);
    // the next tile: reduced (its sum published) before this one finishes
    uint32_t cm_n = 0;
    int64_t Araw_n = 0;
    long long tnn = -1;
    if (tn >= 0) {
      cm_n = round_reduce(flags, epoch, tn, R, cap, filter, x, red, Araw_n);
      tnn = tn + G < n_tiles ? tn + G : -1;
      if (tnn >= 0) round_load(demand, mask, start + int64_t(tnn) * TILE, end, x);
    }
    if (round_finish(c, demand, decision, mask, flags, s, nx, epoch, polls, R, cap, filter, start,
                     end, t, start + int64_t(t) * TILE, cm, Araw, red, s_E, s_brk_sum, acc_sum,
                     acc_cnt, acc_hi))
      break;
    if (tid == 0) s_bt[par] = bt;
    __syncthreads();
    if (tn < 0 || tn > s_bt[par]) break;
    par ^= 1;
    t = tn;
    cm = cm_n;
    Araw = Araw_n;
    tn = tnn;
  }
  if (tid == 0) {
    if (acc_cnt) {
      add_relaxed(&c->p_admitted, acc_cnt);
      max_relaxed(&c->p_hi, acc_hi);
    }
    block_done(c, s, nx, acc_sum, R, end, gridDim.x, out);
  }
}

// ---------------------------------------------------------------------------
// Split round: the same round in three launches, without look-back
// ---------------------------------------------------------------------------
// For the stateless scan, whose workspace the library owns, a round can be
// taken apart: k_split_reduce reads every tile once and keeps its candidate
// sum and candidate bits (1 bit per entry), k_split_scan (one workgroup) scans
// the tile sums, finds the break and decides the break tile row by row, and
// k_split_write writes the decision bytes of the tiles up to the break from
// the bits.  No tile waits for another, and the demands are read in one
// launch and the decisions written in another.  The round's record, slot and
// summary protocol is k_round's: it reads rec[L & 3], writes rec[(L + 1) & 3],
// and the last workgroup of k_split_write writes the pass summary.
// It pays where k_round's look-back does not: in a FIFO pass whose tiles all
// hold candidates (2^26 entries admitted whole: ~149 us against ~190 us per
// call).  Where most tiles hold none (a first-fit round after the walk) the
// three launches cost more than k_round's one (~149 us against ~133 us), so
// only FIFO scans use it; the kernels take either policy.

// Candidate sums (clamped to cap) and candidate bits of every tile of the
// round; bit o of a tile's 64 words is the tile's entry o (queue order), so
// the write pass can turn 16 bits into 16 contiguous decision bytes.  Two
// data buffers: a tile's loads are in flight while the tile before it is
// reduced.
constexpr int SPLIT_WORDS = TILE / 64;  // candidate-bit words per tile

__device__ __forceinline__ void split_tile(long long t, int64_t R, int64_t cap, bool filter,
                                           const int64_t (&x)[RND_ITEMS], int64_t *red,
                                           int64_t *__restrict__ agg,
                                           unsigned long long *__restrict__ bits) {
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  int64_t tsum = 0;
  unsigned long long mine = 0;
#pragma unroll
  for (int j = 0; j < RND_ITEMS; ++j) {
    const int64_t v = x[j];
    const bool cd = v >= 0 && (!filter || v <= R);
    tsum += cd ? (v < cap ? v : cap) : 0;  // <= 16 * cap: no overflow
    // row j of the tile: entries j * RND_THREADS + tid, this wave's 64 of
    // them one word; lane j keeps it
    const unsigned long long m = __ballot(cd);
    if (lane == j) mine = m;
  }
  if (lane < RND_ITEMS) bits[t * SPLIT_WORDS + lane * (RND_THREADS / WAVE) + w] = mine;
  const int64_t A = block_sum<RND_THREADS>(tsum, red);  // <= TILE * cap < 2^59
  if (tid == 0) agg[t] = A < cap ? A : cap;
}

__global__ __launch_bounds__(RND_THREADS) void k_split_reduce(const DevCtl *c,
                                                              const int64_t *__restrict__ demand,
                                                              int64_t mask, uint32_t L,
                                                              int64_t *__restrict__ agg,
                                                              unsigned long long *__restrict__ bits) {
  __shared__ int64_t red[RND_THREADS / WAVE];
  const RoundRec r = c->rec[L & 3];
  if (r.done) return;
  const int64_t R = r.R, start = r.start, end = c->p_end;
  const int64_t cap = R + 1;
  const bool filter = c->filter != 0;
  const long long n_tiles = (end - start + TILE - 1) / TILE;
  const long long G = gridDim.x;
  long long t = blockIdx.x;
  if (t >= n_tiles) return;
  int64_t xa[RND_ITEMS], xb[RND_ITEMS];
  round_load(demand, mask, start + int64_t(t) * TILE, end, xa);
  for (;;) {
    long long tn = t + G;
    if (tn < n_tiles) round_load(demand, mask, start + int64_t(tn) * TILE, end, xb);
    split_tile(t, R, cap, filter, xa, red, agg, bits);
    if (tn >= n_tiles) break;
    t = tn;
    tn = t + G;
    if (tn < n_tiles) round_load(demand, mask, start + int64_t(tn) * TILE, end, xa);
    split_tile(t, R, cap, filter, xb, red, agg, bits);
    if (tn >= n_tiles) break;
    t = tn;
  }
}

// Where a split round breaks (written by k_split_scan for k_split_write).
struct SplitBreak {
  int64_t tile;  // tiles before it admit all their candidates; n_tiles: no break
  int64_t pos;   // the break entry (queue position); decisions are written up to it
};

constexpr int SPLIT_SCAN_THREADS = 1024;
constexpr int SPLIT_BATCH = 16;  // tile sums a thread loads at once

__global__ __launch_bounds__(SPLIT_SCAN_THREADS) void k_split_scan(
    DevCtl *c, const int64_t *__restrict__ demand, int64_t mask, uint32_t L,
    const int64_t *__restrict__ agg, SplitBreak *brk_out, PassSummary *out) {
  constexpr int NT = SPLIT_SCAN_THREADS;
  __shared__ int64_t red[NT / WAVE];
  __shared__ int64_t s_b, s_E, s_brk, s_brk_sum;
  const int tid = threadIdx.x;
  const int s = L & 3, nx = (L + 1) & 3;
  const RoundRec r = c->rec[s];
  if (tid == 0) reset_next_slot(c, L);
  if (r.done) {
    if (tid == 0) {
      c->rec[nx] = r;
      round_summary(c, r.R, r.start, 1, out);
    }
    return;
  }
  const int64_t R = r.R, start = r.start, end = c->p_end;
  const int64_t cap = R + 1;
  const bool filter = c->filter != 0;
  const long long n_tiles = (end - start + TILE - 1) / TILE;
  // each thread sums a contiguous run of tile sums (loaded a batch at a
  // time); one exclusive scan over the runs; the run holding the first tile
  // whose inclusive prefix exceeds R walks its tiles to find it
  const long long per = (n_tiles + NT - 1) / NT;
  const long long lo = (long long)tid * per;
  const long long hi = lo + per < n_tiles ? lo + per : n_tiles;
  int64_t run = 0;
  for (long long k0 = lo; k0 < hi; k0 += SPLIT_BATCH) {
    int64_t v[SPLIT_BATCH];
#pragma unroll
    for (int u = 0; u < SPLIT_BATCH; ++u) v[u] = k0 + u < hi ? agg[k0 + u] : 0;
#pragma unroll
    for (int u = 0; u < SPLIT_BATCH; ++u) run = sat_add(run, v[u], cap);
  }
  int64_t total;
  const int64_t before = block_excl_scan_sat<NT>(run, cap, red, &total);
  // the run that crosses R (one at most), then the tile in it: the run's
  // tile sums are loaded by one thread each and scanned together
  const bool crosses = before <= R && sat_add(before, run, cap) > R;
  const int64_t fr = block_min<NT>(crosses ? tid : NT, red);
  if (tid == fr) s_E = before;
  __syncthreads();
  long long b = n_tiles;
  if (fr < NT) {
    const long long flo = fr * per;
    const long long fhi = flo + per < n_tiles ? flo + per : n_tiles;
    const int64_t a = flo + tid < fhi ? agg[flo + tid] : 0;  // per <= NT (checked on the host)
    int64_t unused;
    const int64_t e = sat_add(s_E, block_excl_scan_sat<NT>(a, cap, red, &unused), cap);
    const int64_t fi = block_min<NT>(flo + tid < fhi && e <= R && sat_add(e, a, cap) > R ? tid : NT,
                                     red);
    if (tid == fi) s_E = e;
    __syncthreads();
    b = flo + fi;  // the run's inclusive prefix exceeds R, so fi < NT
  }
  int64_t brk, brk_sum;
  if (b == n_tiles) {
    // no break: every candidate up to the end is admitted
    brk = end;
    brk_sum = total;  // <= R
  } else {
    // decide the break tile row by row in queue order (the candidates are
    // those k_split_reduce took); its inclusive prefix exceeds R, so some row
    // holds the break
    const int64_t base = start + int64_t(b) * TILE;
    int64_t carry = s_E;
    brk = end;
    brk_sum = 0;
    for (int j = 0; j < TILE / NT; ++j) {
      const int64_t p = base + int64_t(j) * NT + tid;
      int64_t v = p < end ? demand[p & mask] : int64_t(-1);
      const bool cd = v >= 0 && (!filter || v <= R);
      v = cd ? (v < cap ? v : cap) : 0;
      int64_t rowtot;
      const int64_t ex = block_excl_scan_sat<NT>(v, cap, red, &rowtot);
      const int64_t P = sat_add(carry, sat_add(ex, v, cap), cap);
      const int64_t f = block_min<NT>(cd && P > R ? tid : NT, red);
      if (f < NT) {
        if (tid == f) {
          s_brk = p;
          s_brk_sum = sat_add(carry, ex, cap);
        }
        __syncthreads();
        brk = s_brk;
        brk_sum = s_brk_sum;
        break;
      }
      carry = sat_add(carry, rowtot, cap);
    }
  }
  if (tid == 0) {
    add_relaxed(&c->p_admitted_bytes, brk_sum);
    add_relaxed(&c->p_rounds, (int64_t)1);
    const int64_t R2 = R - brk_sum;
    const int64_t nstart = b == n_tiles ? end : brk + 1;
    c->rec[nx].R = R2;
    c->rec[nx].start = nstart;
    c->rec[nx].done = int32_t((!filter || R2 == 0 || nstart >= end) ? 1 : 0);
    brk_out->tile = b;
    brk_out->pos = brk;
  }
}

// Decision bytes of the tiles up to the break, from the candidate bits: a
// thread writes 16 contiguous entries, as one 16-byte store where the tile is
// whole, admitted in full and 16-byte aligned; the workgroup that leaves last
// writes the pass summary.
__global__ __launch_bounds__(RND_THREADS) void k_split_write(
    DevCtl *c, uint8_t *__restrict__ decision, int64_t mask, uint32_t L,
    const unsigned long long *__restrict__ bits, const SplitBreak *brk_in, PassSummary *out) {
  __shared__ int64_t red[RND_THREADS / WAVE];
  const int s = L & 3, nx = (L + 1) & 3;
  const RoundRec r = c->rec[s];
  if (r.done) return;  // k_split_scan wrote the summary
  const int64_t start = r.start, end = c->p_end;
  const long long n_tiles = (end - start + TILE - 1) / TILE;
  const long long b = brk_in->tile;
  const int64_t bpos = brk_in->pos;
  const long long n_dec = b < n_tiles ? b + 1 : n_tiles;
  const int tid = threadIdx.x;
  // contiguous positions map to contiguous bytes only without wrap-around
  const bool vec = mask == -1 && ((uintptr_t(decision) + uint64_t(start)) & 15) == 0;
  int64_t tcnt = 0, tmax = -1;
  const long long G = gridDim.x;
  for (long long t0 = blockIdx.x; t0 < n_dec; t0 += SPLIT_BATCH * G) {
    // the bit words of a batch of this workgroup's tiles, loaded together
    uint32_t mb[SPLIT_BATCH];
#pragma unroll
    for (int u = 0; u < SPLIT_BATCH; ++u) {
      const long long t = t0 + u * G;
      mb[u] = t < n_dec ? uint32_t(bits[t * SPLIT_WORDS + (tid >> 2)] >> (16 * (tid & 3))) & 0xFFFFu
                        : 0u;
    }
#pragma unroll
    for (int u = 0; u < SPLIT_BATCH; ++u) {
    const long long t = t0 + u * G;
    if (t >= n_dec) break;
    const uint32_t m16 = mb[u];
    const int64_t base = start + int64_t(t) * TILE;
    const int64_t p0 = base + 16 * tid;
    if (vec && t < b && base + TILE <= end) {
      uint4 q;
      uint32_t *qw = reinterpret_cast<uint32_t *>(&q);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        qw[k] = ((m16 >> (4 * k)) & 1u) | (((m16 >> (4 * k + 1)) & 1u) << 8) |
                (((m16 >> (4 * k + 2)) & 1u) << 16) | (((m16 >> (4 * k + 3)) & 1u) << 24);
      *reinterpret_cast<uint4 *>(decision + p0) = q;
      tcnt += __builtin_popcount(m16);
      if (m16) tmax = p0 + 31 - __builtin_clz(m16);
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t p = p0 + i;
        if (p < end && (t < b || p <= bpos)) {
          const bool a = ((m16 >> i) & 1u) && (t < b || p < bpos);
          decision[p & mask] = a ? 1 : 0;
          if (a) {
            ++tcnt;
            tmax = p;
          }
        }
      }
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
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this workgroup's totals are in
    const unsigned long long prev = add_relaxed(&c->tiles_done[s], 1ULL);
    if (prev + 1 == (unsigned long long)gridDim.x)
      round_summary(c, ld_relaxed(&c->rec[nx].R), ld_relaxed(&c->rec[nx].start),
                    ld_relaxed(&c->rec[nx].done), out);
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
  out->released_jobs = ld_relaxed(&c->released_jobs);
  out->released_bytes = ld_relaxed(&c->released_bytes);
  out->done = done;
}

// Run by a whole workgroup of CMP_THREADS; `red` is LDS for block scans.
__device__ void compact_pass(DevCtl *c, const QueueArrays &q, const JobArrays &jb, int slot,
                             PassSummary *out, int append, int64_t *red) {
  if (slot >= 0 && !c->rec[slot].done) {
    if (threadIdx.x == 0 && out) write_summary(c, c->rec[slot], 0, out);
    return;
  }
  const int64_t mask = q.capacity - 1;
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

__global__ __launch_bounds__(CMP_THREADS) void k_compact(DevCtl *c, QueueArrays q, JobArrays jb,
                                                         int slot, PassSummary *out, int append) {
  __shared__ int64_t red[CMP_THREADS / WAVE];
  compact_pass(c, q, jb, slot, out, append, red);
}

// Grid-stride part of a masked release; run by every thread of a grid of
// 256-thread workgroups.
__device__ __forceinline__ void release_masked_part(DevCtl *c, const JobArrays &jb,
                                                    const uint8_t *__restrict__ mask, int64_t n,
                                                    int64_t *red) {
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

__global__ __launch_bounds__(256) void k_release_masked(DevCtl *c, JobArrays jb,
                                                        const uint8_t *__restrict__ mask, int64_t n) {
  __shared__ int64_t red[256 / WAVE];
  release_masked_part(c, jb, mask, n, red);
}

// ---------------------------------------------------------------------------
// Device chain: all release/admit rounds in one single-workgroup launch
// ---------------------------------------------------------------------------
// The running jobs a release mask can name (ids < n), listed in any order.
// run_n is 0 before the launch.
__global__ __launch_bounds__(256) void k_run_list(DevCtl *c, const int32_t *__restrict__ state,
                                                  int64_t n, int32_t *__restrict__ run_list) {
  const int lane = lane_id();
  for (int64_t base = blockIdx.x * int64_t(blockDim.x); base < n;
       base += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = base + threadIdx.x;
    const bool run = j < n && state[j] == 1;
    const uint64_t b = __ballot(run);
    if (!b) continue;
    const int leader = __builtin_ctzll(b);
    int64_t at = 0;
    if (lane == leader) at = add_relaxed(&c->run_n, int64_t(__builtin_popcountll(b)));
    at = __shfl(at, leader, WAVE);
    if (run) run_list[at + __builtin_popcountll(b & ((1ULL << lane) - 1))] = int32_t(j);
  }
}

// ---- the device chain's own steps (one workgroup of CMP_THREADS) ----------
// Scheduler scalars the chain keeps in LDS between its steps.
struct ChainState {
  int64_t capacity, used, head, tail, adm_base, run_n, rel_jobs, rel_bytes, R0;
  WinResult w;
};

// Releases every listed job whose mask byte is set and still holds a
// reservation (Sec. IV post-free with bytes == 0) and keeps the entries whose
// mask byte is clear.  A job holds a reservation exactly when it is
// positive, so exchanging it with 0 both claims and reads it: when the list
// names a job twice (each admission appends its job) or names a job that is
// no longer running, the extra entries get 0 back and drop out.  Three
// memory round trips per chunk: ids, mask bytes, exchanges.
constexpr int REL_ITEMS = 8;
constexpr int REL_CHUNK = CMP_THREADS * REL_ITEMS;
__device__ void chain_release(ChainState &L, const JobArrays &jb, const uint8_t *__restrict__ mask,
                              int64_t n_mask, int32_t *run_list, int64_t *red) {
  const int tid = threadIdx.x;
  const int64_t n = L.run_n;
  int64_t kept = 0, bytes = 0, cnt = 0;
  for (int64_t c0 = 0; c0 < n; c0 += REL_CHUNK) {
    int32_t j[REL_ITEMS];
#pragma unroll
    for (int k = 0; k < REL_ITEMS; ++k) {
      const int64_t i = c0 + int64_t(tid) * REL_ITEMS + k;
      j[k] = i < n ? run_list[i] : -1;
      if (j[k] >= n_mask) j[k] = -1;
    }
    uint8_t m[REL_ITEMS];
#pragma unroll
    for (int k = 0; k < REL_ITEMS; ++k) m[k] = j[k] >= 0 ? mask[j[k]] : 0;
    int64_t got[REL_ITEMS];
#pragma unroll
    for (int k = 0; k < REL_ITEMS; ++k)
      got[k] = (j[k] >= 0 && m[k]) ? __hip_atomic_exchange(&jb.res[j[k]], int64_t(0), __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT)
                                   : 0;
    int64_t k_loc = 0;
#pragma unroll
    for (int k = 0; k < REL_ITEMS; ++k) {
      if (got[k] > 0) {
        bytes += got[k];
        ++cnt;
        jb.state[j[k]] = 0;
      }
      k_loc += (j[k] >= 0 && !m[k]) ? 1 : 0;
    }
    // every entry of the chunk is in registers before the first write below
    int64_t tot;
    int64_t at = kept + block_excl_scan<CMP_THREADS>(k_loc, red, &tot);
#pragma unroll
    for (int k = 0; k < REL_ITEMS; ++k)
      if (j[k] >= 0 && !m[k]) run_list[at++] = j[k];
    kept += tot;
  }
  // one reduction for both totals (red holds 2 values per wave)
  bytes = wave_sum(bytes);
  cnt = wave_sum(cnt);
  __syncthreads();
  if (lane_id() == 0) {
    red[2 * (tid / WAVE)] = bytes;
    red[2 * (tid / WAVE) + 1] = cnt;
  }
  __syncthreads();
  if (tid == 0) {
    bytes = cnt = 0;
#pragma unroll
    for (int w = 0; w < CMP_THREADS / WAVE; ++w) {
      bytes += red[2 * w];
      cnt += red[2 * w + 1];
    }
    L.run_n = kept;
    L.used -= bytes;
    L.rel_bytes += bytes;
    L.rel_jobs += cnt;
  }
  __syncthreads();
}

// Queue compaction after a chain round's pass (the stable right-aligned
// compaction of compact_pass, reading the pass result from LDS); admitted
// jobs also go to the running list, at run_n + their admitted-list offset.
__device__ void chain_compact(ChainState &L, const QueueArrays &q, const JobArrays &jb,
                              int32_t *run_list, int64_t n_mask, int64_t run_cap, PassSummary *out,
                              int64_t *red) {
  const int64_t mask = q.capacity - 1;
  const int tid = threadIdx.x;
  const int64_t head = L.head, hi = L.w.hi, adm_base = L.adm_base, A = L.w.admitted;
  const int64_t run_n = L.run_n;
  int64_t surv_hi = hi;
  int64_t adm_hi = adm_base + A;
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
        // the job id only: sequence numbers match admissions to waiting
        // sched_admit requests, and none waits during a chain
        if (a_pos >= 0 && a_pos < q.capacity) q.adm_job[a_pos] = jo[k];
        if (run_list) {
          const int64_t at = run_n + (a_pos - adm_base);
          if (at < run_cap) run_list[at] = jo[k] < n_mask ? jo[k] : -1;
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
    L.head = surv_hi;
    L.used += L.w.admitted_bytes;
    L.adm_base = adm_base + A;
    if (run_list) L.run_n = run_n + A < run_cap ? run_n + A : run_cap;
    out->admitted = A;
    out->admitted_bytes = L.w.admitted_bytes;
    out->R0 = L.R0;
    out->R_after = L.w.R;
    out->rounds = L.w.rounds;
    out->start_final = L.w.start;
    out->hi = hi;
    out->head = L.head;
    out->tail = L.tail;
    out->used = L.used;
    out->adm_base = L.adm_base;
    out->released_jobs = L.rel_jobs;
    out->released_bytes = L.rel_bytes;
    out->done = 1;
  }
  __syncthreads();
}

// rounds release/admit rounds; round r > 0 first releases the listed jobs
// named by masks[(r - 1) * n_mask + j] (run_list == nullptr: no releases).
// Each round's pass runs in the first wave (window walk without a window
// limit, so it always completes), then the whole workgroup compacts the queue,
// appends the admitted jobs to the running list and writes the round's
// summary to out[r].  One workgroup: every step sees the previous one through
// workgroup barriers, and the scheduler scalars stay in LDS; reservations,
// which the release step exchanges atomically, are only touched by atomics
// inside the chain.  run_cap: entries run_list can hold (jobs running at the
// start plus every admission of the chain fit).
__global__ __launch_bounds__(CMP_THREADS) void k_chain(DevCtl *c, QueueArrays q, JobArrays jb,
                                                       const uint8_t *__restrict__ masks,
                                                       int64_t n_mask, int rounds, uint32_t L0,
                                                       int filter, PassSummary *out,
                                                       int32_t *run_list, int64_t run_cap,
                                                       int gated, int64_t new_tail,
                                                       int64_t *verdict) {
  __shared__ int64_t red[2 * CMP_THREADS / WAVE];
  if (gated) {
    // The intake launched right before has no commit of its own: its
    // workgroups counted the invalid requests.  Every wave reads the count
    // before thread 0 clears it (the barrier), so all take the same branch.
    // A clean batch moves the tail; a refused one changes nothing, no round
    // runs, and the running list the list kernel gathered is dropped.
    const unsigned long long bad = c->enq_bad;
    __syncthreads();
    if (threadIdx.x == 0) {
      *verdict = int64_t(bad);
      c->enq_bad = 0;
      if (bad)
        c->run_n = 0;
      else
        c->tail = new_tail;
    }
    if (bad) return;
  }
  __shared__ ChainState L;
  // round summaries stay in LDS until the end: stores to host memory inside
  // the loop would be waited for at every barrier
  __shared__ PassSummary sums[MAX_CHAIN];
  if (threadIdx.x == 0) {
    L.capacity = c->capacity;
    L.used = c->used;
    L.head = c->head;
    L.tail = gated ? new_tail : c->tail;
    L.adm_base = 0;
    L.rel_jobs = c->released_jobs;
    L.rel_bytes = c->released_bytes;
    const int64_t rn = run_list ? ld_relaxed(&c->run_n) : 0;
    L.run_n = rn < run_cap ? rn : run_cap;
  }
  __syncthreads();
  const int64_t qmask = q.capacity - 1;
  for (int r = 0; r < rounds; ++r) {
    // the first wave loads the pass's first windows now: the queue does not
    // change during the release step, so the loads overlap it
    int64_t pre[WIN_PF * WIN_ITEMS];
    if (threadIdx.x < WAVE) {
#pragma unroll
      for (int u = 0; u < WIN_PF; ++u)
        window_load(q.demand, qmask, L.head + u * WIN + threadIdx.x * WIN_ITEMS, L.tail,
                    *reinterpret_cast<int64_t(*)[WIN_ITEMS]>(pre + u * WIN_ITEMS));
    }
    if (r > 0 && run_list)
      chain_release(L, jb, masks + int64_t(r - 1) * n_mask, n_mask, run_list, red);
    if (threadIdx.x < WAVE) {
      const int64_t R0 = L.capacity - L.used;
      if (threadIdx.x == 0) L.R0 = R0;
      window_pass(c, q.demand, q.decision, qmask, L0 + uint32_t(r), 1 << 30, 1, filter, 0, R0,
                  L.head, L.tail, r > 0 ? 1 : 0, threadIdx.x, &L.w, pre);
    }
    __syncthreads();
    chain_compact(L, q, jb, run_list, n_mask, run_cap, sums + r, red);
  }
  if (threadIdx.x == 0) {
    c->head = L.head;
    c->used = L.used;
    c->adm_base = L.adm_base;
    c->released_jobs = L.rel_jobs;
    c->released_bytes = L.rel_bytes;
    if (run_list) st_relaxed(&c->run_n, int64_t(0));
  }
  // summaries to host-mapped memory, 8-byte words spread over the workgroup
  const int64_t words = int64_t(rounds) * int64_t(sizeof(PassSummary) / 8);
  const int64_t *src = reinterpret_cast<const int64_t *>(sums);
  int64_t *dst = reinterpret_cast<int64_t *>(out);
  for (int64_t i = threadIdx.x; i < words; i += CMP_THREADS) dst[i] = src[i];
}

// Checked intake: every workgroup validates and writes its share of the
// batch past the tail and adds its count of invalid requests (rare, so the
// counter sees almost no traffic); k_enqueue_commit then moves the tail only
// if the count is zero and reports it through host-mapped memory.
__global__ __launch_bounds__(256) void k_enqueue_checked(DevCtl *c, QueueArrays q, int64_t at,
                                                         int64_t n, const int32_t *__restrict__ job,
                                                         const int64_t *__restrict__ demand,
                                                         const int32_t *__restrict__ prio_of_job,
                                                         int64_t seq0, int32_t n_jobs,
                                                         int64_t capacity) {
  __shared__ int64_t red[256 / WAVE];
  int64_t bad = 0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t j = job[i];
    const int64_t d = demand[i];
    const bool ok = j >= 0 && j < n_jobs && d >= 1 && d <= capacity;
    bad += ok ? 0 : 1;
    const int64_t pm = (at + i) & (q.capacity - 1);
    q.demand[pm] = d;
    q.job[pm] = j;
    q.prio[pm] = ok ? prio_of_job[j] : 0;
    q.seq[pm] = seq0 + i;
  }
  bad = block_sum<256>(bad, red);
  if (threadIdx.x == 0 && bad) add_relaxed(&c->enq_bad, (unsigned long long)bad);
}

__global__ void k_enqueue_commit(DevCtl *c, int64_t new_tail, int64_t *verdict) {
  if (threadIdx.x || blockIdx.x) return;
  const unsigned long long b = c->enq_bad;
  if (!b) c->tail = new_tail;
  c->enq_bad = 0;
  *verdict = int64_t(b);
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
  SCHED_HIP_TRY(hipHostMalloc(&e.h_flag, 64, hipHostMallocMapped));
  memset(e.h_flag, 0, 64);
  SCHED_HIP_TRY(hipHostGetDevicePointer((void **)&e.d_flag, e.h_flag, 0));
  SCHED_HIP_TRY(hipMalloc(&e.d_flags, sizeof(unsigned long long) * e.max_tiles));
  SCHED_HIP_TRY(hipMemset(e.d_flags, 0, sizeof(unsigned long long) * e.max_tiles));
  if (int rc = adm_engine_grid(e, device)) return rc;
  e.launch = 1;
  e.epoch = 0;
  return SCHED_OK;
}

int adm_engine_attach(AdmEngine &e, int device, DevCtl *d_ctl, unsigned long long *d_flags,
                      int64_t max_tiles) {
  e.device = device;
  e.max_tiles = max_tiles;
  SCHED_HIP_TRY(hipHostMalloc(&e.h_ctl, sizeof(DevCtl), hipHostMallocDefault));
  memset(e.h_ctl, 0, sizeof(DevCtl));
  SCHED_HIP_TRY(hipHostMalloc(&e.h_sum, sizeof(PassSummary) * MAX_CHAIN, hipHostMallocMapped));
  memset(e.h_sum, 0, sizeof(PassSummary) * MAX_CHAIN);
  SCHED_HIP_TRY(hipHostGetDevicePointer((void **)&e.d_sum, e.h_sum, 0));
  SCHED_HIP_TRY(hipHostMalloc(&e.h_flag, 64, hipHostMallocMapped));
  memset(e.h_flag, 0, 64);
  SCHED_HIP_TRY(hipHostGetDevicePointer((void **)&e.d_flag, e.h_flag, 0));
  e.d_ctl = d_ctl;
  e.d_flags = d_flags;
  return adm_engine_grid(e, device);
}

int adm_engine_grid(AdmEngine &e, int device) {
  int cus = 0;
  SCHED_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  // The round grid: four workgroups per CU (at most what the device holds
  // at once).  Each workgroup keeps one tile of loads in flight while it
  // finishes the tile before (the next tile is reduced first, so that its
  // sum is published early); with tiles dealt in interleaved order a
  // candidate-free round of 2^26 entries streams in ~113 us with four per
  // CU, and a FIFO round in which every tile holds candidates (and so looks
  // back) in ~180 us, against ~240 us when a tile's sum was published only
  // once the tile before it had finished.
  int per_cu = 0;
  SCHED_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_round, RND_THREADS, 0));
  per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
  e.round_grid = cus * per_cu;
  return SCHED_OK;
}

int adm_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return SCHED_OK;
  k_fill_u64<<<grid_for(n, 256, 4096), 256, 0, s>>>(p, n, v);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int adm_split_init(AdmEngine &e) {
  // k_split_scan gives each of its threads at most one tile sum of the run
  // that crosses R
  const int64_t per = (e.max_tiles + SPLIT_SCAN_THREADS - 1) / SPLIT_SCAN_THREADS;
  if (per > SPLIT_SCAN_THREADS) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipMalloc(&e.d_agg, sizeof(int64_t) * e.max_tiles));
  SCHED_HIP_TRY(hipMalloc(&e.d_bits, sizeof(unsigned long long) * SPLIT_WORDS * e.max_tiles));
  SCHED_HIP_TRY(hipMalloc(&e.d_brk, sizeof(SplitBreak)));
  e.split = true;
  return SCHED_OK;
}

void adm_engine_free(AdmEngine &e) {
  if (e.d_agg) (void)hipFree(e.d_agg);
  if (e.d_bits) (void)hipFree(e.d_bits);
  if (e.d_brk) (void)hipFree(e.d_brk);
  e.d_agg = nullptr;
  e.d_bits = nullptr;
  e.d_brk = nullptr;
  e.split = false;
  if (e.d_ctl) (void)hipFree(e.d_ctl);
  if (e.h_ctl) (void)hipHostFree(e.h_ctl);
  if (e.d_flags) (void)hipFree(e.d_flags);
  if (e.h_sum) (void)hipHostFree(e.h_sum);
  if (e.h_flag) (void)hipHostFree(e.h_flag);
  e.h_sum = nullptr;
  e.d_sum = nullptr;
  e.h_flag = nullptr;
  e.d_flag = nullptr;
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
  out->released_jobs = h.released_jobs;
  out->released_bytes = h.released_bytes;
}

// Polls a round's look-back makes on a missing predecessor before it sums
// that predecessor's candidates itself (process-wide).
static std::atomic<int32_t> g_lookback_polls{LOOKBACK_POLLS_DEFAULT};
void adm_set_lookback_polls(int32_t polls) { g_lookback_polls.store(polls); }
// windows a stateless FIFO scan walks before the grid rounds take over
constexpr int FIFO_WALK_WINDOWS = 2;

// Round kernels until the pass recorded in slot L & 3 is done; returns the
// launch id whose slot holds the final state.
static int run_rounds(AdmEngine &e, const int64_t *demand, uint8_t *decision, int64_t mask,
                      int64_t span_hint, hipStream_t s, uint32_t *Lio, bool split = false) {
  uint32_t L = *Lio;
  const int grid = grid_for(span_hint, TILE, e.round_grid);
  // every round decides at least one entry, so a pass needs at most
  // span + 1 rounds; anything beyond that is an internal error
  int64_t budget = span_hint + 2 * e.rounds_per_check + 2;
  for (;;) {
    if ((budget -= e.rounds_per_check) < 0) return SCHED_E_INTERNAL;
    for (int i = 0; i < e.rounds_per_check; ++i) {
      if (split) {
        SplitBreak *brk = static_cast<SplitBreak *>(e.d_brk);
        SCHED_PROF_LAUNCH("k_split_reduce", s,
                          (k_split_reduce<<<grid, RND_THREADS, 0, s>>>(e.d_ctl, demand, mask, L,
                                                                       e.d_agg, e.d_bits)));
        SCHED_HIP_TRY(hipGetLastError());
        SCHED_PROF_LAUNCH("k_split_scan", s,
                          (k_split_scan<<<1, SPLIT_SCAN_THREADS, 0, s>>>(e.d_ctl, demand, mask, L,
                                                                         e.d_agg, brk, e.d_sum)));
        SCHED_HIP_TRY(hipGetLastError());
        SCHED_PROF_LAUNCH("k_split_write", s,
                          (k_split_write<<<grid, RND_THREADS, 0, s>>>(e.d_ctl, decision, mask, L,
                                                                      e.d_bits, brk, e.d_sum)));
        SCHED_HIP_TRY(hipGetLastError());
        L = advance(e);
        continue;
      }
      uint32_t ep;
      if (int rc = next_epoch(e, s, &ep)) return rc;
      SCHED_PROF_LAUNCH("k_round", s,
                        (k_round<<<grid, RND_THREADS, 0, s>>>(e.d_ctl, demand, decision, mask,
                                                              e.d_flags, L, ep,
                                                              g_lookback_polls.load(), e.d_sum)));
      SCHED_HIP_TRY(hipGetLastError());
      L = advance(e);
    }
    // the round that closed the batch wrote the pass summary
    if (e.sum_copy)
      SCHED_HIP_TRY(hipMemcpyAsync(e.h_sum, e.d_sum, sizeof(PassSummary), hipMemcpyDeviceToHost, s));
    SCHED_HIP_TRY(hipStreamSynchronize(s));
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
                                                        start, end, append, WIN_EMPTY_EXIT)));
  SCHED_HIP_TRY(hipGetLastError());
  *Lio = advance(e);
  return SCHED_OK;
}

int adm_scan(AdmEngine &e, int policy, const int64_t *demand, uint8_t *decision, int64_t start,
             int64_t end, int64_t R0, int window_limit, hipStream_t s, PassOut *out) {
  uint32_t L = uint32_t(e.launch);
  const int filter = policy == SCHED_POLICY_MMU ? 1 : 0;
  // Under FIFO the first break ends the pass, so one grid round decides
  // whatever the walk leaves at streaming rate; the walk only pays when the
  // break comes early.  A window without a break says it does not: past
  // FIFO_WALK_WINDOWS windows the grid takes over (a FIFO pass over 2^26
  // entries that are all admitted walked 64 windows, ~150 us, before).
  if (!filter && window_limit > FIFO_WALK_WINDOWS) window_limit = FIFO_WALK_WINDOWS;
  // the grid rounds go right behind the window kernel without a host check in
  // between: when the window walk already finished the pass they return at
  // once (a few microseconds each, less than a synchronisation)
  if (window_limit > 0) {
    if (int rc = launch_window(e, demand, decision, -1, window_limit, filter, 0, R0, start, end, 0,
                               s, &L))
      return rc;
  } else {
    k_prologue<<<1, 64, 0, s>>>(e.d_ctl, L, filter, 0, R0, start, end);
    SCHED_HIP_TRY(hipGetLastError());
  }
  // FIFO scans take the split round where the engine has its buffers (one
  // round: the first break ends the pass); first fit keeps k_round, which
  // was faster for it
  if (int rc = run_rounds(e, demand, decision, -1, end - start, s, &L, e.split && !filter))
    return rc;
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
              const uint8_t *masks, int64_t n_mask, int32_t *run_list, hipStream_t s, bool gated,
              bool none_running, int64_t new_tail) {
  if (rounds <= 0 || rounds > MAX_CHAIN) return SCHED_E_INVALID;
  const int filter = policy == SCHED_POLICY_MMU ? 1 : 0;
  const bool listed = rounds > 1 && masks && n_mask > 0;
  if (listed && (!run_list || n_mask > jb.max_jobs)) return SCHED_E_INVALID;
  // (run_n is 0 between chains, so an empty list needs no kernel)
  if (listed && !none_running) {
    SCHED_PROF_LAUNCH("k_run_list", s,
                      (k_run_list<<<grid_for(n_mask, 256, 1024), 256, 0, s>>>(e.d_ctl, jb.state,
                                                                              n_mask, run_list)));
    SCHED_HIP_TRY(hipGetLastError());
  }
  const uint32_t L0 = uint32_t(e.launch);
  SCHED_PROF_LAUNCH("k_chain", s,
                    (k_chain<<<1, CMP_THREADS, 0, s>>>(e.d_ctl, q, jb, masks, listed ? n_mask : 0,
                                                       rounds, L0, filter, e.d_sum,
                                                       listed ? run_list : nullptr,
                                                       int64_t(jb.max_jobs) + q.capacity,
                                                       gated ? 1 : 0, new_tail, e.d_flag)));
  SCHED_HIP_TRY(hipGetLastError());
  e.launch += rounds;
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

int adm_enqueue_launch(AdmEngine &e, const QueueArrays &q, int64_t at, int64_t n, const int32_t *job,
                       const int64_t *demand, const int32_t *prio_of_job, int64_t seq0,
                       int32_t n_jobs, int64_t capacity, hipStream_t s, bool commit) {
  volatile int64_t *v = e.h_flag;
  *v = -1;
  k_enqueue_checked<<<grid_for(n, 256, 4096), 256, 0, s>>>(e.d_ctl, q, at, n, job, demand,
                                                           prio_of_job, seq0, n_jobs, capacity);
  SCHED_HIP_TRY(hipGetLastError());
  if (commit) {
    k_enqueue_commit<<<1, 64, 0, s>>>(e.d_ctl, at + n, e.d_flag);
    SCHED_HIP_TRY(hipGetLastError());
  }
  return SCHED_OK;
}

int adm_enqueue_checked(AdmEngine &e, const QueueArrays &q, int64_t at, int64_t n, const int32_t *job,
                        const int64_t *demand, const int32_t *prio_of_job, int64_t seq0,
                        int32_t n_jobs, int64_t capacity, hipStream_t s, int64_t *n_bad) {
  volatile int64_t *v = e.h_flag;
  if (int rc = adm_enqueue_launch(e, q, at, n, job, demand, prio_of_job, seq0, n_jobs, capacity, s,
                                  true))
    return rc;
  SCHED_HIP_TRY(hipStreamSynchronize(s));
  const int64_t b = *v;
  if (b < 0) return SCHED_E_INTERNAL;
  *n_bad = b;
  return SCHED_OK;
}

int adm_zero_decisions(uint8_t *decision, int64_t n, hipStream_t s) {
  if (n <= 0) return SCHED_OK;
  k_fill_u8<<<grid_for(n, 256, 4096), 256, 0, s>>>(decision, n, 0);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

}  // namespace schedk
