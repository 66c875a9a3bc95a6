// CPU model of one workgroup of an earlier build of the grid-round kernel,
// the 8192-entry-tile build whose first run hung on the GPU, for the inputs
// of the test that was running: a single-tile queue, no window walk, one
// workgroup taking tickets.
//
// The kernel's per-thread code is executed literally by 256 std::threads:
// __syncthreads is a std::barrier over the workgroup; the wave primitives
// (__shfl_xor, __shfl_up, __ballot) exchange values through a per-wave buffer
// between two per-wave barriers; LDS variables (red, s_t, s_E, s_brk_sum) are
// plain shared memory, so a race in their use would show up as a wrong
// value.  The 32 rows of the break-tile scan are unrolled exactly as in that
// build (every row guarded by `if (!found)`).  Every barrier a thread passes
// is logged with its call site; after each round all 256 logs must be equal,
// which is the source-level condition for the barriers to match.  A thread
// that waits at a barrier the others never reach would hang the model: a
// watchdog then prints the logs and exits with status 3.
//
// Input (stdin): policy n R, then n demands.  Output: "rounds K", the
// decision vector as one line of 0/1, "admitted A bytes B", and "barriers
// consistent" or a report of the first difference.
#include <atomic>
#include <barrier>
#include <chrono>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

namespace {

constexpr int NT = 256, WAVE = 64, NW = NT / WAVE;
constexpr int RND_ITEMS = 32, TILE = NT * RND_ITEMS;

struct Rec {
  int64_t R, start;
  int done;
};
struct Ctl {
  Rec rec[4];
  long long break_tile[4];
  unsigned long long ticket[4];
  int64_t p_admitted, p_admitted_bytes, p_hi, p_rounds, p_end;
  int filter;
};

// ---- the workgroup -----------------------------------------------------------
std::barrier<> *g_blk;
std::barrier<> *g_wave[NW];
int64_t g_xchg[NW][WAVE];
uint64_t g_ballot[NW][WAVE];
std::vector<int> g_log[NT];

thread_local int tl_tid;

int lane_id() { return tl_tid % WAVE; }
void syncthreads(int site) {
  g_log[tl_tid].push_back(site);
  g_blk->arrive_and_wait();
}
int64_t shfl_xor(int64_t v, int off) {
  const int w = tl_tid / WAVE, l = lane_id();
  g_xchg[w][l] = v;
  g_wave[w]->arrive_and_wait();
  const int64_t u = g_xchg[w][l ^ off];
  g_wave[w]->arrive_and_wait();
  return u;
}
int64_t shfl_up(int64_t v, int off) {
  const int w = tl_tid / WAVE, l = lane_id();
  g_xchg[w][l] = v;
  g_wave[w]->arrive_and_wait();
  const int64_t u = l >= off ? g_xchg[w][l - off] : v;
  g_wave[w]->arrive_and_wait();
  return u;
}

int64_t sat_add(int64_t a, int64_t b, int64_t cap) {
  const int64_t s = a + b;
  return s < cap ? s : cap;
}
int64_t wave_sum(int64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += shfl_xor(v, off);
  return v;
}
int64_t wave_min(int64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t u = shfl_xor(v, off);
    v = u < v ? u : v;
  }
  return v;
}
int64_t wave_max(int64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t u = shfl_xor(v, off);
    v = u > v ? u : v;
  }
  return v;
}
int64_t wave_incl_scan_sat(int64_t v, int64_t cap) {
  const int lane = lane_id();
  for (int off = 1; off < WAVE; off <<= 1) {
    const int64_t u = shfl_up(v, off);
    if (lane >= off) v = sat_add(v, u, cap);
  }
  return v;
}

// block collectives with the LDS protocol of that build (barrier, write red,
// barrier, read red); `site` numbers the call site in the log
int64_t block_sum(int64_t v, int64_t *red, int site) {
  v = wave_sum(v);
  const int w = tl_tid / WAVE;
  syncthreads(site);
  if (lane_id() == 0) red[w] = v;
  syncthreads(site + 1);
  int64_t s = 0;
  for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}
int64_t block_min(int64_t v, int64_t *red, int site) {
  v = wave_min(v);
  const int w = tl_tid / WAVE;
  syncthreads(site);
  if (lane_id() == 0) red[w] = v;
  syncthreads(site + 1);
  int64_t s = red[0];
  for (int i = 1; i < NW; ++i) s = red[i] < s ? red[i] : s;
  return s;
}
int64_t block_max(int64_t v, int64_t *red, int site) {
  v = wave_max(v);
  const int w = tl_tid / WAVE;
  syncthreads(site);
  if (lane_id() == 0) red[w] = v;
  syncthreads(site + 1);
  int64_t s = red[0];
  for (int i = 1; i < NW; ++i) s = red[i] > s ? red[i] : s;
  return s;
}
int64_t block_excl_scan_sat(int64_t v, int64_t cap, int64_t *red, int64_t *total, int site) {
  const int w = tl_tid / WAVE;
  const int64_t incl = wave_incl_scan_sat(v, cap);
  int64_t wexcl = shfl_up(incl, 1);
  if (lane_id() == 0) wexcl = 0;
  syncthreads(site);
  if (lane_id() == WAVE - 1) red[w] = incl;
  syncthreads(site + 1);
  int64_t before = 0, tot = 0;
  for (int i = 0; i < NW; ++i) {
    if (i < w) before = sat_add(before, red[i], cap);
    tot = sat_add(tot, red[i], cap);
  }
  *total = tot;
  return sat_add(before, wexcl, cap);
}

// LDS of the kernel
int64_t red[NW];
long long s_t;
int64_t s_E, s_brk_sum;

// One launch of the round kernel by a grid of one workgroup (launch id L),
// per thread.  The look-back is not reached: the only tile is tile 0.
void round_thread(int tid, Ctl *c, const int64_t *demand, uint8_t *decision, uint32_t L) {
  tl_tid = tid;
  const int s = L & 3, nx = (L + 1) & 3;
  const Rec r = c->rec[s];
  syncthreads(1);  // (model only) every thread has read rec before thread 0 resets the next slot
  if (tid == 0) {
    c->break_tile[nx] = LLONG_MAX;
    c->ticket[nx] = 0;
    if (r.done) c->rec[nx] = r;
  }
  if (r.done) return;
  const int64_t R = r.R, start = r.start, end = c->p_end;
  const int64_t cap = R + 1;
  const bool filter = c->filter != 0;
  const long long n_tiles = (end - start + TILE - 1) / TILE;
  for (;;) {
    if (tid == 0) {
      const long long t = (long long)(c->ticket[s]++);
      const long long bt = c->break_tile[s];
      s_t = (t < n_tiles && t <= bt) ? t : -1;
    }
    syncthreads(10);
    const long long t = s_t;
    if (t < 0) break;
    const int64_t base = start + int64_t(t) * TILE;
    int64_t x[RND_ITEMS];
    int64_t tsum = 0;
    for (int j = 0; j < RND_ITEMS; ++j) {
      const int64_t p = base + int64_t(j) * NT + tid;
      const int64_t v = p < end ? demand[p] : -1;
      const bool cd = v >= 0 && (!filter || v <= R);
      x[j] = cd ? v : -1;
      tsum += cd ? v : 0;
    }
    const int64_t Araw = block_sum(tsum, red, 20);
    const int64_t A = Araw < cap ? Araw : cap;
    if (tid < WAVE) {
      const int lane = tid;
      int64_t E = 0;
      if (t != 0) {
        fprintf(stderr, "model covers single-tile queues only\n");
        std::_Exit(4);
      }
      if (lane == 0) {
        if (E <= R && sat_add(E, A, cap) > R && (long long)t < c->break_tile[s]) c->break_tile[s] = t;
        s_E = E;
      }
    }
    syncthreads(30);
    const int64_t E = s_E;
    if (E > R) continue;
    int64_t tcnt = 0, tmax = -1;
    if (Araw == 0) {
      for (int j = 0; j < RND_ITEMS; ++j) {
        const int64_t p = base + int64_t(j) * NT + tid;
        if (p < end) decision[p] = 0;
      }
      if (tid == 0 && t == n_tiles - 1) {
        c->p_admitted_bytes += E;
        c->p_rounds += 1;
        c->rec[nx].R = R - E;
        c->rec[nx].start = end;
        c->rec[nx].done = 1;
      }
      continue;
    }
    if (sat_add(E, A, cap) <= R) {
      for (int j = 0; j < RND_ITEMS; ++j) {
        const int64_t p = base + int64_t(j) * NT + tid;
        if (p < end) {
          const bool a = x[j] >= 0;
          decision[p] = a ? 1 : 0;
          if (a) {
            ++tcnt;
            tmax = p;
          }
        }
      }
      const int64_t cnt = block_sum(tcnt, red, 40);
      const int64_t mx = block_max(tmax, red, 42);
      if (tid == 0) {
        if (cnt) {
          c->p_admitted += cnt;
          if (mx + 1 > c->p_hi) c->p_hi = mx + 1;
        }
        if (t == n_tiles - 1) {
          const int64_t sum = E + A;
          c->p_admitted_bytes += sum;
          c->p_rounds += 1;
          c->rec[nx].R = R - sum;
          c->rec[nx].start = end;
          c->rec[nx].done = 1;
        }
      }
      continue;
    }
    // the break tile: 32 rows, each guarded by !found, as unrolled in that build
    int64_t carry = E, brk = -1, brk_sum = 0;
    bool found = false;
    for (int j = 0; j < RND_ITEMS; ++j) {
      if (!found) {
        const int64_t p = base + int64_t(j) * NT + tid;
        const int64_t v = x[j] >= 0 ? x[j] : 0;
        int64_t rowtot;
        const int64_t ex = block_excl_scan_sat(v, cap, red, &rowtot, 100 + 10 * j);
        const int64_t P = sat_add(carry, sat_add(ex, v, cap), cap);
        const bool over = x[j] >= 0 && P > R;
        const int64_t f = block_min(over ? tid : NT, red, 102 + 10 * j);
        if (f < NT) {
          if (tid == f) s_brk_sum = sat_add(carry, ex, cap);
          if (tid <= f && p < end) {
            const bool a = x[j] >= 0 && tid < f;
            decision[p] = a ? 1 : 0;
            if (a) {
              ++tcnt;
              tmax = p;
            }
          }
          syncthreads(104 + 10 * j);
          brk = base + int64_t(j) * NT + f;
          brk_sum = s_brk_sum;
          found = true;
        } else {
          if (p < end) {
            const bool a = x[j] >= 0;
            decision[p] = a ? 1 : 0;
            if (a) {
              ++tcnt;
              tmax = p;
            }
          }
          carry = sat_add(carry, rowtot, cap);
        }
      }
    }
    const int64_t cnt = block_sum(tcnt, red, 50);
    const int64_t mx = block_max(tmax, red, 52);
    if (tid == 0) {
      if (cnt) {
        c->p_admitted += cnt;
        if (mx + 1 > c->p_hi) c->p_hi = mx + 1;
      }
      c->p_admitted_bytes += brk_sum;
      c->p_rounds += 1;
      const int64_t R2 = R - brk_sum;
      c->rec[nx].R = R2;
      c->rec[nx].start = brk + 1;
      c->rec[nx].done = (!filter || R2 == 0 || brk + 1 >= end) ? 1 : 0;
    }
  }
}

std::atomic<int> g_finished{0};

void dump_logs() {
  for (int t = 0; t < NT; t += 63) {
    fprintf(stderr, "thread %d:", t);
    for (int x : g_log[t]) fprintf(stderr, " %d", x);
    fprintf(stderr, "\n");
  }
}

}  // namespace

int main() {
  int policy = 0;
  long long n = 0, R0 = 0;
  if (scanf("%d %lld %lld", &policy, &n, &R0) != 3 || n < 0 || n > TILE) return 2;
  std::vector<int64_t> d(size_t(n > 0 ? n : 1));
  for (long long i = 0; i < n; ++i)
    if (scanf("%ld", &d[size_t(i)]) != 1) return 2;
  std::vector<uint8_t> dec(size_t(n > 0 ? n : 1), 7);
  Ctl c{};
  // prologue (launch id 1): the pass state in slot 1
  uint32_t L = 1;
  c.rec[L & 3] = Rec{R0, 0, (0 >= n || R0 <= 0) ? 1 : 0};
  c.break_tile[L & 3] = LLONG_MAX;
  c.ticket[L & 3] = 0;
  c.p_end = n;
  c.filter = policy == 1 ? 1 : 0;
  c.p_hi = 0;
  std::barrier<> blk(NT);
  g_blk = &blk;
  for (int w = 0; w < NW; ++w) g_wave[w] = new std::barrier<>(WAVE);
  bool consistent = true;
  int rounds = 0;
  for (int launch = 0; launch < n + 4; ++launch) {
    for (auto &lg : g_log) lg.clear();
    g_finished = 0;
    std::vector<std::thread> th;
    for (int t = 0; t < NT; ++t)
      th.emplace_back([&, t] {
        round_thread(t, &c, d.data(), dec.data(), L);
        g_finished.fetch_add(1);
      });
    const auto t0 = std::chrono::steady_clock::now();
    while (g_finished.load() < NT) {
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(20)) {
        fprintf(stderr, "a barrier was never completed (launch %d)\n", launch);
        dump_logs();
        std::_Exit(3);
      }
      std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
    for (auto &x : th) x.join();
    for (int t = 1; t < NT; ++t)
      if (g_log[t] != g_log[0]) {
        consistent = false;
        fprintf(stderr, "launch %d: thread %d passed other barriers than thread 0\n", launch, t);
        dump_logs();
        break;
      }
    ++rounds;
    L += 1;
    if (c.rec[L & 3].done) break;
  }
  printf("rounds %d\n", rounds);
  for (long long i = 0; i < n; ++i) putchar(dec[size_t(i)] == 1 ? '1' : (dec[size_t(i)] == 0 ? '0' : '?'));
  printf("\nadmitted %ld bytes %ld\n", (long)c.p_admitted, (long)c.p_admitted_bytes);
  printf("%s\n", consistent ? "barriers consistent" : "barriers inconsistent");
  return consistent ? 0 : 1;
}
