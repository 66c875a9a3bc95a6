// Admission engine: device-resident pass state and the host driver that runs
// one pass of the FIFO or first-fit (MMU) policy over an int64 demand array.
#pragma once

#include "common.h"

namespace schedk {

// Window kernel: one wave, 64 lanes x 16 consecutive entries.
constexpr int WIN_THREADS = 64;
constexpr int WIN_ITEMS = 4;
constexpr int WIN_PF = 4;       // windows the single-wave walk keeps loaded
constexpr int WIN_EMPTY_EXIT = 2;  // candidate-free windows after which a limited walk hands over
constexpr int WIN = WIN_THREADS * WIN_ITEMS;
// Compaction: one workgroup, 256 threads x 8 entries per chunk.
constexpr int CMP_THREADS = 256;
constexpr int CMP_ITEMS = 8;
constexpr int CMP_CHUNK = CMP_THREADS * CMP_ITEMS;
// Round kernel: 256 threads x 16 entries per tile.
constexpr int RND_THREADS = 256;
constexpr int RND_ITEMS = 16;
constexpr int TILE = RND_THREADS * RND_ITEMS;

// Largest free-memory value a pass accepts: R + 1 must fit the 46-bit value
// field of a look-back flag word.
constexpr int64_t MAX_FREE = (int64_t(1) << 46) - 2;

// The state a pass carries from one launch to the next.  Launch L reads
// rec[L & 3] and its epilogue writes rec[(L + 1) & 3], so workgroups of L that
// start late never see the next round's parameters.
struct RoundRec {
  int64_t R;       // free memory at the start of the round
  int64_t start;   // first undecided queue position
  int32_t done;    // pass finished
  int32_t pad;
};

struct DevCtl {
  // scheduler state (persistent across passes)
  int64_t capacity;
  int64_t used;
  int64_t head;            // first live queue position
  int64_t tail;            // one past the last live queue position
  int64_t released_bytes;
  int64_t released_jobs;
  // totals of the current pass
  int64_t p_admitted;
  int64_t p_admitted_bytes;
  int64_t p_hi;            // last admitted position + 1 (max over rounds)
  int64_t p_rounds;
  int64_t p_R0;
  int64_t p_end;           // end position of the pass
  int32_t filter;          // 1: first-fit (MMU) rounds, 0: FIFO
  int32_t pad;
  int64_t adm_base;        // where the next admitted list starts (chains append)
  RoundRec rec[4];
  // the break markers are read once per tile by every workgroup of a round:
  // they take a 256-byte line of their own, away from any word that changes
  alignas(256) long long break_tile[4];
  long long break_pad[28];
  unsigned long long tiles_done[4];  // tiles finished in the round of a slot
  unsigned long long round_sum[4];   // candidate sums of those tiles
  int64_t run_n;                     // entries of the running list of a device chain
  unsigned long long enq_bad;        // invalid requests seen by a checked intake
};

// What a pass reports to the host; written by the device into host-mapped
// pinned memory (no copy kernel on the way back).
struct PassSummary {
  int64_t admitted, admitted_bytes, R0, R_after, rounds, start_final, hi;
  int64_t head, tail, used, adm_base;
  int64_t released_jobs, released_bytes;  // totals since the last reset
  int32_t done, pad;
};
constexpr int MAX_CHAIN = 256;
constexpr int32_t LOOKBACK_POLLS_DEFAULT = 256;
void adm_set_lookback_polls(int32_t polls);

struct AdmEngine {
  DevCtl *d_ctl = nullptr;
  DevCtl *h_ctl = nullptr;          // pinned host mirror
  PassSummary *h_sum = nullptr;     // host-mapped summaries, host view
  PassSummary *d_sum = nullptr;     // same memory, device view
  int64_t *h_flag = nullptr;        // host-mapped verdict of a checked intake
  int64_t *d_flag = nullptr;
  unsigned long long *d_flags = nullptr;
  int64_t max_tiles = 0;
  uint64_t launch = 1;              // launch counter of the pass chain
  uint32_t epoch = 0;               // last look-back epoch handed out
  int round_grid = 0;               // persistent grid of the round kernel
  int rounds_per_check = 1;         // round launches between host checks
  int device = 0;
  bool sum_copy = false;            // d_sum is plain device memory: copy it to h_sum
  // split rounds (adm_split_init): tile sums, candidate bits, break record
  bool split = false;
  int64_t *d_agg = nullptr;
  unsigned long long *d_bits = nullptr;
  void *d_brk = nullptr;
};

int adm_engine_init(AdmEngine &e, int device, int64_t max_entries);
// Buffers for split rounds (k_split_reduce / k_split_scan / k_split_write:
// 8 B per tile and 1 bit per entry); the engine's FIFO scans use them from
// then on instead of k_round.
int adm_split_init(AdmEngine &e);
// An engine over another process's control block and look-back flags (HIP
// IPC mappings): only the host-side buffers are allocated here.
int adm_engine_attach(AdmEngine &e, int device, DevCtl *d_ctl, unsigned long long *d_flags,
                      int64_t max_tiles);
// The round kernel's persistent grid for the device (sets e.round_grid).
int adm_engine_grid(AdmEngine &e, int device);
int adm_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s);
void adm_engine_free(AdmEngine &e);

struct PassOut {
  int64_t admitted, admitted_bytes, R0, R_after, rounds, start_final, hi;
  int64_t head, tail, used;
  int64_t released_jobs, released_bytes;  // totals since the last reset
};

// One pass over demand[start, end) with free memory R0 (stateless form: the
// caller supplies R0, start and end).  decision[] receives 1 for admitted
// entries and 0 for the entries the pass rejected.  Synchronises the stream.
int adm_scan(AdmEngine &e, int policy, const int64_t *demand, uint8_t *decision, int64_t start,
             int64_t end, int64_t R0, int window_limit, hipStream_t s, PassOut *out);

// Ctx form: R0 = capacity - used and [head, tail) are read on the device by
// the prologue kernel; compaction and accounting follow.  Synchronises.
struct QueueArrays;
struct JobArrays;
int adm_pass_ctx(AdmEngine &e, int policy, const QueueArrays &q, const JobArrays &jb,
                 int window_limit, int64_t span_hint, hipStream_t s, PassOut *out);

// Device-side state the context keeps per queue entry and per job.
struct QueueArrays {
  int64_t *demand;   // < 0 marks a withdrawn request
  int32_t *job;
  int32_t *prio;
  int64_t *seq;
  uint8_t *decision;
  int64_t capacity;  // entries, a power of two; position p lives at p & (capacity - 1)
  // admitted list of the last pass (queue order): job ids, and the request
  // sequence numbers that match admissions to waiting sched_admit requests
  int32_t *adm_job;
  int64_t *adm_seq;
};
struct JobArrays {
  int64_t *res;      // reservation bytes
  int32_t *state;    // 0 idle, 1 holds a reservation
  int32_t max_jobs;
};

// Stable compaction of the window [head, hi) after a pass: admitted entries
// and withdrawn holes leave, survivors are right-aligned, the admitted list is
// written in queue order and the admitted demands are charged to their jobs
// and to `used`.  Stream-ordered.
int adm_compact(AdmEngine &e, const QueueArrays &q, const JobArrays &j, hipStream_t s, int slot,
                PassSummary *d_out, int append);

// `rounds` release+admit rounds chained on the device (one host sync): round
// r > 0 first releases every running job j < n_mask with masks[(r-1) * n_mask
// + j] != 0, then runs a full pass (windows until done) and compaction.  The
// admitted lists of the rounds are appended one after the other.  run_list
// is device scratch of jb.max_jobs + q.capacity int32 entries (the running
// jobs a mask can name, plus every admission of the chain).
// gated: an intake launched right before without its commit
// (adm_enqueue_launch with commit = false) is committed by the chain: a
// clean batch moves the tail to new_tail, the verdict goes to *e.h_flag, and
// a refused batch leaves everything as it was (no round runs).
// none_running: the caller knows that no job is running (nothing admitted
// since every job was reset), so the running list starts empty without the
// list kernel's scan of the job states.
int adm_chain(AdmEngine &e, int policy, const QueueArrays &q, const JobArrays &jb, int rounds,
              const uint8_t *masks, int64_t n_mask, int32_t *run_list, hipStream_t s,
              bool gated = false, bool none_running = false, int64_t new_tail = 0);

int adm_zero_decisions(uint8_t *decision, int64_t n, hipStream_t s);

// Intake of n requests at queue position `at` with validation in the same
// launch: every request needs a job in [0, n_jobs) and a demand in
// [1, capacity].  The entries are written past the tail either way; the tail
// only moves when the whole batch is valid.  Synchronises the stream;
// *n_bad receives the number of invalid requests (0: appended).
int adm_enqueue_checked(AdmEngine &e, const QueueArrays &q, int64_t at, int64_t n, const int32_t *job,
                        const int64_t *demand, const int32_t *prio_of_job, int64_t seq0,
                        int32_t n_jobs, int64_t capacity, hipStream_t s, int64_t *n_bad);
// The same intake without the wait: the verdict (number of invalid
// requests) lands in host-mapped *e.h_flag once the stream reaches it (-1
// until then).  commit = false leaves the commit (tail, verdict) to a gated
// chain launched right behind.
int adm_enqueue_launch(AdmEngine &e, const QueueArrays &q, int64_t at, int64_t n, const int32_t *job,
                       const int64_t *demand, const int32_t *prio_of_job, int64_t seq0,
                       int32_t n_jobs, int64_t capacity, hipStream_t s, bool commit);
int adm_release_masked(AdmEngine &e, const JobArrays &j, const uint8_t *mask, int64_t n,
                       hipStream_t s);
int adm_enqueue(AdmEngine &e, const QueueArrays &q, int64_t at, int64_t n, const int32_t *job,
                const int64_t *demand, const int32_t *prio_of_job, int64_t seq0, hipStream_t s);

}  // namespace schedk
