// Context layout shared by the runtime translation units.
#pragma once

#include <condition_variable>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "admission.h"
#include "pages.h"

struct SlabState;

struct sched_ctx {
  std::mutex mu;
  std::condition_variable cv;
  sched_config_t cfg{};
  int device = 0;
  int64_t capacity = 0;
  int policy = SCHED_POLICY_MMU;
  int window_limit = 16;
  bool closing = false;
  // sched_reset only orders its kernels on `stream`; until something waits for
  // them, calls that could observe the state by another route settle first
  bool reset_pending = false;
  hipStream_t stream = nullptr;

  schedk::AdmEngine eng;
  schedk::QueueArrays q{};
  schedk::JobArrays jb{};
  int32_t *d_prio_of_job = nullptr;
  int32_t *d_run_list = nullptr;  // running jobs a chain's release masks can name
  void *d_scratch = nullptr;   // 4 KiB of small device staging
  void *h_stage = nullptr;     // 4 KiB of pinned host staging

  // host-side bookkeeping
  int32_t n_jobs = 0;
  std::vector<int32_t> prio, timeout_ms, pending;
  // owner[j]: process holding job j's memory (0: none); owned: the jobs whose
  // owner was set, for the sanity check (entries cleared since are skipped)
  std::vector<int32_t> owner, owned;
  std::unordered_map<int64_t, int32_t> host_seq;  // waiting requests made with sched_admit
  std::vector<int64_t> last_admitted_seqs;
  int64_t seq_next = 0;
  int64_t head_h = 0, tail_h = 0, used_h = 0;
  int64_t last_A = 0;
  int64_t rel_jobs_seen = 0, rel_bytes_seen = 0;  // release totals at the last pass result
  int64_t last_adm_off = 0;
  int32_t *h_adm_job = nullptr;
  int64_t *h_adm_seq = nullptr;
  int64_t h_adm_cap = 0;
  sched_stats_t stats{};

  // priority ordering: workspace (priority policies only, sized for the
  // queue at creation), the range of every known job's priority, and the
  // tail at the last ordering (the queue is still ordered while it holds)
  void *prio_tmp = nullptr;
  size_t prio_tmp_bytes = 0;
  int32_t prio_lo = INT32_MAX, prio_hi = INT32_MIN;
  int64_t prio_sorted_tail = 0;

  SlabState *slab = nullptr;

  void note_admitted(int64_t seq);
  ~sched_ctx();
};

int sched_run_pass_locked(sched_ctx *c, hipStream_t s, sched_pass_result_t *res);
// Waits for a reset still in flight on the context stream (mutex held).
int sched_settle_reset_locked(sched_ctx *c);
int sched_priority_reorder_locked(sched_ctx *c, hipStream_t s);
int sched_priority_alloc(sched_ctx *c);
void sched_priority_note(sched_ctx *c, int32_t prio);

int sched_slab_init(sched_ctx *c, int64_t pool_bytes, int32_t n_tenants);

// Page tier (slab.hip): a pool of pool_pages pages and n_slots placement
// slots; tenants are the slab's (jobs), quotas their reservations.
struct PageTier;
int pg_create(sched_ctx *c, int64_t pool_pages, int32_t n_slots, hipStream_t s, PageTier **out);
void pg_destroy(PageTier *t);
// job_status[j] (may be NULL) receives 0 for every job of a placement that
// succeeded, else the placement's status.
int pg_place(sched_ctx *c, PageTier *t, int32_t n, const schedk::PgReq *reqs, const int32_t *jobs,
             const int64_t *bytes, int32_t *job_status, hipStream_t s);
int pg_release(sched_ctx *c, PageTier *t, int32_t n, const schedk::PgReq *reqs,
               const int32_t *jobs, const int64_t *bytes, hipStream_t s);
schedk::PageMap pg_map(const PageTier *t, int32_t slot, int64_t pages);
int pg_counters(PageTier *t, hipStream_t s, schedk::PgCounters *out);
int pg_check_free(PageTier *t, hipStream_t s, int64_t *bad);
void sched_slab_free(sched_ctx *c);
int64_t sched_slab_pool_used(sched_ctx *c);
// Tenants are the context's jobs and their quotas the jobs' reservations.
bool sched_slab_quota_is_reservation(sched_ctx *c);
