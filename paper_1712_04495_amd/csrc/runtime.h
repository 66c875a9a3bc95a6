// Context layout shared by the runtime translation units.
#pragma once

#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "admission.h"
#include "pages.h"
#include "shared.h"

struct SlabState;
struct sched_ctx;

// The context's lock (the mutex of its host block): taking it loads the
// admission engine's launch counter and look-back epoch from the block,
// releasing it stores them back; on a shared context it also waits for the
// process's own device work, so the next holder, in any process, sees it.
// A holder that died with the lock leaves it to the next taker (robust mutex).
class CtxLock {
 public:
  explicit CtxLock(sched_ctx *c) : c_(c) {}
  void lock();
  void unlock();
  // for CtxCond: what lock() and unlock() do around the mutex itself
  void enter();
  void leave();

 private:
  sched_ctx *c_;
};

class CtxCond {
 public:
  explicit CtxCond(sched_ctx *c) : c_(c) {}
  void notify_all();
  // waits until notified or `until` (steady clock), the lock held on entry and exit
  void wait_until(std::unique_lock<CtxLock> &lk, std::chrono::steady_clock::time_point until);

 private:
  sched_ctx *c_;
};

struct sched_ctx {
  CtxLock mu{this};
  CtxCond cv{this};
  SharedHost *sh = nullptr;  // host state (private block, or the shared mapping)
  bool attached = false;     // opened with sched_attach: device arrays are IPC mappings
  void *shm_map = nullptr;   // the shared mapping (when shared or attached)
  size_t shm_bytes = 0;
  std::string shm_name;      // set in the process that shared the context
  sched_config_t cfg{};
  int device = 0;
  int64_t capacity = 0;
  int policy = SCHED_POLICY_MMU;
  int window_limit = 16;
  // sched_reset only orders its kernels on `stream`; until something waits for
  // them, calls that could observe the state by another route settle first
  bool reset_pending = false;
  // no job has been admitted since the last sched_reset (the reset sets it;
  // every pass, chain and restore clears it): a chain's running list then
  // starts empty without scanning the job states
  bool none_running = false;
  hipStream_t stream = nullptr;

  schedk::AdmEngine eng;
  schedk::QueueArrays q{};
  schedk::JobArrays jb{};
  int32_t *d_prio_of_job = nullptr;
  int32_t *d_run_list = nullptr;  // running jobs a chain's release masks can name
  void *d_scratch = nullptr;   // 4 KiB of small device staging
  void *h_stage = nullptr;     // 4 KiB of pinned host staging

  std::vector<int64_t> last_admitted_seqs;
  int32_t *h_adm_job = nullptr;
  int64_t *h_adm_seq = nullptr;
  int64_t h_adm_cap = 0;

  // priority ordering workspace (priority policies only, sized for the queue
  // at creation); the ordering state itself is in the host block
  void *prio_tmp = nullptr;
  size_t prio_tmp_bytes = 0;

  SlabState *slab = nullptr;

  bool shared() const { return sh && sh->shared; }
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
