// Scheduler context and the life-cycle entry points of the C ABI.
//
// The paper keeps its scheduler state -- total memory, total used, itemised
// use per client and the queue of waiting clients (Sec. III-B) -- in host
// shared memory guarded by a file lock.  Here that state lives in device
// memory: a ring of pending requests (structure of arrays), a per-job
// reservation table and a control block with capacity and used bytes.  One
// context mutex serialises the calls (the role the file lock plays in the
// paper), admission passes run on the device, and waiters block on a
// condition variable that every pass signals (the role of the user signal).
// The host side of the state is one block (shared.h) that other processes
// can map once the context is shared; they then open the device arrays
// through HIP IPC handles and take the same lock.
#include <fcntl.h>
#include <signal.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <time.h>
#include <unistd.h>

#include <cerrno>
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "admission.h"
#include "runtime.h"

using namespace schedk;

void sched_note_hip_error(hipError_t e, const char *what, const char *file, int line) {
  fprintf(stderr, "[sched] HIP error %d (%s) at %s:%d: %s\n", int(e), hipGetErrorString(e), file,
          line, what);
}

// ---------------------------------------------------------------------------
// Host block (shared.h)
// ---------------------------------------------------------------------------
namespace {
size_t up64(size_t x) { return (x + 63) / 64 * 64; }
int64_t req_slots(int64_t q_cap) {
  int64_t n = 1024;
  while (n < 2 * q_cap && n < (int64_t(1) << 22)) n <<= 1;
  return n;
}
}  // namespace

size_t SharedHost::size_for(int32_t max_jobs, int64_t q_cap) {
  size_t o = up64(sizeof(SharedHost));
  o += 4 * up64(sizeof(int32_t) * size_t(max_jobs));  // prio, timeout, pending, owner
  o += up64(sizeof(int32_t) * size_t(max_jobs));      // owned
  o += up64(sizeof(SeqEntry) * size_t(req_slots(q_cap)));
  return o;
}

SharedHost *SharedHost::init_at(void *zeroed, size_t bytes, int32_t max_jobs, int64_t q_cap,
                                bool pshared) {
  SharedHost *h = static_cast<SharedHost *>(zeroed);
  h->magic = SHARED_MAGIC;
  h->version = SHARED_VERSION;
  h->bytes = bytes;
  h->max_jobs = max_jobs;
  h->q_capacity = q_cap;
  size_t o = up64(sizeof(SharedHost));
  const size_t arr = up64(sizeof(int32_t) * size_t(max_jobs));
  h->off_prio = o;
  h->off_timeout = o += arr;
  h->off_pending = o += arr;
  h->off_owner = o += arr;
  h->off_owned = o += arr;
  h->off_req = o += arr;
  h->req_cap = req_slots(q_cap);
  h->prio_lo = INT32_MAX;
  h->prio_hi = INT32_MIN;
  for (int32_t j = 0; j < max_jobs; ++j) h->timeout_ms()[j] = 60000;
  init_sync(h, pshared);
  return h;
}

void SharedHost::init_sync(SharedHost *h, bool pshared) {
  pthread_mutexattr_t ma;
  pthread_mutexattr_init(&ma);
  pthread_mutexattr_setrobust(&ma, PTHREAD_MUTEX_ROBUST);
  if (pshared) pthread_mutexattr_setpshared(&ma, PTHREAD_PROCESS_SHARED);
  pthread_mutex_init(&h->mu, &ma);
  pthread_mutexattr_destroy(&ma);
  pthread_condattr_t ca;
  pthread_condattr_init(&ca);
  pthread_condattr_setclock(&ca, CLOCK_MONOTONIC);
  if (pshared) pthread_condattr_setpshared(&ca, PTHREAD_PROCESS_SHARED);
  pthread_cond_init(&h->cv, &ca);
  pthread_condattr_destroy(&ca);
}

bool SharedHost::req_contains(int64_t seq) {
  const SeqEntry *t = req();
  const int64_t m = req_cap - 1;
  for (int64_t i = seq & m, k = 0; k < req_cap; i = (i + 1) & m, ++k) {
    if (t[i].key == 0) return false;
    if (t[i].key == seq + 1) return true;
  }
  return false;
}

bool SharedHost::req_put(int64_t seq, int32_t job) {
  if (4 * (req_used + 1) > 3 * req_cap) req_rebuild();
  if (4 * (req_used + 1) > 3 * req_cap) return false;
  SeqEntry *t = req();
  const int64_t m = req_cap - 1;
  int64_t i = seq & m;
  while (t[i].key > 0) i = (i + 1) & m;
  if (t[i].key == 0) ++req_used;
  t[i].key = seq + 1;
  t[i].job = job;
  ++req_live;
  return true;
}

bool SharedHost::req_take(int64_t seq, int32_t *job) {
  SeqEntry *t = req();
  const int64_t m = req_cap - 1;
  for (int64_t i = seq & m, k = 0; k < req_cap; i = (i + 1) & m, ++k) {
    if (t[i].key == 0) return false;
    if (t[i].key == seq + 1) {
      *job = t[i].job;
      t[i].key = -1;
      --req_live;
      return true;
    }
  }
  return false;
}

void SharedHost::req_erase_job(int32_t job) {
  SeqEntry *t = req();
  for (int64_t i = 0; i < req_cap; ++i)
    if (t[i].key > 0 && t[i].job == job) {
      t[i].key = -1;
      --req_live;
    }
}

void SharedHost::req_clear() {
  if (req_used) memset(req(), 0, sizeof(SeqEntry) * size_t(req_cap));
  req_live = req_used = 0;
}

void SharedHost::req_rebuild() {
  std::vector<SeqEntry> live;
  live.reserve(size_t(req_live));
  req_for_each([&](int64_t seq, int32_t job) { live.push_back(SeqEntry{seq, job, 0}); });
  req_clear();
  for (const SeqEntry &e : live) req_put(e.key, e.job);
}

// ---- the context lock -------------------------------------------------------
namespace {
void mutex_acquire(pthread_mutex_t *m) {
  if (pthread_mutex_lock(m) == EOWNERDEAD) pthread_mutex_consistent(m);  // holder died
}
}  // namespace

void CtxLock::enter() {
  c_->eng.launch = c_->sh->eng_launch;
  c_->eng.epoch = c_->sh->eng_epoch;
}

void CtxLock::leave() {
  c_->sh->eng_launch = c_->eng.launch;
  c_->sh->eng_epoch = c_->eng.epoch;
  if (c_->shared()) (void)hipStreamSynchronize(c_->stream);
}

void CtxLock::lock() {
  mutex_acquire(&c_->sh->mu);
  enter();
}

void CtxLock::unlock() {
  leave();
  pthread_mutex_unlock(&c_->sh->mu);
}

void CtxCond::notify_all() { pthread_cond_broadcast(&c_->sh->cv); }

void CtxCond::wait_until(std::unique_lock<CtxLock> &, std::chrono::steady_clock::time_point until) {
  c_->mu.leave();
  const auto left = until - std::chrono::steady_clock::now();
  const int64_t ns =
      std::max<int64_t>(0, std::chrono::duration_cast<std::chrono::nanoseconds>(left).count());
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  const int64_t t = int64_t(ts.tv_nsec) + ns % 1000000000;
  ts.tv_sec += time_t(ns / 1000000000 + t / 1000000000);
  ts.tv_nsec = long(t % 1000000000);
  if (pthread_cond_timedwait(&c_->sh->cv, &c_->sh->mu, &ts) == EOWNERDEAD)
    pthread_mutex_consistent(&c_->sh->mu);
  c_->mu.enter();
}

namespace {

__global__ void k_release_one(DevCtl *c, JobArrays jb, int32_t job, int64_t amount) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t left = jb.res[job] - amount;
  jb.res[job] = left;
  if (left == 0) jb.state[job] = 0;
  c->used -= amount;
  c->released_bytes += amount;
  if (left == 0) c->released_jobs += 1;
}

// Marks every waiting request of `job` in [head, tail) withdrawn (demand -1).
__global__ void k_withdraw(DevCtl *c, QueueArrays q, int32_t job, int64_t *count) {
  const int64_t head = c->head, tail = c->tail, mask = q.capacity - 1;
  for (int64_t p = head + blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < tail;
       p += int64_t(gridDim.x) * blockDim.x) {
    const int64_t pm = p & mask;
    if (q.job[pm] == job && q.demand[pm] >= 0) {
      q.demand[pm] = -1;
      atomicAdd((unsigned long long *)count, 1ULL);
    }
  }
}

__global__ void k_set_capacity(DevCtl *c, int64_t capacity) {
  c->capacity = capacity;
  c->used = 0;
  c->head = 0;
  c->tail = 0;
}

int64_t pow2_at_least(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace

sched_ctx::~sched_ctx() {}

// Staging every process keeps for itself.
static int ctx_alloc_private(sched_ctx *c) {
  SCHED_HIP_TRY(hipMalloc(&c->d_scratch, 4096));
  SCHED_HIP_TRY(hipHostMalloc(&c->h_stage, 4096, hipHostMallocDefault));
  c->h_adm_cap = 1 << 16;
  SCHED_HIP_TRY(hipHostMalloc(&c->h_adm_job, sizeof(int32_t) * c->h_adm_cap, hipHostMallocDefault));
  SCHED_HIP_TRY(hipHostMalloc(&c->h_adm_seq, sizeof(int64_t) * c->h_adm_cap, hipHostMallocDefault));
  return SCHED_OK;
}

static int ctx_alloc(sched_ctx *c) {
  const int64_t Q = c->q.capacity;
  const int32_t J = c->jb.max_jobs;
  SCHED_HIP_TRY(hipMalloc(&c->q.demand, sizeof(int64_t) * Q));
  SCHED_HIP_TRY(hipMalloc(&c->q.job, sizeof(int32_t) * Q));
  SCHED_HIP_TRY(hipMalloc(&c->q.prio, sizeof(int32_t) * Q));
  SCHED_HIP_TRY(hipMalloc(&c->q.seq, sizeof(int64_t) * Q));
  SCHED_HIP_TRY(hipMalloc(&c->q.decision, Q));
  SCHED_HIP_TRY(hipMemset(c->q.decision, 0, Q));
  SCHED_HIP_TRY(hipMalloc(&c->q.adm_job, sizeof(int32_t) * Q));
  SCHED_HIP_TRY(hipMalloc(&c->q.adm_seq, sizeof(int64_t) * Q));
  SCHED_HIP_TRY(hipMalloc(&c->jb.res, sizeof(int64_t) * J));
  SCHED_HIP_TRY(hipMemset(c->jb.res, 0, sizeof(int64_t) * J));
  SCHED_HIP_TRY(hipMalloc(&c->jb.state, sizeof(int32_t) * J));
  SCHED_HIP_TRY(hipMemset(c->jb.state, 0, sizeof(int32_t) * J));
  SCHED_HIP_TRY(hipMalloc(&c->d_prio_of_job, sizeof(int32_t) * J));
  SCHED_HIP_TRY(hipMemset(c->d_prio_of_job, 0, sizeof(int32_t) * J));
  // running jobs at the start of a chain (<= J) plus its admissions (<= Q)
  SCHED_HIP_TRY(hipMalloc(&c->d_run_list, sizeof(int32_t) * (int64_t(J) + Q)));
  return ctx_alloc_private(c);
}

// The device arrays another process opens through IPC, in IpcArr order.
static void **shared_arrays(sched_ctx *c, void **out[IPC_N]) {
  out[IPC_DEMAND] = (void **)&c->q.demand;
  out[IPC_JOB] = (void **)&c->q.job;
  out[IPC_PRIO] = (void **)&c->q.prio;
  out[IPC_SEQ] = (void **)&c->q.seq;
  out[IPC_DECISION] = (void **)&c->q.decision;
  out[IPC_ADM_JOB] = (void **)&c->q.adm_job;
  out[IPC_ADM_SEQ] = (void **)&c->q.adm_seq;
  out[IPC_RES] = (void **)&c->jb.res;
  out[IPC_STATE] = (void **)&c->jb.state;
  out[IPC_PRIO_OF_JOB] = (void **)&c->d_prio_of_job;
  out[IPC_RUN_LIST] = (void **)&c->d_run_list;
  out[IPC_CTL] = (void **)&c->eng.d_ctl;
  out[IPC_FLAGS] = (void **)&c->eng.d_flags;
  return out[0];
}

static void ctx_free(sched_ctx *c) {
  if (c->attached) {  // arrays opened through IPC are closed, not freed
    void **arr[IPC_N];
    shared_arrays(c, arr);
    for (int k = 0; k < IPC_N; ++k)
      if (*arr[k]) {
        (void)hipIpcCloseMemHandle(*arr[k]);
        *arr[k] = nullptr;
      }
  }
  void *dev[] = {c->q.demand, c->q.job, c->q.prio, c->q.seq, c->q.decision, c->q.adm_job,
                 c->q.adm_seq, c->jb.res, c->jb.state, c->d_prio_of_job,
                 c->d_scratch, c->prio_tmp, c->d_run_list};
  for (void *p : dev)
    if (p) (void)hipFree(p);
  void *host[] = {c->h_stage, c->h_adm_job, c->h_adm_seq};
  for (void *p : host)
    if (p) (void)hipHostFree(p);
  adm_engine_free(c->eng);
  sched_slab_free(c);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  if (c->shm_map) {
    (void)munmap(c->shm_map, c->shm_bytes);
    if (!c->shm_name.empty()) (void)shm_unlink(c->shm_name.c_str());
  } else if (c->sh) {
    pthread_mutex_destroy(&c->sh->mu);
    pthread_cond_destroy(&c->sh->cv);
    free(c->sh);
  }
  c->sh = nullptr;
}

extern "C" int sched_create(const sched_config_t *cfg, sched_ctx_t **out) {
  if (!cfg || !out) return SCHED_E_INVALID;
  if (cfg->policy < SCHED_POLICY_FIFO || cfg->policy > SCHED_POLICY_PRIO_MMU) return SCHED_E_INVALID;
  if (cfg->max_jobs <= 0 || cfg->queue_capacity <= 0 || cfg->capacity_bytes < 0 ||
      cfg->headroom_bytes < 0 || cfg->slab_pool_bytes < 0 || cfg->max_tenants < 0)
    return SCHED_E_INVALID;
  int ndev = 0;
  SCHED_HIP_TRY(hipGetDeviceCount(&ndev));
  if (cfg->device < 0 || cfg->device >= ndev) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(cfg->device));
  int64_t capacity = cfg->capacity_bytes;
  if (capacity == 0) {
    size_t fr = 0, tot = 0;
    SCHED_HIP_TRY(hipMemGetInfo(&fr, &tot));
    capacity = int64_t(fr) - cfg->headroom_bytes;
  }
  if (capacity <= 0 || capacity > MAX_FREE) return SCHED_E_INVALID;

  sched_ctx *c = new sched_ctx();
  c->cfg = *cfg;
  c->device = cfg->device;
  c->capacity = capacity;
  c->policy = cfg->policy;
  c->window_limit = cfg->window_limit > 0 ? cfg->window_limit : 64;
  c->q.capacity = pow2_at_least(std::max<int64_t>(cfg->queue_capacity, WIN));
  c->jb.max_jobs = cfg->max_jobs;
  const size_t hb = SharedHost::size_for(cfg->max_jobs, c->q.capacity);
  void *mem = calloc(1, hb);
  if (!mem) {
    delete c;
    return SCHED_E_INTERNAL;
  }
  c->sh = SharedHost::init_at(mem, hb, cfg->max_jobs, c->q.capacity, false);
  int rc = SCHED_OK;
  if (hipStreamCreate(&c->stream) != hipSuccess) rc = SCHED_E_INTERNAL;
  if (rc == SCHED_OK) rc = ctx_alloc(c);
  if (rc == SCHED_OK) rc = adm_engine_init(c->eng, c->device, c->q.capacity);
  if (rc == SCHED_OK) {
    k_set_capacity<<<1, 1, 0, c->stream>>>(c->eng.d_ctl, capacity);
    if (hipGetLastError() != hipSuccess) rc = SCHED_E_INTERNAL;
  }
  if (rc == SCHED_OK &&
      (c->policy == SCHED_POLICY_PRIO_FIFO || c->policy == SCHED_POLICY_PRIO_MMU))
    rc = sched_priority_alloc(c);
  if (rc == SCHED_OK && cfg->slab_pool_bytes > 0) {
    const int32_t T = cfg->max_tenants > 0 ? cfg->max_tenants : cfg->max_jobs;
    rc = sched_slab_init(c, cfg->slab_pool_bytes, T);
  }
  if (rc == SCHED_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = SCHED_E_INTERNAL;
  if (rc != SCHED_OK) {
    ctx_free(c);
    delete c;
    return rc;
  }
  c->sh->device = c->device;
  c->sh->policy = c->policy;
  c->sh->window_limit = c->window_limit;
  c->sh->capacity = capacity;
  c->sh->max_tiles = c->eng.max_tiles;
  c->sh->eng_launch = c->eng.launch;
  c->sh->eng_epoch = c->eng.epoch;
  *out = c;
  return SCHED_OK;
}

extern "C" int sched_destroy(sched_ctx_t *c) {
  if (!c) return SCHED_E_INVALID;
  {
    std::lock_guard<CtxLock> g(c->mu);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->attached) {
      c->sh->attached -= 1;  // a detach: the context goes on in the other processes
    } else {
      c->sh->closing = true;
    }
  }
  c->cv.notify_all();
  ctx_free(c);
  delete c;
  return SCHED_OK;
}

// ---------------------------------------------------------------------------
// Sharing between processes
// ---------------------------------------------------------------------------
extern "C" int sched_share(sched_ctx_t *c, const char *name) {
  if (!c || !name || name[0] != '/' || strlen(name) > 200 || c->attached || c->shared() ||
      c->slab)
    return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  SharedHost *old = c->sh;
  mutex_acquire(&old->mu);
  int rc = SCHED_OK;
  if (!old->req_empty()) rc = SCHED_E_INVALID;  // no thread may wait on the private block
  // every exported allocation stays below 2 GiB
  const int64_t Q = c->q.capacity, J = c->jb.max_jobs;
  const int64_t biggest =
      std::max<int64_t>({8 * Q, 4 * (J + Q), 8 * int64_t(J), 8 * c->eng.max_tiles});
  if (rc == SCHED_OK && biggest >= (int64_t(1) << 31)) rc = SCHED_E_INVALID;
  int fd = -1;
  void *map = MAP_FAILED;
  if (rc == SCHED_OK) {
    fd = shm_open(name, O_CREAT | O_EXCL | O_RDWR, 0600);
    if (fd < 0 || ftruncate(fd, off_t(old->bytes)) != 0) rc = SCHED_E_INVALID;
  }
  if (rc == SCHED_OK) {
    map = mmap(nullptr, old->bytes, PROT_READ | PROT_WRITE, MAP_SHARED, fd, 0);
    if (map == MAP_FAILED) rc = SCHED_E_INTERNAL;
  }
  if (fd >= 0) close(fd);
  if (rc == SCHED_OK) {
    // the block as it stands, with a process-shared mutex and condition
    memcpy(map, old, old->bytes);
    SharedHost *h = static_cast<SharedHost *>(map);
    memset(&h->mu, 0, sizeof(h->mu));
    memset(&h->cv, 0, sizeof(h->cv));
    SharedHost::init_sync(h, true);
    h->eng_launch = c->eng.launch;
    h->eng_epoch = c->eng.epoch;
    h->owner_pid = int32_t(getpid());
    if (hipDeviceGetPCIBusId(h->pci_bus_id, sizeof(h->pci_bus_id), c->device) != hipSuccess)
      rc = SCHED_E_INTERNAL;
    void **arr[IPC_N];
    shared_arrays(c, arr);
    for (int k = 0; k < IPC_N && rc == SCHED_OK; ++k)
      if (hipIpcGetMemHandle(&h->ipc[k], *arr[k]) != hipSuccess) rc = SCHED_E_INTERNAL;
    if (rc == SCHED_OK) {
      h->shared = 1;
      c->sh = h;
      c->shm_map = map;
      c->shm_bytes = old->bytes;
      c->shm_name = name;
    }
  }
  pthread_mutex_unlock(&old->mu);
  if (rc == SCHED_OK) {
    pthread_mutex_destroy(&old->mu);
    pthread_cond_destroy(&old->cv);
    free(old);
  } else {
    if (map != MAP_FAILED) (void)munmap(map, old->bytes);
    (void)shm_unlink(name);
  }
  return rc;
}

extern "C" int sched_attach(const char *name, sched_ctx_t **out) {
  if (!name || !out) return SCHED_E_INVALID;
  const int fd = shm_open(name, O_RDWR, 0600);
  if (fd < 0) return SCHED_E_INVALID;
  struct stat st;
  void *map = MAP_FAILED;
  if (fstat(fd, &st) == 0 && size_t(st.st_size) >= sizeof(SharedHost))
    map = mmap(nullptr, size_t(st.st_size), PROT_READ | PROT_WRITE, MAP_SHARED, fd, 0);
  close(fd);
  if (map == MAP_FAILED) return SCHED_E_INVALID;
  SharedHost *h = static_cast<SharedHost *>(map);
  if (h->magic != SHARED_MAGIC || h->version != SHARED_VERSION || !h->shared ||
      h->bytes != size_t(st.st_size)) {
    (void)munmap(map, size_t(st.st_size));
    return SCHED_E_INVALID;
  }
  int dev = -1;
  if (hipDeviceGetByPCIBusId(&dev, h->pci_bus_id) != hipSuccess || hipSetDevice(dev) != hipSuccess) {
    (void)munmap(map, size_t(st.st_size));
    return SCHED_E_INVALID;
  }
  sched_ctx *c = new sched_ctx();
  c->sh = h;
  c->attached = true;
  c->shm_map = map;
  c->shm_bytes = size_t(st.st_size);
  c->device = dev;
  c->capacity = h->capacity;
  c->policy = h->policy;
  c->window_limit = h->window_limit;
  c->q.capacity = h->q_capacity;
  c->jb.max_jobs = h->max_jobs;
  c->cfg.device = dev;
  c->cfg.policy = h->policy;
  c->cfg.capacity_bytes = h->capacity;
  c->cfg.max_jobs = h->max_jobs;
  c->cfg.queue_capacity = h->q_capacity;
  c->cfg.window_limit = h->window_limit;
  int rc = SCHED_OK;
  void **arr[IPC_N];
  shared_arrays(c, arr);
  for (int k = 0; k < IPC_N && rc == SCHED_OK; ++k)
    if (hipIpcOpenMemHandle(arr[k], h->ipc[k], hipIpcMemLazyEnablePeerAccess) != hipSuccess) {
      *arr[k] = nullptr;
      rc = SCHED_E_INTERNAL;
    }
  if (rc == SCHED_OK && hipStreamCreate(&c->stream) != hipSuccess) rc = SCHED_E_INTERNAL;
  if (rc == SCHED_OK) rc = ctx_alloc_private(c);
  if (rc == SCHED_OK) rc = adm_engine_attach(c->eng, dev, c->eng.d_ctl, c->eng.d_flags, h->max_tiles);
  if (rc == SCHED_OK &&
      (c->policy == SCHED_POLICY_PRIO_FIFO || c->policy == SCHED_POLICY_PRIO_MMU))
    rc = sched_priority_alloc(c);
  if (rc != SCHED_OK) {
    c->sh = nullptr;  // the block stays to the other processes
    (void)munmap(map, c->shm_bytes);
    c->shm_map = nullptr;
    ctx_free(c);
    delete c;
    return rc;
  }
  {
    std::lock_guard<CtxLock> g(c->mu);
    h->attached += 1;
  }
  *out = c;
  return SCHED_OK;
}

static int register_locked(sched_ctx *c, int32_t n, int32_t priority, int32_t timeout_ms,
                           sched_job_t *first) {
  if (n <= 0 || c->sh->n_jobs + int64_t(n) > c->jb.max_jobs) return SCHED_E_INVALID;
  const int32_t j0 = c->sh->n_jobs;
  for (int32_t i = 0; i < n; ++i) {
    c->sh->prio()[j0 + i] = priority;
    c->sh->timeout_ms()[j0 + i] = timeout_ms;
  }
  sched_priority_note(c, priority);
  SCHED_HIP_TRY(hipSetDevice(c->device));
  // device copy of the priorities of the new jobs
  std::vector<int32_t> pr(n, priority);
  SCHED_HIP_TRY(hipMemcpyAsync(c->d_prio_of_job + j0, pr.data(), sizeof(int32_t) * n,
                               hipMemcpyHostToDevice, c->stream));
  SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
  c->sh->n_jobs += n;
  *first = j0;
  return SCHED_OK;
}

extern "C" int sched_register(sched_ctx_t *c, int32_t priority, int32_t timeout_ms,
                              sched_job_t *out_job) {
  if (!c || !out_job) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  return register_locked(c, 1, priority, timeout_ms, out_job);
}

extern "C" int sched_register_batch(sched_ctx_t *c, int32_t n, int32_t priority,
                                    int32_t timeout_ms, sched_job_t *out_first) {
  if (!c || !out_first) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  return register_locked(c, n, priority, timeout_ms, out_first);
}

// One admission pass + compaction + host bookkeeping.  Caller holds c->mu.
int sched_run_pass_locked(sched_ctx *c, hipStream_t s, sched_pass_result_t *res) {
  auto t0 = std::chrono::steady_clock::now();
  c->none_running = false;
  const int64_t head_before = c->sh->head_h;
  PassOut po{};
  const int pol = (c->policy == SCHED_POLICY_FIFO || c->policy == SCHED_POLICY_PRIO_FIFO) ? SCHED_POLICY_FIFO : SCHED_POLICY_MMU;
  if (c->policy == SCHED_POLICY_PRIO_FIFO || c->policy == SCHED_POLICY_PRIO_MMU) {
    if (int rc = sched_priority_reorder_locked(c, s)) return rc;
  }
  if (int rc = adm_pass_ctx(c->eng, pol, c->q, c->jb, c->window_limit, c->sh->tail_h - c->sh->head_h, s,
                            &po))
    return rc;
  // read back the admitted list when host-side requests wait on it
  const int64_t A = po.admitted;
  const int64_t ncopy = std::min<int64_t>(A, c->h_adm_cap);
  if (!c->sh->req_empty() && ncopy > 0) {
    SCHED_HIP_TRY(hipMemcpyAsync(c->h_adm_job, c->q.adm_job, sizeof(int32_t) * ncopy,
                                 hipMemcpyDeviceToHost, s));
    SCHED_HIP_TRY(hipMemcpyAsync(c->h_adm_seq, c->q.adm_seq, sizeof(int64_t) * ncopy,
                                 hipMemcpyDeviceToHost, s));
    SCHED_HIP_TRY(hipStreamSynchronize(s));
  }
  c->last_admitted_seqs.clear();
  if (!c->sh->req_empty()) {
    if (A > c->h_adm_cap) {
      // large admitted list: fetch it in full into a host vector
      std::vector<int32_t> jobs(A);
      std::vector<int64_t> seqs(A);
      SCHED_HIP_TRY(hipMemcpy(jobs.data(), c->q.adm_job, sizeof(int32_t) * A, hipMemcpyDeviceToHost));
      SCHED_HIP_TRY(hipMemcpy(seqs.data(), c->q.adm_seq, sizeof(int64_t) * A, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < A; ++i) c->note_admitted(seqs[i]);
    } else {
      for (int64_t i = 0; i < A; ++i) c->note_admitted(c->h_adm_seq[i]);
    }
  }
  c->sh->head_h = po.head;
  c->sh->tail_h = po.tail;
  c->sh->used_h = po.used;
  c->sh->last_A = A;
  c->sh->last_adm_off = 0;
  c->sh->stats.passes += 1;
  c->sh->stats.rounds += po.rounds;
  c->sh->stats.admitted += A;
  auto t1 = std::chrono::steady_clock::now();
  c->sh->stats.last_pass_us_x1000 =
      std::chrono::duration_cast<std::chrono::nanoseconds>(t1 - t0).count();
  if (res) {
    res->admitted = A;
    res->admitted_bytes = po.admitted_bytes;
    res->free_before = po.R0;
    res->free_after = po.R_after;
    res->rounds = po.rounds;
    res->scanned = po.start_final - head_before;
    res->pending_after = po.tail - po.head;
    res->compacted = po.hi - head_before;
    res->released = po.released_jobs - c->sh->rel_jobs_seen;
    res->released_bytes = po.released_bytes - c->sh->rel_bytes_seen;
  }
  c->sh->rel_jobs_seen = po.released_jobs;
  c->sh->rel_bytes_seen = po.released_bytes;
  c->cv.notify_all();
  return SCHED_OK;
}

void sched_ctx::note_admitted(int64_t seq) {
  int32_t job = -1;
  if (!sh->req_take(seq, &job)) return;
  if (sh->pending()[job] > 0) sh->pending()[job] -= 1;
  last_admitted_seqs.push_back(seq);
}

static int withdraw_locked(sched_ctx *c, sched_job_t job) {
  unsigned long long *cnt = (unsigned long long *)c->d_scratch;
  SCHED_HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), c->stream));
  const int64_t live = std::max<int64_t>(c->sh->tail_h - c->sh->head_h, 1);
  const int grid = int(std::min<int64_t>((live + 255) / 256, 1024));
  k_withdraw<<<grid, 256, 0, c->stream>>>(c->eng.d_ctl, c->q, job, (int64_t *)cnt);
  SCHED_HIP_TRY(hipGetLastError());
  unsigned long long n = 0;
  SCHED_HIP_TRY(hipMemcpyAsync(&n, cnt, sizeof(n), hipMemcpyDeviceToHost, c->stream));
  SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
  // the table holds the job's waiting requests only if it counts some
  if (c->sh->pending()[job] > 0) c->sh->req_erase_job(job);
  c->sh->pending()[job] = 0;
  c->sh->stats.withdrawn += int64_t(n);
  return SCHED_OK;
}

static int read_res(sched_ctx *c, sched_job_t job, int64_t *v);

static bool pid_alive(int32_t pid) { return kill(pid, 0) == 0 || errno == EPERM; }

// Sanity check (Sec. III-B, third robustness feature; Sec. IV): every job
// whose owner process has ended loses its waiting requests and its whole
// reservation, which then serves the waiting requests (one pass, run only
// when something was reclaimed).
static int sanity_locked(sched_ctx *c, int64_t *out_jobs, int64_t *out_bytes) {
  int64_t nj = 0, nb = 0;
  int32_t *owned = c->sh->owned();
  for (int32_t k = 0; k < c->sh->n_owned;) {
    const int32_t j = owned[k];
    if (c->sh->owner()[j] > 0 && pid_alive(c->sh->owner()[j])) {
      ++k;
      continue;
    }
    if (c->sh->owner()[j] > 0) {
      if (c->sh->pending()[j] > 0)
        if (int rc = withdraw_locked(c, j)) return rc;
      int64_t res = 0;
      if (int rc = read_res(c, j, &res)) return rc;
      if (res > 0) {
        k_release_one<<<1, 1, 0, c->stream>>>(c->eng.d_ctl, c->jb, j, res);
        SCHED_HIP_TRY(hipGetLastError());
        c->sh->stats.released_bytes += res;
        nb += res;
      }
      c->sh->owner()[j] = 0;
      ++nj;
    }
    owned[k] = owned[--c->sh->n_owned];  // reclaimed now or cleared before
  }
  if (nj) {
    if (int rc = sched_run_pass_locked(c, c->stream, nullptr)) return rc;
    c->cv.notify_all();
  }
  if (out_jobs) *out_jobs = nj;
  if (out_bytes) *out_bytes = nb;
  return SCHED_OK;
}

static int wait_locked(sched_ctx *c, std::unique_lock<CtxLock> &lk, sched_job_t job,
                       int32_t timeout_ms) {
  if (timeout_ms < 0) timeout_ms = c->sh->timeout_ms()[job];
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
  // a blocked client checks every 50 ms that the holders are still alive
  const auto tick = std::chrono::milliseconds(50);
  while (c->sh->pending()[job] > 0 && !c->sh->closing) {
    const auto now = std::chrono::steady_clock::now();
    if (now >= deadline) break;
    c->cv.wait_until(lk, std::min(deadline, now + tick));
    if (c->sh->pending()[job] > 0 && !c->sh->closing)
      if (int rc = sanity_locked(c, nullptr, nullptr)) return rc;
  }
  if (c->sh->pending()[job] == 0) return SCHED_OK;
  // timed out: withdraw under the mutex, so the request is either admitted
  // (by a pass that ran before this point) or withdrawn, never both
  if (int rc = withdraw_locked(c, job)) return rc;
  return SCHED_TIMEOUT;
}

extern "C" int sched_admit(sched_ctx_t *c, sched_job_t job, int32_t device, int64_t bytes,
                           uint32_t flags) {
  if (!c) return SCHED_E_INVALID;
  std::unique_lock<CtxLock> lk(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (job < 0 || job >= c->sh->n_jobs || device != c->device || bytes <= 0) return SCHED_E_INVALID;
  if (bytes > c->capacity) return SCHED_E_TOOBIG;
  if (c->sh->tail_h - c->sh->head_h + 1 > c->q.capacity) return SCHED_E_NOMEM;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  // stage the request and append it at the queue tail
  int32_t *hj = (int32_t *)c->h_stage;
  int64_t *hd = (int64_t *)((char *)c->h_stage + 64);
  hj[0] = job;
  hd[0] = bytes;
  int32_t *dj = (int32_t *)((char *)c->d_scratch + 256);
  int64_t *dd = (int64_t *)((char *)c->d_scratch + 512);
  SCHED_HIP_TRY(hipMemcpyAsync(dj, hj, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  SCHED_HIP_TRY(hipMemcpyAsync(dd, hd, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  const int64_t seq = c->sh->seq_next++;
  if (int rc = adm_enqueue(c->eng, c->q, c->sh->tail_h, 1, dj, dd, c->d_prio_of_job, seq, c->stream))
    return rc;
  c->sh->tail_h += 1;
  if (!c->sh->req_put(seq, job)) return SCHED_E_NOMEM;
  c->sh->pending()[job] += 1;
  if (int rc = sched_run_pass_locked(c, c->stream, nullptr)) return rc;
  // memory is insufficient: check whether the holders are still alive (a
  // reclaim runs a pass of its own)
  if (c->sh->req_contains(seq))
    if (int rc = sanity_locked(c, nullptr, nullptr)) return rc;
  if (!c->sh->req_contains(seq)) {
    // admitted in this pass; other requests of the job may still wait
    if (c->sh->pending()[job] == 0 || (flags & SCHED_NONBLOCK)) return SCHED_OK;
  } else if (flags & SCHED_NONBLOCK) {
    return SCHED_NOT_READY;
  }
  return wait_locked(c, lk, job, -1);
}

extern "C" int sched_wait(sched_ctx_t *c, sched_job_t job, int32_t timeout_ms) {
  if (!c) return SCHED_E_INVALID;
  std::unique_lock<CtxLock> lk(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (job < 0 || job >= c->sh->n_jobs) return SCHED_E_INVALID;
  return wait_locked(c, lk, job, timeout_ms);
}

static int read_res(sched_ctx *c, sched_job_t job, int64_t *v) {
  SCHED_HIP_TRY(hipMemcpyAsync(c->h_stage, c->jb.res + job, sizeof(int64_t), hipMemcpyDeviceToHost,
                               c->stream));
  SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
  *v = *(int64_t *)c->h_stage;
  return SCHED_OK;
}

extern "C" int sched_release(sched_ctx_t *c, sched_job_t job, int32_t device, int64_t bytes) {
  if (!c) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (job < 0 || job >= c->sh->n_jobs || bytes < 0) return SCHED_E_INVALID;
  if (device >= 0 && device != c->device) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  int64_t res = 0;
  if (int rc = read_res(c, job, &res)) return rc;
  if (bytes > res) return SCHED_E_INVALID;
  const int64_t amount = bytes == 0 ? res : bytes;
  if (amount > 0) {
    k_release_one<<<1, 1, 0, c->stream>>>(c->eng.d_ctl, c->jb, job, amount);
    SCHED_HIP_TRY(hipGetLastError());
    c->sh->stats.released_bytes += amount;
  }
  if (int rc = sched_run_pass_locked(c, c->stream, nullptr)) return rc;
  // releasing everything is the client's shutdown (Sec. IV): check the other
  // holders as well
  return bytes == 0 ? sanity_locked(c, nullptr, nullptr) : SCHED_OK;
}

extern "C" int sched_set_owner(sched_ctx_t *c, sched_job_t job, int32_t pid) {
  if (!c) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (job < 0 || job >= c->sh->n_jobs || pid < 0) return SCHED_E_INVALID;
  if (pid > 0 && c->sh->owner()[job] == 0) c->sh->owned()[c->sh->n_owned++] = job;
  c->sh->owner()[job] = pid;
  return SCHED_OK;
}

extern "C" int sched_sanity_check(sched_ctx_t *c, int64_t *reclaimed_jobs,
                                  int64_t *reclaimed_bytes) {
  if (!c) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  return sanity_locked(c, reclaimed_jobs, reclaimed_bytes);
}

extern "C" int sched_reservation(sched_ctx_t *c, sched_job_t job, int64_t *out) {
  if (!c || !out) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (job < 0 || job >= c->sh->n_jobs) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  return read_res(c, job, out);
}

extern "C" int sched_stats(sched_ctx_t *c, sched_stats_t *out) {
  if (!c || !out) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  SCHED_HIP_TRY(hipMemcpyAsync(c->eng.h_ctl, c->eng.d_ctl, sizeof(DevCtl), hipMemcpyDeviceToHost,
                               c->stream));
  SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
  const DevCtl &h = *c->eng.h_ctl;
  sched_stats_t s = c->sh->stats;
  s.capacity = c->capacity;
  s.used = h.used;
  s.pending = h.tail - h.head;
  s.released_bytes = h.released_bytes;
  int64_t running = 0;
  {
    std::vector<int32_t> st(c->sh->n_jobs);
    if (c->sh->n_jobs) {
      SCHED_HIP_TRY(hipMemcpy(st.data(), c->jb.state, sizeof(int32_t) * c->sh->n_jobs,
                              hipMemcpyDeviceToHost));
    }
    for (int32_t v : st) running += v != 0;
  }
  s.running = running;
  s.slab_pool_used = sched_slab_pool_used(c);
  s.violations = c->sh->stats.violations;
  *out = s;
  return SCHED_OK;
}

// ---------------------------------------------------------------------------
// Device-batched admission
// ---------------------------------------------------------------------------
static hipStream_t pick(sched_ctx *c, sched_stream_t s) {
  return s ? (hipStream_t)s : c->stream;
}
int sched_settle_reset_locked(sched_ctx *c) {
  if (c->reset_pending) {
    SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
    c->reset_pending = false;
  }
  return SCHED_OK;
}
// The caller's stream, ordered after a pending reset: work on the context
// stream follows it in stream order, work elsewhere waits for it.
static int pick_ordered(sched_ctx *c, sched_stream_t s, hipStream_t *out) {
  *out = pick(c, s);
  return *out == c->stream ? SCHED_OK : sched_settle_reset_locked(c);
}

extern "C" int sched_enqueue_batch(sched_ctx_t *c, int64_t n, const int32_t *d_job,
                                   const int64_t *d_demand, sched_stream_t stream) {
  if (!c || n < 0 || (n > 0 && (!d_job || !d_demand))) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (n == 0) return SCHED_OK;
  if (c->sh->tail_h - c->sh->head_h + n > c->q.capacity) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  hipStream_t s;
  if (int rc = pick_ordered(c, stream, &s)) return rc;
  int64_t n_bad = 0;
  if (int rc = adm_enqueue_checked(c->eng, c->q, c->sh->tail_h, n, d_job, d_demand, c->d_prio_of_job,
                                   c->sh->seq_next, c->sh->n_jobs, c->capacity, s, &n_bad))
    return rc;
  if (s == c->stream) c->reset_pending = false;  // the intake synchronised the stream
  if (n_bad) return SCHED_E_INVALID;
  c->sh->seq_next += n;
  c->sh->tail_h += n;
  return SCHED_OK;
}

extern "C" int sched_pass(sched_ctx_t *c, sched_stream_t stream, sched_pass_result_t *out) {
  if (!c) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  SCHED_HIP_TRY(hipSetDevice(c->device));
  sched_pass_result_t r{};
  hipStream_t s;
  if (int rc = pick_ordered(c, stream, &s)) return rc;
  if (int rc = sched_run_pass_locked(c, s, &r)) return rc;
  if (out) *out = r;
  return SCHED_OK;
}

extern "C" int sched_last_admitted(sched_ctx_t *c, int32_t *d_out, int64_t cap, int64_t *out_n,
                                   sched_stream_t stream) {
  if (!c || !out_n || cap < 0 || (cap > 0 && !d_out)) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  SCHED_HIP_TRY(hipSetDevice(c->device));
  const int64_t n = std::min<int64_t>(cap, c->sh->last_A);
  hipStream_t s;
  if (int rc = pick_ordered(c, stream, &s)) return rc;
  if (n > 0)
    SCHED_HIP_TRY(hipMemcpyAsync(d_out, c->q.adm_job + c->sh->last_adm_off, sizeof(int32_t) * n,
                                 hipMemcpyDeviceToDevice, s));
  *out_n = c->sh->last_A;
  return SCHED_OK;
}

// The host side of a device chain that has finished (its summaries are in
// the engine's host-mapped memory): per-round results, statistics, the
// mirrored queue state and the admitted ids.
static int chain_finish(sched_ctx *c, int32_t rounds, hipStream_t s, sched_pass_result_t *out,
                        int32_t *d_admitted, int64_t cap) {
  int64_t head_before = c->sh->head_h, total = 0;
  for (int r = 0; r < rounds; ++r) {
    const PassSummary &h = c->eng.h_sum[r];
    if (out) {
      sched_pass_result_t &o = out[r];
      o.admitted = h.admitted;
      o.admitted_bytes = h.admitted_bytes;
      o.free_before = h.R0;
      o.free_after = h.R_after;
      o.rounds = h.rounds;
      o.scanned = h.start_final - head_before;
      o.pending_after = h.tail - h.head;
      o.compacted = h.hi - head_before;
      o.released = h.released_jobs - c->sh->rel_jobs_seen;
      o.released_bytes = h.released_bytes - c->sh->rel_bytes_seen;
    }
    c->sh->rel_jobs_seen = h.released_jobs;
    c->sh->rel_bytes_seen = h.released_bytes;
    head_before = h.head;
    total += h.admitted;
    c->sh->stats.passes += 1;
    c->sh->stats.rounds += h.rounds;
    c->sh->stats.admitted += h.admitted;
  }
  if (s == c->stream) c->reset_pending = false;  // the chain synchronised the stream
  const PassSummary &last = c->eng.h_sum[rounds - 1];
  c->sh->head_h = last.head;
  c->sh->tail_h = last.tail;
  c->sh->used_h = last.used;
  c->sh->last_A = last.admitted;
  c->sh->last_adm_off = last.adm_base - last.admitted;
  if (cap > 0 && total > 0)
    SCHED_HIP_TRY(hipMemcpyAsync(d_admitted, c->q.adm_job, sizeof(int32_t) * std::min(cap, total),
                                 hipMemcpyDeviceToDevice, s));
  return SCHED_OK;
}

static bool chain_args_ok(sched_ctx *c, int32_t rounds, const uint8_t *d_masks, int64_t n_mask,
                          int32_t *d_admitted, int64_t cap) {
  return c && rounds > 0 && rounds <= MAX_CHAIN && n_mask >= 0 &&
         !(rounds > 1 && n_mask > 0 && !d_masks) && cap >= 0 && !(cap > 0 && !d_admitted) &&
         !c->shared();
}

static bool chain_state_ok(sched_ctx *c, int64_t n_mask) {
  return n_mask <= c->sh->n_jobs && c->sh->req_empty() &&
         (c->policy == SCHED_POLICY_FIFO || c->policy == SCHED_POLICY_MMU);
}

extern "C" int sched_pass_chain(sched_ctx_t *c, int32_t rounds, const uint8_t *d_masks,
                                int64_t n_mask, sched_stream_t stream, sched_pass_result_t *out,
                                int32_t *d_admitted, int64_t cap) {
  if (!chain_args_ok(c, rounds, d_masks, n_mask, d_admitted, cap)) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (!chain_state_ok(c, n_mask)) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  hipStream_t s;
  if (int rc = pick_ordered(c, stream, &s)) return rc;
  const bool none = c->none_running;
  c->none_running = false;
  if (int rc = adm_chain(c->eng, c->policy, c->q, c->jb, rounds, d_masks, n_mask, c->d_run_list, s,
                         false, none))
    return rc;
  return chain_finish(c, rounds, s, out, d_admitted, cap);
}

extern "C" int sched_enqueue_chain(sched_ctx_t *c, int64_t n, const int32_t *d_job,
                                   const int64_t *d_demand, int32_t rounds, const uint8_t *d_masks,
                                   int64_t n_mask, sched_stream_t stream, sched_pass_result_t *out,
                                   int32_t *d_admitted, int64_t cap) {
  if (!chain_args_ok(c, rounds, d_masks, n_mask, d_admitted, cap)) return SCHED_E_INVALID;
  if (n < 0 || (n > 0 && (!d_job || !d_demand))) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (!chain_state_ok(c, n_mask)) return SCHED_E_INVALID;
  if (c->sh->tail_h - c->sh->head_h + n > c->q.capacity) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  hipStream_t s;
  if (int rc = pick_ordered(c, stream, &s)) return rc;
  if (n > 0)
    if (int rc = adm_enqueue_launch(c->eng, c->q, c->sh->tail_h, n, d_job, d_demand,
                                    c->d_prio_of_job, c->sh->seq_next, c->sh->n_jobs, c->capacity, s,
                                    false))
      return rc;
  // the chain is queued right behind the intake and commits it (gated): a
  // refused intake leaves it nothing to do, and the one synchronisation is
  // the chain's own
  const bool none = c->none_running;
  c->none_running = false;
  if (int rc = adm_chain(c->eng, c->policy, c->q, c->jb, rounds, d_masks, n_mask, c->d_run_list, s,
                         n > 0, none, c->sh->tail_h + n))
    return rc;
  if (s == c->stream) c->reset_pending = false;
  if (n > 0) {
    const int64_t b = *reinterpret_cast<volatile int64_t *>(c->eng.h_flag);
    if (b < 0) return SCHED_E_INTERNAL;
    if (b) return SCHED_E_INVALID;
    c->sh->seq_next += n;
    c->sh->tail_h += n;
  }
  return chain_finish(c, rounds, s, out, d_admitted, cap);
}

extern "C" int sched_release_masked(sched_ctx_t *c, const uint8_t *d_mask, int64_t n,
                                    sched_stream_t stream) {
  if (!c || n < 0 || (n > 0 && !d_mask)) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (n > c->sh->n_jobs) return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  hipStream_t s;
  if (int rc = pick_ordered(c, stream, &s)) return rc;
  return adm_release_masked(c->eng, c->jb, d_mask, n, s);
}

// ---------------------------------------------------------------------------
// Stateless scan
// ---------------------------------------------------------------------------
namespace {
struct ScanWs {
  std::mutex mu;
  AdmEngine eng;
  int64_t cap_entries = 0;
};
ScanWs g_scan[64];

constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace of a scan over up to n entries: control block, pass summary,
// one look-back flag per tile (+1).
size_t scan_ws_bytes(int64_t n, size_t *off_sum, size_t *off_flags) {
  if (n < 0) n = 0;
  const size_t o_sum = align256(sizeof(DevCtl));
  const size_t o_flags = o_sum + align256(sizeof(PassSummary));
  if (off_sum) *off_sum = o_sum;
  if (off_flags) *off_flags = o_flags;
  return o_flags + sizeof(unsigned long long) * size_t((n + TILE - 1) / TILE + 1);
}

// The round grid per device (an occupancy query; cached).
int scan_grid(int dev, int *grid) {
  static std::mutex mu;
  static int cached[64] = {0};
  std::lock_guard<std::mutex> g(mu);
  if (!cached[dev]) {
    AdmEngine tmp;
    if (int rc = adm_engine_grid(tmp, dev)) return rc;
    cached[dev] = tmp.round_grid;
  }
  *grid = cached[dev];
  return SCHED_OK;
}

// A scan engine over `bytes` of device memory at `base` for n entries (no
// allocation): the pass summary is plain device memory copied into
// *host_sum; the control block and the flags of the tiles the scan uses are
// zeroed on stream s, so a fresh epoch sequence is safe whatever the memory
// held.
int scan_engine_over(char *base, size_t bytes, int64_t n, int dev, PassSummary *host_sum,
                     hipStream_t s, AdmEngine *e) {
  size_t o_sum = 0, o_flags = 0;
  if (scan_ws_bytes(n, &o_sum, &o_flags) > bytes || (uintptr_t(base) & 255)) return SCHED_E_INVALID;
  *e = AdmEngine{};
  e->device = dev;
  e->d_ctl = reinterpret_cast<DevCtl *>(base);
  e->d_sum = reinterpret_cast<PassSummary *>(base + o_sum);
  e->h_sum = host_sum;
  e->sum_copy = true;
  e->d_flags = reinterpret_cast<unsigned long long *>(base + o_flags);
  e->max_tiles = (n + TILE - 1) / TILE + 1;
  if (int rc = scan_grid(dev, &e->round_grid)) return rc;
  if (int rc = adm_fill_u64(reinterpret_cast<unsigned long long *>(base), int64_t(o_sum / 8), 0ULL, s))
    return rc;
  return adm_fill_u64(e->d_flags, e->max_tiles, 0ULL, s);
}

int scan_finish(AdmEngine &eng, int32_t policy, int64_t n, const int64_t *d_demand, int64_t R,
                uint8_t *d_decision, int32_t write_all, int32_t window_limit, hipStream_t s,
                sched_scan_result_t *out) {
  PassOut po{};
  if (int rc = adm_scan(eng, policy, d_demand, d_decision, 0, n, R, window_limit, s, &po)) return rc;
  if (write_all && po.start_final < n) {
    if (int rc = adm_zero_decisions(d_decision + po.start_final, n - po.start_final, s)) return rc;
    SCHED_HIP_TRY(hipStreamSynchronize(s));
  }
  out->admitted = po.admitted;
  out->admitted_bytes = po.admitted_bytes;
  out->free_after = po.R_after;
  out->rounds = po.rounds;
  out->last_admitted = po.hi - 1 >= 0 && po.admitted > 0 ? po.hi - 1 : -1;
  return SCHED_OK;
}
}  // namespace

extern "C" size_t sched_scan_workspace_size(int64_t n) { return scan_ws_bytes(n, nullptr, nullptr); }

extern "C" int sched_scan(int32_t policy, int64_t n, const int64_t *d_demand, int64_t R,
                          uint8_t *d_decision, int32_t write_all, int32_t window_limit, void *d_ws,
                          size_t ws_bytes, sched_stream_t stream, sched_scan_result_t *out) {
  if (!out || n < 0 || R < 0 || R > MAX_FREE) return SCHED_E_INVALID;
  if (policy != SCHED_POLICY_FIFO && policy != SCHED_POLICY_MMU) return SCHED_E_INVALID;
  if (n > 0 && (!d_demand || !d_decision)) return SCHED_E_INVALID;
  int dev = 0;
  SCHED_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return SCHED_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (d_ws) {  // the caller's workspace: nothing is allocated
    AdmEngine eng;
    PassSummary hs{};
    if (int rc = scan_engine_over((char *)d_ws, ws_bytes, n, dev, &hs, s, &eng)) return rc;
    return scan_finish(eng, policy, n, d_demand, R, d_decision, write_all, window_limit, s, out);
  }
  ScanWs &w = g_scan[dev];
  std::lock_guard<std::mutex> g(w.mu);
  if (w.cap_entries < n || !w.eng.d_ctl) {
    adm_engine_free(w.eng);
    if (int rc = adm_engine_init(w.eng, dev, std::max<int64_t>(n, 1 << 20))) return rc;
    const char *split = getenv("SCHED_SCAN_SPLIT");
    if (!(split && split[0] == '0'))
      if (int rc = adm_split_init(w.eng)) return rc;
    w.cap_entries = std::max<int64_t>(n, 1 << 20);
  }
  return scan_finish(w.eng, policy, n, d_demand, R, d_decision, write_all, window_limit, s, out);
}

// ---------------------------------------------------------------------------
// Stateless scan without allocation
// ---------------------------------------------------------------------------
// The workspace lives in a file-scope device array of fixed size: each GPU
// the library runs on holds its own copy for the life of the process.  Host
// code never passes the array's name to a kernel; it uses the device address
// hipGetSymbolAddress returns for the current device, taken once per device.
namespace {
constexpr int64_t NOALLOC_MAX_N = int64_t(1) << 28;
constexpr size_t NOALLOC_BYTES =
    align256(sizeof(DevCtl)) + align256(sizeof(PassSummary)) +
    sizeof(unsigned long long) * size_t((NOALLOC_MAX_N + TILE - 1) / TILE + 1);
}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
struct NoAllocDev {
  std::mutex mu;
  char *ptr = nullptr;  // this device's copy of `scratch`
};
NoAllocDev g_noalloc[64];
}  // namespace

extern "C" int sched_scan_noalloc(int32_t policy, int64_t n, const int64_t *d_demand, int64_t R,
                                  uint8_t *d_decision, int32_t write_all, int32_t window_limit,
                                  sched_stream_t stream, sched_scan_result_t *out) {
  if (!out || n < 0 || n > NOALLOC_MAX_N || R < 0 || R > MAX_FREE) return SCHED_E_INVALID;
  if (policy != SCHED_POLICY_FIFO && policy != SCHED_POLICY_MMU) return SCHED_E_INVALID;
  if (n > 0 && (!d_demand || !d_decision)) return SCHED_E_INVALID;
  int dev = 0;
  SCHED_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return SCHED_E_INVALID;
  NoAllocDev &g = g_noalloc[dev];
  std::lock_guard<std::mutex> lk(g.mu);  // calls on one GPU share its array: one at a time
  if (!g.ptr) SCHED_HIP_TRY(hipGetSymbolAddress((void **)&g.ptr, HIP_SYMBOL(scratch)));
  hipStream_t s = (hipStream_t)stream;
  AdmEngine eng;
  PassSummary hs{};
  if (int rc = scan_engine_over(g.ptr, NOALLOC_BYTES, n, dev, &hs, s, &eng)) return rc;
  return scan_finish(eng, policy, n, d_demand, R, d_decision, write_all, window_limit, s, out);
}

// Reservations, states and the queue's decision bytes (q_cap of them, a power
// of two >= 256, 16-byte aligned) to zero in one launch.
__global__ void k_reset_jobs(DevCtl *c, JobArrays jb, uint8_t *decision, int64_t q_cap) {
  const int64_t t0 = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t j = t0; j < jb.max_jobs; j += stride) {
    jb.res[j] = 0;
    jb.state[j] = 0;
  }
  uint4 *d16 = reinterpret_cast<uint4 *>(decision);
  for (int64_t i = t0; i < q_cap / 16; i += stride) d16[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->used = 0;
    c->head = 0;
    c->tail = 0;
    c->released_bytes = 0;
    c->released_jobs = 0;
    c->run_n = 0;
    c->enq_bad = 0;
  }
}

extern "C" int sched_reset(sched_ctx_t *c) {
  if (!c || c->shared()) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  SCHED_HIP_TRY(hipSetDevice(c->device));
  {
    const int64_t items = std::max<int64_t>(c->jb.max_jobs, c->q.capacity / 16);
    const int grid = int(std::min<int64_t>((items + 255) / 256, 4096));
    k_reset_jobs<<<grid, 256, 0, c->stream>>>(c->eng.d_ctl, c->jb, c->q.decision, c->q.capacity);
  }
  SCHED_HIP_TRY(hipGetLastError());
  c->reset_pending = true;
  c->none_running = true;
  // pending[j] counts the host-side waiting requests of job j, which are
  // exactly the entries of the request table naming j (a scan of the whole
  // table, so only when it holds any)
  if (!c->sh->req_empty())
    c->sh->req_for_each([&](int64_t, int32_t j) { c->sh->pending()[j] = 0; });
  c->sh->req_clear();
  c->sh->head_h = c->sh->tail_h = c->sh->used_h = 0;
  c->sh->prio_sorted_tail = 0;  // an empty queue is ordered
  c->sh->last_A = 0;
  c->sh->rel_jobs_seen = c->sh->rel_bytes_seen = 0;
  c->cv.notify_all();
  return SCHED_OK;
}

extern "C" int sched_set_lookback_polls(int32_t polls) {
  if (polls < 0) return SCHED_E_INVALID;
  adm_set_lookback_polls(polls);
  return SCHED_OK;
}

extern "C" const char *sched_version(void) { return "sched-mi355x 0.2 (gfx950)"; }

extern "C" int64_t sched_abi_sizeof(int32_t which) {
  switch (which) {
    case 0: return sizeof(sched_config_t);
    case 1: return sizeof(sched_stats_t);
    case 2: return sizeof(sched_pass_result_t);
    case 3: return sizeof(sched_job_desc_t);
    case 4: return sizeof(sched_job_result_t);
    case 5: return sizeof(sched_serve_opts_t);
    case 6: return sizeof(sched_serve_summary_t);
    case 7: return sizeof(sched_slab_info_t);
    case 8: return sizeof(sched_scan_result_t);
    default: return -1;
  }
}

// ---------------------------------------------------------------------------
// Checkpoint and restore (Sec. III-B, first and second robustness features:
// a backup of the shared state, and an integrity check that recovers from it)
// ---------------------------------------------------------------------------
namespace {

// Buffer layout, little-endian: the header, then per registered job
// {prio, timeout_ms, owner, 0 : int32; reservation : int64}, then per waiting
// request in queue order {demand : int64; job, prio : int32}.  The checksum is
// FNV-1a 64 (Fowler, Noll, Vo) over the whole buffer with its own field zero.
struct CkptHeader {
  char magic[8];
  uint32_t version;
  int32_t policy;
  int64_t capacity;
  int64_t used;
  int32_t n_jobs;
  int32_t reserved;
  int64_t n_pending;
  uint64_t checksum;
  uint64_t pad;
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header layout");
struct CkptJob {
  int32_t prio, timeout_ms, owner, zero;
  int64_t res;
};
struct CkptReq {
  int64_t demand;
  int32_t job, prio;
};
constexpr char kCkptMagic[8] = {'S', 'C', 'H', 'E', 'D', 'C', 'K', '1'};

uint64_t fnv1a64(const unsigned char *p, size_t n, uint64_t h = 0xcbf29ce484222325ULL) {
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ULL;
  }
  return h;
}

uint64_t ckpt_checksum(const unsigned char *buf, size_t bytes) {
  CkptHeader h;
  memcpy(&h, buf, sizeof h);
  h.checksum = 0;
  const uint64_t x = fnv1a64(reinterpret_cast<const unsigned char *>(&h), sizeof h);
  return fnv1a64(buf + sizeof h, bytes - sizeof h, x);
}

__global__ void k_set_used(DevCtl *c, int64_t used) { c->used = used; }

// Integrity check of a checkpoint (Sec. III-B, second robustness feature):
// the format, the checksum, then the accounting invariants of the shared
// state -- every reservation within [0, capacity], their sum equal to the
// used total, every waiting request naming a job of the checkpoint with that
// job's priority and a demand in [1, capacity].
bool ckpt_parse(const unsigned char *in, size_t bytes, int32_t max_jobs, CkptHeader *h,
                std::vector<CkptJob> *jobs, std::vector<CkptReq> *reqs) {
  if (bytes < sizeof(CkptHeader)) return false;
  memcpy(h, in, sizeof *h);
  if (memcmp(h->magic, kCkptMagic, 8) != 0 || h->version != 1) return false;
  if (h->n_jobs < 0 || h->n_jobs > max_jobs || h->n_pending < 0 ||
      uint64_t(h->n_pending) > bytes / sizeof(CkptReq))
    return false;
  if (bytes != sizeof *h + sizeof(CkptJob) * size_t(h->n_jobs) +
                   sizeof(CkptReq) * size_t(h->n_pending))
    return false;
  if (ckpt_checksum(in, bytes) != h->checksum) return false;
  if (h->capacity <= 0 || h->used < 0 || h->used > h->capacity) return false;
  jobs->resize(h->n_jobs);
  reqs->resize(h->n_pending);
  if (h->n_jobs) memcpy(jobs->data(), in + sizeof *h, sizeof(CkptJob) * size_t(h->n_jobs));
  if (h->n_pending)
    memcpy(reqs->data(), in + sizeof *h + sizeof(CkptJob) * size_t(h->n_jobs),
           sizeof(CkptReq) * size_t(h->n_pending));
  int64_t sum = 0;
  for (const CkptJob &r : *jobs) {
    if (r.res < 0 || r.res > h->capacity - sum || r.owner < 0 || r.zero != 0) return false;
    sum += r.res;
  }
  if (sum != h->used) return false;
  for (const CkptReq &r : *reqs)
    if (r.job < 0 || r.job >= h->n_jobs || r.demand < 1 || r.demand > h->capacity ||
        r.prio != (*jobs)[r.job].prio)
      return false;
  return true;
}

}  // namespace

extern "C" int sched_checkpoint(sched_ctx_t *c, void *buf, size_t cap, size_t *out_bytes) {
  if (!c || !out_bytes || c->shared()) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  SCHED_HIP_TRY(hipMemcpyAsync(c->eng.h_ctl, c->eng.d_ctl, sizeof(DevCtl), hipMemcpyDeviceToHost,
                               c->stream));
  SCHED_HIP_TRY(hipStreamSynchronize(c->stream));
  const int64_t head = c->eng.h_ctl->head, tail = c->eng.h_ctl->tail, used = c->eng.h_ctl->used;
  const int64_t live = tail - head;
  if (live < 0 || live > c->q.capacity) return SCHED_E_INTERNAL;
  const size_t bound = sizeof(CkptHeader) + sizeof(CkptJob) * size_t(c->sh->n_jobs) +
                       sizeof(CkptReq) * size_t(live);
  if (!buf) {  // size query: an upper bound (withdrawn entries are dropped)
    *out_bytes = bound;
    return SCHED_OK;
  }
  std::vector<int64_t> res(c->sh->n_jobs), dem(live), seq(live);
  std::vector<int32_t> job(live), pri(live);
  if (c->sh->n_jobs)
    SCHED_HIP_TRY(hipMemcpy(res.data(), c->jb.res, sizeof(int64_t) * c->sh->n_jobs,
                            hipMemcpyDeviceToHost));
  // the live ring range in at most two pieces
  const int64_t Q = c->q.capacity;
  for (int64_t done = 0; done < live;) {
    const int64_t p = (head + done) & (Q - 1);
    const int64_t n = std::min(live - done, Q - p);
    SCHED_HIP_TRY(hipMemcpy(dem.data() + done, c->q.demand + p, sizeof(int64_t) * n,
                            hipMemcpyDeviceToHost));
    SCHED_HIP_TRY(hipMemcpy(job.data() + done, c->q.job + p, sizeof(int32_t) * n,
                            hipMemcpyDeviceToHost));
    SCHED_HIP_TRY(hipMemcpy(pri.data() + done, c->q.prio + p, sizeof(int32_t) * n,
                            hipMemcpyDeviceToHost));
    SCHED_HIP_TRY(hipMemcpy(seq.data() + done, c->q.seq + p, sizeof(int64_t) * n,
                            hipMemcpyDeviceToHost));
    done += n;
  }
  // waiting requests in the order the policy serves them: arrival order, or
  // (priority, arrival) for the priority policies; withdrawn entries dropped
  std::vector<int64_t> order;
  order.reserve(live);
  for (int64_t i = 0; i < live; ++i)
    if (dem[i] >= 0) order.push_back(i);
  const bool by_prio = c->policy == SCHED_POLICY_PRIO_FIFO || c->policy == SCHED_POLICY_PRIO_MMU;
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    if (by_prio && pri[a] != pri[b]) return pri[a] < pri[b];
    return seq[a] < seq[b];
  });
  const int64_t waiting = int64_t(order.size());
  const size_t bytes = sizeof(CkptHeader) + sizeof(CkptJob) * size_t(c->sh->n_jobs) +
                       sizeof(CkptReq) * size_t(waiting);
  if (cap < bytes) return SCHED_E_INVALID;
  unsigned char *out = static_cast<unsigned char *>(buf);
  CkptHeader h{};
  memcpy(h.magic, kCkptMagic, 8);
  h.version = 1;
  h.policy = c->policy;
  h.capacity = c->capacity;
  h.used = used;
  h.n_jobs = c->sh->n_jobs;
  h.n_pending = waiting;
  size_t at = sizeof h;
  for (int32_t j = 0; j < c->sh->n_jobs; ++j) {
    const CkptJob r{c->sh->prio()[j], c->sh->timeout_ms()[j], c->sh->owner()[j], 0, res[j]};
    memcpy(out + at, &r, sizeof r);
    at += sizeof r;
  }
  for (const int64_t i : order) {
    const CkptReq r{dem[i], job[i], pri[i]};
    memcpy(out + at, &r, sizeof r);
    at += sizeof r;
  }
  memcpy(out, &h, sizeof h);
  h.checksum = ckpt_checksum(out, bytes);
  memcpy(out, &h, sizeof h);
  // a state that fails the integrity check is never handed out as a backup
  CkptHeader hv;
  std::vector<CkptJob> jv;
  std::vector<CkptReq> rv;
  if (!ckpt_parse(out, bytes, c->jb.max_jobs, &hv, &jv, &rv)) return SCHED_E_INTERNAL;
  *out_bytes = bytes;
  return SCHED_OK;
}

extern "C" int sched_restore(sched_ctx_t *c, const void *buf, size_t bytes) {
  if (!c || !buf || c->shared()) return SCHED_E_INVALID;
  std::lock_guard<CtxLock> g(c->mu);
  c->none_running = false;
  if (int rc = sched_settle_reset_locked(c)) return rc;
  CkptHeader h;
  std::vector<CkptJob> jobs;
  std::vector<CkptReq> reqs;
  if (!ckpt_parse(static_cast<const unsigned char *>(buf), bytes, c->jb.max_jobs, &h, &jobs, &reqs))
    return SCHED_E_INVALID;
  // the target is a fresh context of the same pool and policy
  if (h.policy != c->policy || h.capacity != c->capacity || c->sh->n_jobs != 0 ||
      c->sh->tail_h != c->sh->head_h || h.n_pending > c->q.capacity)
    return SCHED_E_INVALID;
  // apply: the jobs, their reservations, the used total, the waiting queue
  SCHED_HIP_TRY(hipSetDevice(c->device));
  std::vector<int32_t> pr(h.n_jobs), st(h.n_jobs);
  std::vector<int64_t> rs(h.n_jobs);
  for (int32_t j = 0; j < h.n_jobs; ++j) {
    pr[j] = jobs[j].prio;
    rs[j] = jobs[j].res;
    st[j] = jobs[j].res > 0 ? 1 : 0;
  }
  std::vector<int32_t> qj(h.n_pending);
  std::vector<int64_t> qd(h.n_pending);
  for (int64_t i = 0; i < h.n_pending; ++i) {
    qj[i] = reqs[i].job;
    qd[i] = reqs[i].demand;
  }
  int32_t *dj = nullptr;
  int64_t *dd = nullptr;
  hipError_t e = hipSuccess;
  if (h.n_pending) {
    e = hipMalloc(&dj, sizeof(int32_t) * h.n_pending);
    if (e == hipSuccess) e = hipMalloc(&dd, sizeof(int64_t) * h.n_pending);
    if (e == hipSuccess)
      e = hipMemcpy(dj, qj.data(), sizeof(int32_t) * h.n_pending, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(dd, qd.data(), sizeof(int64_t) * h.n_pending, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && h.n_jobs) {
    e = hipMemcpy(c->d_prio_of_job, pr.data(), sizeof(int32_t) * h.n_jobs, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(c->jb.res, rs.data(), sizeof(int64_t) * h.n_jobs, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(c->jb.state, st.data(), sizeof(int32_t) * h.n_jobs, hipMemcpyHostToDevice);
  }
  int rc = e == hipSuccess ? SCHED_OK : SCHED_E_INTERNAL;
  if (rc == SCHED_OK) {
    k_set_used<<<1, 1, 0, c->stream>>>(c->eng.d_ctl, h.used);
    if (hipGetLastError() != hipSuccess) rc = SCHED_E_INTERNAL;
  }
  if (rc == SCHED_OK && h.n_pending)
    rc = adm_enqueue(c->eng, c->q, c->sh->tail_h, h.n_pending, dj, dd, c->d_prio_of_job, c->sh->seq_next,
                     c->stream);
  if (rc == SCHED_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = SCHED_E_INTERNAL;
  if (dj) (void)hipFree(dj);
  if (dd) (void)hipFree(dd);
  if (rc) return rc;
  for (int32_t j = 0; j < h.n_jobs; ++j) {
    c->sh->prio()[j] = jobs[j].prio;
    sched_priority_note(c, jobs[j].prio);
    c->sh->timeout_ms()[j] = jobs[j].timeout_ms;
    c->sh->owner()[j] = jobs[j].owner;
    if (jobs[j].owner > 0) c->sh->owned()[c->sh->n_owned++] = j;
  }
  c->sh->n_jobs = h.n_jobs;
  // the restored requests wait like requests made here: sched_wait works on
  // them and the passes report their admission
  for (int64_t i = 0; i < h.n_pending; ++i) {
    if (!c->sh->req_put(c->sh->seq_next + i, qj[i])) return SCHED_E_NOMEM;
    c->sh->pending()[qj[i]] += 1;
  }
  c->sh->seq_next += h.n_pending;
  c->sh->tail_h += h.n_pending;
  c->sh->used_h = h.used;
  return SCHED_OK;
}
