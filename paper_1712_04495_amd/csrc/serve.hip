// Serving loop: memory-safe co-scheduling of a job mix on one GPU.
//
// Jobs arrive (open loop), declare their memory demand (pre-allocation,
// Sec. IV), wait in the device queue, are admitted by the policy of Sec. V
// when memory frees up, run concurrently with the other admitted jobs, and
// post-free their reservation when they end (Sec. II life cycle).  One host
// controller thread drives everything: it stages arrivals into the device
// queue, polls job completion events, posts releases, runs an admission pass
// whenever something changed and launches the admitted jobs -- large ones on
// a pool of streams, small ones packed into one persistent batched launch.
//
// Memory: an admitted job (or a batch of small ones) is placed in the page
// tier (pages.h) right after the pass that admitted it: one placement kernel
// per launch round charges each job's buffers to its reservation and maps
// their pages; the job's kernels wait for it with an event and address their
// buffers through the page table.  Admission keeps the charged bytes within
// the capacity and the pool holds one spare page per placement slot, so a
// placement of an admitted job cannot fail; the device counts any that does
// as a memory-safety violation.  When a job's completion is observed its
// placement is released (pages pushed back, charges returned) and then its
// reservation, both on the control stream, in that order.
//
// Two clocks:
//  * real time: arrivals follow their timestamps, durations are measured;
//  * virtual: events are processed one at a time in the order (time,
//    releases before arrivals, job index) with one pass after every event,
//    and a job ends exactly vdur seconds after its admission.  The schedule
//    is then a deterministic function of the inputs (admission decisions are
//    still made by the device kernels) and can be compared entry by entry
//    with a CPU replay.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <deque>
#include <iterator>
#include <queue>
#include <thread>
#include <tuple>
#include <vector>

#include "batch.h"
#include "runtime.h"

using namespace schedk;

namespace {

__global__ void k_release_list(DevCtl *c, JobArrays jb, const int32_t *__restrict__ ids, int64_t n) {
  __shared__ int64_t red[256 / WAVE];
  int64_t bytes = 0, cnt = 0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t j = ids[i];
    if (jb.state[j]) {
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

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

int64_t rup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Buffer bytes a job allocates (each array rounded up to 4 KiB); must not
// exceed its declared demand.  A GEMM's N must be a power of two in
// [256, 16384] (every operand row inside one page).
int64_t job_bytes(const sched_job_desc_t &j) {
  switch (j.kind) {
    case SCHED_JOB_TRIAD: return j.size > 0 ? 3 * rup(4 * j.size, 4096) : -1;
    case SCHED_JOB_GEMM:
      if (j.size < 256 || j.size > 16384 || (j.size & (j.size - 1))) return -1;
      return 2 * rup(2 * j.size * j.size, 4096) + rup(4 * j.size * j.size, 4096);
    case SCHED_JOB_HIST: return j.size > 0 ? rup(4 * j.size, 4096) + rup(4 * SCHED_HIST_BINS, 4096) : -1;
    default: return -1;
  }
}

int64_t pages_of(int64_t bytes) { return (bytes + PG_BYTES - 1) / PG_BYTES; }

int grid_of(int64_t n, int cap) {
  int64_t g = (n + 255) / 256;
  return int(std::max<int64_t>(1, std::min<int64_t>(g, cap)));
}

struct Running {
  int32_t job;          // -1 for a batch
  int32_t batch;        // index into batch_jobs, -1 for a single job
  int32_t slot;         // placement slot
  hipEvent_t ev_start, ev_end;
  hipStream_t stream;
};

// A placement to launch after the round's placement kernel.
struct Pending {
  int32_t job;          // -1: the batch in batch_take
  int32_t slot;
  int64_t pages;
  size_t si;            // stream index (single jobs)
};

// Pinned, host-mapped staging for the placement and release kernels' inputs
// (the kernels read it directly).  Reset only after the control stream has
// synchronised, when every kernel that read it has run.
struct Staging {
  char *h = nullptr, *d = nullptr;
  size_t cap = 0, used = 0;
  int init(size_t bytes) {
    SCHED_HIP_TRY(hipHostMalloc(&h, bytes, hipHostMallocMapped));
    SCHED_HIP_TRY(hipHostGetDevicePointer((void **)&d, h, 0));
    cap = bytes;
    return SCHED_OK;
  }
  // host and device views of `bytes` bytes, 16-B aligned; nullptr when full
  template <typename T>
  T *take(size_t count, T **dev) {
    const size_t b = (sizeof(T) * count + 15) / 16 * 16;
    if (used + b > cap) return nullptr;
    T *p = (T *)(h + used);
    *dev = (T *)(d + used);
    used += b;
    return p;
  }
  void free_() {
    if (h) (void)hipHostFree(h);
    h = d = nullptr;
  }
};

struct Serve {
  sched_ctx *c;
  const sched_job_desc_t *J;
  int64_t n;
  sched_serve_opts_t o;
  sched_job_result_t *res;
  sched_serve_summary_t sum{};
  hipStream_t stream_ctl;
  std::vector<hipStream_t> streams;
  size_t next_stream = 0;
  hipStream_t bstream = nullptr;
  hipEvent_t ev0 = nullptr;
  std::chrono::steady_clock::time_point h0;
  unsigned long long *d_digest = nullptr;
  float *d_samples = nullptr;
  int32_t *d_place_st = nullptr;   // per job: placement status (-1: never placed)
  std::vector<hipEvent_t> ev_free;
  // in-flight work per stream, oldest first (one extra queue for batches):
  // work on one stream completes in order, so only heads are polled
  std::vector<std::deque<Running>> inflight;
  std::vector<std::vector<int32_t>> batch_jobs;
  int32_t *h_job = nullptr, *d_job = nullptr;   // arrival staging
  int64_t *h_dem = nullptr, *d_dem = nullptr;
  int32_t *h_rel = nullptr, *d_rel = nullptr;   // release staging
  std::vector<int32_t> pending_small;           // admitted, waiting for the batch slot
  bool batch_running = false;
  int32_t *h_adm = nullptr;
  int64_t h_cap = 0;
  BatchEngine *beng = nullptr;
  int64_t finished = 0;
  int64_t cur_running = 0;
  // page tier
  PageTier *pt = nullptr;
  Staging stage;
  std::vector<int32_t> free_slots;
  std::deque<int32_t> slot_wait;                // admitted, waiting for a placement slot
  hipEvent_t ev_placed = nullptr;
  std::vector<Pending> round;                   // placements of the current launch round
  std::vector<int32_t> batch_take;              // jobs of the batch in `round`
  std::vector<int32_t> released_slots;          // completions of the current poll
  std::vector<std::vector<int32_t>> slot_jobs;  // jobs charged by each live slot

  double host_now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - h0).count();
  }
  double dev_time(hipEvent_t e) const {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev0, e) != hipSuccess) return -1.0;
    return ms * 1e-3;
  }
  hipEvent_t take_event() {
    if (!ev_free.empty()) {
      hipEvent_t e = ev_free.back();
      ev_free.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }

  int init() {
    stream_ctl = c->stream;
    // HIP spreads a process's streams over its hardware queues
    // (GPU_MAX_HW_QUEUES, 4 by default) round robin in creation order.  A job
    // stream that shares the control stream's queue makes every admission pass
    // wait in order behind job kernels: on the head-of-line mix, three job
    // streams beside the control stream made a pass take ~0.5 ms instead of
    // ~0.1 ms.  Without batching, job streams are therefore capped at the
    // queues left after the control stream and one for the runtime's own
    // (null-stream) work.  Batching serves oversubscribed throughput runs,
    // where more job streams pay off despite slower passes (C5: ~25 K jobs/s
    // with three job streams, ~22 K with two), so there the request stands.
    const bool batching = o.batch_small && !o.serial;
    int hw_queues = 4;
    if (const char *q = getenv("GPU_MAX_HW_QUEUES")) hw_queues = std::max(1, atoi(q));
    const int ns = std::max(1, batching ? o.n_streams : std::min(o.n_streams, hw_queues - 2));
    if (batching) SCHED_HIP_TRY(hipStreamCreate(&bstream));
    streams.resize(ns);
    for (auto &s : streams) SCHED_HIP_TRY(hipStreamCreate(&s));
    inflight.resize(ns + 1);
    SCHED_HIP_TRY(hipMalloc(&d_digest, sizeof(unsigned long long) * std::max<int64_t>(n, 1)));
    k_zero_u64<<<grid_of(n, 1024), 256, 0, stream_ctl>>>(d_digest, n);
    SCHED_HIP_TRY(hipGetLastError());
    SCHED_HIP_TRY(hipMalloc(&d_samples, sizeof(float) * GEMM_SAMPLES * std::max<int64_t>(n, 1)));
    SCHED_HIP_TRY(hipMalloc(&d_place_st, sizeof(int32_t) * std::max<int64_t>(n, 1)));
    k_fill_i32<<<grid_of(n, 1024), 256, 0, stream_ctl>>>(d_place_st, n, -1);
    SCHED_HIP_TRY(hipGetLastError());
    if (o.mode == SCHED_SERVE_REALTIME) {
      // placement slots: one spare page each on top of the capacity
      const int64_t want = o.max_placed > 0 ? o.max_placed : std::min<int64_t>(n, 16384);
      const int32_t slots = int32_t(std::max<int64_t>(1, std::min<int64_t>(want, 1 << 20)));
      const int64_t pages = pages_of(c->capacity) + slots;
      if (int rc = pg_create(c, pages, slots, stream_ctl, &pt)) return rc;
      free_slots.resize(slots);
      for (int32_t i = 0; i < slots; ++i) free_slots[i] = slots - 1 - i;
      slot_jobs.resize(slots);
      if (int rc = stage.init(size_t(8) << 20)) return rc;
      SCHED_HIP_TRY(hipEventCreateWithFlags(&ev_placed, hipEventDisableTiming));
      sum.pool_pages = pages;
      sum.placement_slots = slots;
    }
    h_cap = std::max<int64_t>(n, 1);
    SCHED_HIP_TRY(hipHostMalloc(&h_job, sizeof(int32_t) * h_cap, hipHostMallocDefault));
    SCHED_HIP_TRY(hipHostMalloc(&h_dem, sizeof(int64_t) * h_cap, hipHostMallocDefault));
    SCHED_HIP_TRY(hipHostMalloc(&h_adm, sizeof(int32_t) * h_cap, hipHostMallocDefault));
    SCHED_HIP_TRY(hipMalloc(&d_job, sizeof(int32_t) * h_cap));
    SCHED_HIP_TRY(hipMalloc(&d_dem, sizeof(int64_t) * h_cap));
    SCHED_HIP_TRY(hipHostMalloc(&h_rel, sizeof(int32_t) * h_cap, hipHostMallocDefault));
    SCHED_HIP_TRY(hipMalloc(&d_rel, sizeof(int32_t) * h_cap));
    // priorities of jobs 0..n-1
    for (int64_t i = 0; i < n; ++i) {
      h_job[i] = J[i].priority;
      sched_priority_note(c, J[i].priority);
    }
    SCHED_HIP_TRY(hipMemcpyAsync(c->d_prio_of_job, h_job, sizeof(int32_t) * n, hipMemcpyHostToDevice,
                                 stream_ctl));
    if (o.batch_small && !o.serial) {
      beng = new BatchEngine();
      if (int rc = batch_init(*beng, c->device, 8192)) return rc;
      if (int rc = batch_autotune(*beng, o.tune_cache, bstream)) return rc;
      sum.tuned_block = beng->block;
      sum.tuned_chunk = beng->chunk;
      sum.tuned_per_cu = beng->per_cu;
      sum.tuned_gemm_tile = beng->tile;
      sum.tuned_gemm_per_cu = beng->per_cu1;
      sum.tuned_from_cache = beng->from_cache ? 1 : 0;
    }
    SCHED_HIP_TRY(hipDeviceSynchronize());
    SCHED_HIP_TRY(hipEventCreate(&ev0));
    SCHED_HIP_TRY(hipEventRecord(ev0, stream_ctl));
    SCHED_HIP_TRY(hipEventSynchronize(ev0));
    h0 = std::chrono::steady_clock::now();
    return SCHED_OK;
  }

  void fini() {
    (void)hipDeviceSynchronize();
    for (auto &q : inflight)
      for (auto &r : q) {
        if (r.ev_start) ev_free.push_back(r.ev_start);
        if (r.ev_end) ev_free.push_back(r.ev_end);
      }
    for (auto e : ev_free) (void)hipEventDestroy(e);
    for (auto s : streams) (void)hipStreamDestroy(s);
    if (bstream) (void)hipStreamDestroy(bstream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev_placed) (void)hipEventDestroy(ev_placed);
    if (pt) pg_destroy(pt);
    pt = nullptr;
    stage.free_();
    void *dev[] = {d_digest, d_samples, d_place_st, d_job, d_dem, d_rel};
    for (void *p : dev)
      if (p) (void)hipFree(p);
    void *host[] = {h_job, h_dem, h_adm, h_rel};
    for (void *p : host)
      if (p) (void)hipHostFree(p);
    if (beng) {
      batch_free(*beng);
      delete beng;
    }
  }

  int64_t demand_of(int64_t j) const { return o.serial ? c->capacity : J[j].demand; }

  // Request intake: appends k staged (job, demand) pairs to the queue.
  int enqueue(int64_t k) {
    if (k == 0) return SCHED_OK;
    if (c->sh->tail_h - c->sh->head_h + k > c->q.capacity) return SCHED_E_NOMEM;
    SCHED_HIP_TRY(hipMemcpyAsync(d_job, h_job, sizeof(int32_t) * k, hipMemcpyHostToDevice, stream_ctl));
    SCHED_HIP_TRY(hipMemcpyAsync(d_dem, h_dem, sizeof(int64_t) * k, hipMemcpyHostToDevice, stream_ctl));
    if (int rc = adm_enqueue(c->eng, c->q, c->sh->tail_h, k, d_job, d_dem, c->d_prio_of_job, c->sh->seq_next,
                             stream_ctl))
      return rc;
    c->sh->seq_next += k;
    c->sh->tail_h += k;
    return SCHED_OK;
  }

  // Returns the reservations of k finished jobs (staged in h_rel).
  int release(int64_t k) {
    if (k == 0) return SCHED_OK;
    SCHED_HIP_TRY(hipMemcpyAsync(d_rel, h_rel, sizeof(int32_t) * k, hipMemcpyHostToDevice, stream_ctl));
    k_release_list<<<grid_of(k, 64), 256, 0, stream_ctl>>>(c->eng.d_ctl, c->jb, d_rel, k);
    SCHED_HIP_TRY(hipGetLastError());
    return SCHED_OK;
  }

  // One admission pass; the admitted job ids (queue order) land in h_adm.
  // The pass synchronises the control stream, so the staging is free again.
  int pass(int64_t *n_adm) {
    sched_pass_result_t pr{};
    if (int rc = sched_run_pass_locked(c, stream_ctl, &pr)) return rc;
    const int64_t A = pr.admitted;
    if (A > 0) {
      SCHED_HIP_TRY(hipMemcpyAsync(h_adm, c->q.adm_job, sizeof(int32_t) * A, hipMemcpyDeviceToHost,
                                   stream_ctl));
      SCHED_HIP_TRY(hipStreamSynchronize(stream_ctl));
    }
    stage.used = 0;
    sum.passes += 1;
    sum.peak_used = std::max<int64_t>(sum.peak_used, c->sh->used_h);
    *n_adm = A;
    return SCHED_OK;
  }

  // Staging room for `reqs` requests and `jobs` job entries; synchronises the
  // control stream to recycle the staging when it is full.
  int stage_room(size_t reqs, size_t jobs) {
    const size_t need = (sizeof(PgReq) * reqs + 15) / 16 * 16 + (4 * jobs + 15) / 16 * 16 +
                        (8 * jobs + 15) / 16 * 16;
    if (need > stage.cap) return SCHED_E_INVALID;
    if (stage.used + need > stage.cap) {
      SCHED_HIP_TRY(hipStreamSynchronize(stream_ctl));
      stage.used = 0;
    }
    return SCHED_OK;
  }

  // The placement kernel for the requests of this launch round, then the
  // event every job stream of the round waits on.
  int place_round() {
    if (round.empty()) return SCHED_OK;
    size_t n_jobs = 0;
    for (const Pending &p : round) n_jobs += p.job >= 0 ? 1 : batch_take.size();
    if (int rc = stage_room(round.size(), n_jobs)) return rc;
    PgReq *d_rq;
    int32_t *d_j;
    int64_t *d_b;
    PgReq *rq = stage.take<PgReq>(round.size(), &d_rq);
    int32_t *hj = stage.take<int32_t>(n_jobs, &d_j);
    int64_t *hb = stage.take<int64_t>(n_jobs, &d_b);
    size_t off = 0;
    for (size_t i = 0; i < round.size(); ++i) {
      const Pending &p = round[i];
      const size_t k = p.job >= 0 ? 1 : batch_take.size();
      rq[i] = PgReq{p.slot, int32_t(k), p.pages, int64_t(off)};
      for (size_t q = 0; q < k; ++q) {
        const int32_t j = p.job >= 0 ? p.job : batch_take[q];
        hj[off + q] = j;
        hb[off + q] = job_bytes(J[j]);
      }
      off += k;
    }
    if (int rc = pg_place(c, pt, int32_t(round.size()), d_rq, d_j, d_b, d_place_st, stream_ctl))
      return rc;
    SCHED_HIP_TRY(hipEventRecord(ev_placed, stream_ctl));
    sum.placements += int64_t(round.size());
    return SCHED_OK;
  }

  // Buffers and work of one placed job on stream s.
  int launch_single(int32_t j, int32_t slot, int64_t pages, hipStream_t s, Running *r) {
    const sched_job_desc_t &d = J[j];
    r->job = j;
    r->batch = -1;
    r->slot = slot;
    r->stream = s;
    r->ev_start = take_event();
    r->ev_end = take_event();
    const PageMap m = pg_map(pt, slot, pages);
    SCHED_HIP_TRY(hipEventRecord(r->ev_start, s));
    unsigned long long *dg = d_digest + j;
    if (d.kind == SCHED_JOB_TRIAD) {
      const uint64_t arr = uint64_t(rup(4 * d.size, 4096));
      if (int rc = pgt_triad_fill(m, arr, 2 * arr, d.size, d.seed, s)) return rc;
      if (int rc = pgt_triad(m, 0, arr, 2 * arr, 3.0f, d.size, o.iters, s)) return rc;
      if (o.digest)
        if (int rc = pgt_digest(m, 0, d.size, dg, s)) return rc;
    } else if (d.kind == SCHED_JOB_GEMM) {
      const int64_t N = d.size;
      const uint64_t ab = uint64_t(rup(2 * N * N, 4096));
      if (int rc = pgt_gemm_fill(m, 0, N, N, 2 * d.seed, s)) return rc;
      if (int rc = pgt_gemm_fill(m, ab, N, N, 2 * d.seed + 1, s)) return rc;
      if (int rc = pgt_gemm(m, 0, ab, 2 * ab, N, s)) return rc;
      if (o.digest) {
        if (int rc = pgt_digest(m, 2 * ab, N * N, dg, s)) return rc;
        if (int rc = pgt_gemm_samples(m, 2 * ab, N, d.seed, d_samples + int64_t(j) * GEMM_SAMPLES, s))
          return rc;
      }
    } else {
      const uint64_t kb = uint64_t(rup(4 * d.size, 4096));
      if (int rc = pgt_hist_fill(m, 0, d.size, d.seed, s)) return rc;
      if (int rc = pgt_hist(m, 0, d.size, SCHED_HIST_BINS - 1, kb, s)) return rc;
      if (o.digest)
        if (int rc = pgt_digest(m, kb, SCHED_HIST_BINS, dg, s)) return rc;
    }
    SCHED_HIP_TRY(hipEventRecord(r->ev_end, s));
    return SCHED_OK;
  }

  // Small jobs admitted together: one placement, one persistent batched
  // launch.  GEMM jobs come first in the placement: each takes a whole number
  // of pages, so all their arrays start at page boundaries.
  int launch_batch(const std::vector<int32_t> &jobs, int32_t slot, int64_t pages, Running *r) {
    r->job = -1;
    r->batch = int32_t(batch_jobs.size());
    r->slot = slot;
    r->stream = bstream;
    r->ev_start = take_event();
    r->ev_end = take_event();
    SCHED_HIP_TRY(hipEventRecord(r->ev_start, bstream));
    std::vector<BatchDesc> ds;
    ds.reserve(jobs.size());
    uint64_t base = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int32_t j : jobs) {
        const sched_job_desc_t &jd = J[j];
        if ((jd.kind == SCHED_JOB_GEMM) != (pass == 0)) continue;
        BatchDesc d{};
        d.n = jd.size;
        d.seed = jd.seed;
        d.kind = jd.kind;
        d.digest = o.digest ? d_digest + j : nullptr;
        if (jd.kind == SCHED_JOB_TRIAD) {
          const uint64_t arr = uint64_t(rup(4 * jd.size, 4096));
          d.o0 = base;
          d.o1 = base + arr;
          d.o2 = base + 2 * arr;
          d.iters = o.iters;
        } else if (jd.kind == SCHED_JOB_HIST) {
          d.o0 = base;
          d.o1 = base + uint64_t(rup(4 * jd.size, 4096));
        } else {
          const uint64_t ab = uint64_t(rup(2 * jd.size * jd.size, 4096));
          if (base % PG_BYTES || job_bytes(jd) % PG_BYTES) return SCHED_E_INTERNAL;
          d.o0 = base;
          d.o1 = base + ab;
          d.o2 = base + 2 * ab;
          d.samples = o.digest ? d_samples + int64_t(j) * GEMM_SAMPLES : nullptr;
        }
        ds.push_back(d);
        res[j].batched = 1;
        base += uint64_t(job_bytes(jd));
      }
    // the pinned table is rewritten only when no batch is in flight
    if (int rc = batch_fill(*beng, ds, beng->chunk, pg_map(pt, slot, pages), pages)) return rc;
    if (int rc = batch_launch(*beng, bstream, o.use_graph != 0)) return rc;
    SCHED_HIP_TRY(hipEventRecord(r->ev_end, bstream));
    batch_running = true;
    sum.batches += 1;
    sum.batched_jobs += int64_t(jobs.size());
    batch_jobs.push_back(jobs);
    return SCHED_OK;
  }

  // A free placement slot, or -1.
  int32_t take_slot() {
    if (free_slots.empty()) return -1;
    const int32_t s = free_slots.back();
    free_slots.pop_back();
    return s;
  }

  // Queues admitted job j for placement in this launch round, or for a slot
  // (behind the jobs already waiting for one, in admission order).
  void plan_single(int32_t j) {
    if (!slot_wait.empty() || free_slots.empty()) {
      slot_wait.push_back(j);
      sum.slot_waits += 1;
      return;
    }
    place_single(j, take_slot());
  }

  void place_single(int32_t j, int32_t slot) {
    const size_t si = pick_stream();
    round.push_back(Pending{j, slot, pages_of(job_bytes(J[j])), si});
    slot_jobs[slot].assign(1, j);
    res[j].t_place = host_now();
    ++next_stream;
    // the stream's nominal backlog includes the job from now on
    pending_backlog[si] += J[j].vdur_s;
  }

  // Placement kernel, then the work of every job of the round.
  int launch_round() {
    if (round.empty()) return SCHED_OK;
    if (int rc = place_round()) return rc;
    std::vector<char> waited(streams.size() + 1, 0);
    for (const Pending &p : round) {
      Running r{};
      if (p.job >= 0) {
        hipStream_t s = streams[p.si];
        if (!waited[p.si]) {
          SCHED_HIP_TRY(hipStreamWaitEvent(s, ev_placed, 0));
          waited[p.si] = 1;
        }
        if (int rc = launch_single(p.job, p.slot, p.pages, s, &r)) return rc;
        inflight[p.si].push_back(r);
        pending_backlog[p.si] -= J[p.job].vdur_s;
        cur_running += 1;
      } else {
        SCHED_HIP_TRY(hipStreamWaitEvent(bstream, ev_placed, 0));
        if (int rc = launch_batch(batch_take, p.slot, p.pages, &r)) return rc;
        inflight.back().push_back(r);
        cur_running += int64_t(batch_take.size());
      }
    }
    round.clear();
    batch_take.clear();
    sum.max_running = std::max<int64_t>(sum.max_running, cur_running);
    return SCHED_OK;
  }

  int launch_admitted(int64_t A, double now) {
    for (int64_t i = 0; i < A; ++i) {
      const int32_t j = h_adm[i];
      res[j].t_admit = now;
      if (beng && J[j].demand < o.small_bytes) {
        pending_small.push_back(j);
        continue;
      }
      plan_single(j);
    }
    plan_batch();
    return launch_round();
  }

  // The job stream with the least expected backlog: the sum of the nominal
  // durations of the jobs still in flight on it (ties in round-robin order).
  // Streams run their jobs in order, so a short job placed behind a long one
  // would hold its reservation until the long one ends.
  std::vector<double> pending_backlog;
  size_t pick_stream() {
    if (pending_backlog.size() != streams.size()) pending_backlog.assign(streams.size(), 0.0);
    size_t best = next_stream % streams.size();
    double best_load = backlog(best);
    for (size_t k = 1; k < streams.size(); ++k) {
      const size_t si = (next_stream + k) % streams.size();
      const double l = backlog(si);
      if (l < best_load) {
        best = si;
        best_load = l;
      }
    }
    return best;
  }
  double backlog(size_t si) const {
    double t = si < pending_backlog.size() ? pending_backlog[si] : 0.0;
    for (const Running &r : inflight[si])
      if (r.job >= 0) t += J[r.job].vdur_s;
    return t;
  }

  // Jobs waiting for a slot, oldest first, while slots are free.
  int launch_slot_waiters() {
    while (!slot_wait.empty() && !free_slots.empty()) {
      const int32_t j = slot_wait.front();
      slot_wait.pop_front();
      place_single(j, take_slot());
    }
    return SCHED_OK;
  }

  // The waiting small jobs (at most what one placement maps) as one batch
  // placement of this round, when no batch is in flight.
  void plan_batch() {
    if (!beng || batch_running || pending_small.empty() || !batch_take.empty()) return;
    const int32_t slot = take_slot();
    if (slot < 0) return;  // retried after the next completion
    int64_t bytes = 0;
    size_t k = 0;
    while (k < pending_small.size() && k < size_t(beng->max_desc)) {
      const int64_t b = job_bytes(J[pending_small[k]]);
      if (pages_of(bytes + b) > PG_MAX_PAGES) break;
      bytes += b;
      ++k;
    }
    batch_take.assign(pending_small.begin(), pending_small.begin() + k);
    pending_small.erase(pending_small.begin(), pending_small.begin() + k);
    slot_jobs[slot] = batch_take;
    const double now = host_now();
    for (int32_t j : batch_take) res[j].t_place = now;
    round.push_back(Pending{-1, slot, pages_of(bytes), 0});
    batch_running = true;
  }

  // Completed jobs -> results + staged releases; returns how many staged.
  int64_t poll_completions() {
    int64_t k = 0;
    for (auto &q : inflight) {
      while (!q.empty()) {
        Running &r = q.front();
        if (hipEventQuery(r.ev_end) != hipSuccess) break;
        const double ts = dev_time(r.ev_start), te = dev_time(r.ev_end);
        auto done_one = [&](int32_t j) {
          res[j].t_start = ts;
          res[j].t_end = te;
          h_rel[k++] = j;
          finished += 1;
          cur_running -= 1;
          if (res[j].status == SCHED_OK) sum.completed += 1;
        };
        if (r.batch >= 0) {
          for (int32_t j : batch_jobs[r.batch]) done_one(j);
          batch_running = false;
        } else {
          done_one(r.job);
        }
        released_slots.push_back(r.slot);
        ev_free.push_back(r.ev_start);
        ev_free.push_back(r.ev_end);
        q.pop_front();
      }
    }
    return k;
  }

  // Releases the placements of the completed jobs: pages back to the pool,
  // charges back to the jobs.  Comes before the release of their
  // reservations on the same stream.
  int release_placements() {
    if (released_slots.empty()) return SCHED_OK;
    size_t n_jobs = 0;
    for (int32_t s : released_slots) n_jobs += slot_jobs[s].size();
    if (int rc = stage_room(released_slots.size(), n_jobs)) return rc;
    PgReq *d_rq;
    int32_t *d_j;
    int64_t *d_b;
    PgReq *rq = stage.take<PgReq>(released_slots.size(), &d_rq);
    int32_t *hj = stage.take<int32_t>(n_jobs, &d_j);
    int64_t *hb = stage.take<int64_t>(n_jobs, &d_b);
    size_t off = 0;
    for (size_t i = 0; i < released_slots.size(); ++i) {
      const int32_t s = released_slots[i];
      const std::vector<int32_t> &js = slot_jobs[s];
      rq[i] = PgReq{s, int32_t(js.size()), 0, int64_t(off)};
      for (size_t q = 0; q < js.size(); ++q) {
        hj[off + q] = js[q];
        hb[off + q] = job_bytes(J[js[q]]);
      }
      off += js.size();
    }
    if (int rc = pg_release(c, pt, int32_t(released_slots.size()), d_rq, d_j, d_b, stream_ctl))
      return rc;
    for (int32_t s : released_slots) {
      slot_jobs[s].clear();
      free_slots.push_back(s);
    }
    released_slots.clear();
    return SCHED_OK;
  }

  int run_realtime() {
    int64_t ai = 0;
    const double scale = o.time_scale > 0 ? o.time_scale : 1.0;
    while (finished < n) {
      const double now = host_now();
      bool changed = false;
      int64_t k = 0;
      while (ai < n && J[ai].arrival_s * scale <= now) {
        res[ai].t_arrive = J[ai].arrival_s * scale;
        const int64_t d = demand_of(ai);
        const int64_t jb = job_bytes(J[ai]);
        if (d > c->capacity || jb < 0 || jb > J[ai].demand || pages_of(jb) > PG_MAX_PAGES) {
          res[ai].status = d > c->capacity ? SCHED_E_TOOBIG : SCHED_E_INVALID;
          sum.rejected += 1;
          finished += 1;
        } else {
          h_job[k] = int32_t(ai);
          h_dem[k] = d;
          ++k;
        }
        ++ai;
      }
      if (k) {
        if (int rc = enqueue(k)) return rc;
        changed = true;
      }
      double t1 = host_now();
      const int64_t r = poll_completions();
      if (r) {
        if (int rc = release_placements()) return rc;
        if (int rc = release(r)) return rc;
        changed = true;
      }
      double t2 = host_now();
      sum.host_poll_s += t2 - t1;
      if (r) {
        if (int rc = launch_slot_waiters()) return rc;
        plan_batch();
        if (int rc = launch_round()) return rc;
      }
      t1 = host_now();
      sum.host_launch_s += t1 - t2;
      if (changed) {
        int64_t A = 0;
        if (int rc = pass(&A)) return rc;
        t2 = host_now();
        sum.host_pass_s += t2 - t1;
        if (A)
          if (int rc = launch_admitted(A, t2)) return rc;
        sum.host_launch_s += host_now() - t2;
        continue;
      }
      // idle: wait for the next arrival or a completion (short sleeps: a
      // completion is noticed within a few microseconds, which matters most
      // for exclusive serial runs, where every job waits for the last one)
      double wait = 5e-6;
      if (ai < n) wait = std::min(wait, std::max(0.0, J[ai].arrival_s * scale - now));
      if (wait > 2e-6) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
      sum.host_idle_s += host_now() - t1;
    }
    SCHED_HIP_TRY(hipDeviceSynchronize());
    return SCHED_OK;
  }

  int run_virtual() {
    // (time, kind: 0 release before 1 arrival, job)
    typedef std::tuple<double, int, int64_t> Ev;
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> pq;
    for (int64_t j = 0; j < n; ++j) pq.emplace(J[j].arrival_s, 1, j);
    while (!pq.empty()) {
      const Ev e = pq.top();
      pq.pop();
      const double t = std::get<0>(e);
      const int64_t j = std::get<2>(e);
      if (std::get<1>(e) == 0) {
        h_rel[0] = int32_t(j);
        if (int rc = release(1)) return rc;
        res[j].t_end = t;
        finished += 1;
        sum.completed += 1;
      } else {
        res[j].t_arrive = t;
        const int64_t d = demand_of(j);
        if (d > c->capacity) {
          res[j].status = SCHED_E_TOOBIG;
          sum.rejected += 1;
          finished += 1;
          continue;
        }
        h_job[0] = int32_t(j);
        h_dem[0] = d;
        if (int rc = enqueue(1)) return rc;
      }
      int64_t A = 0;
      if (int rc = pass(&A)) return rc;
      for (int64_t i = 0; i < A; ++i) {
        const int32_t a = h_adm[i];
        res[a].t_admit = t;
        res[a].t_place = t;
        res[a].t_start = t;
        pq.emplace(t + J[a].vdur_s, 0, int64_t(a));
      }
    }
    return SCHED_OK;
  }

  // Device-side results: digests, GEMM samples, placement statuses, and the
  // page tier's counters and end-of-run check.
  int collect() {
    SCHED_HIP_TRY(hipDeviceSynchronize());
    if (o.digest && n > 0) {
      std::vector<unsigned long long> dg(n);
      std::vector<float> sp(size_t(n) * GEMM_SAMPLES);
      SCHED_HIP_TRY(hipMemcpy(dg.data(), d_digest, sizeof(unsigned long long) * n,
                              hipMemcpyDeviceToHost));
      SCHED_HIP_TRY(hipMemcpy(sp.data(), d_samples, sizeof(float) * sp.size(), hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < n; ++i) {
        res[i].digest = dg[i];
        if (J[i].kind == SCHED_JOB_GEMM)
          for (int k = 0; k < GEMM_SAMPLES; ++k) res[i].sample[k] = sp[size_t(i) * GEMM_SAMPLES + k];
      }
    }
    if (!pt) return SCHED_OK;
    std::vector<int32_t> st(std::max<int64_t>(n, 1));
    SCHED_HIP_TRY(hipMemcpy(st.data(), d_place_st, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i)
      if (res[i].status == SCHED_OK && st[i] > 0) {  // admitted but not placed
        res[i].status = SCHED_E_NOMEM;
        sum.completed -= 1;
      }
    PgCounters pc{};
    if (int rc = pg_counters(pt, stream_ctl, &pc)) return rc;
    sum.violations += pc.violations + pc.over_admitted;
    sum.peak_pages = pc.peak_pages;
    sum.pages_left = pc.pages_used;
    sum.charged_left = pc.charged;
    int64_t bad = 0;
    if (pc.pages_used == 0 && pc.nodes_used == 0) {
      if (int rc = pg_check_free(pt, stream_ctl, &bad)) return rc;
    } else {
      bad = -1;  // placements left: the check needs every page back
    }
    sum.page_check = bad;
    return SCHED_OK;
  }

  void summarize() {
    std::vector<double> waits, turns;
    double last = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (res[j].status != SCHED_OK) continue;
      waits.push_back(res[j].t_place - res[j].t_arrive);
      turns.push_back(res[j].t_end - res[j].t_arrive);
      last = std::max(last, res[j].t_end);
    }
    auto pct = [](std::vector<double> v, double p) {
      if (v.empty()) return std::nan("");
      std::sort(v.begin(), v.end());
      int64_t k = int64_t(std::ceil(p * double(v.size()) / 100.0));
      k = std::max<int64_t>(k, 1);
      return v[size_t(k - 1)];
    };
    sum.p50_wait_s = pct(waits, 50);
    sum.p99_wait_s = pct(waits, 99);
    sum.p50_turn_s = pct(turns, 50);
    sum.p99_turn_s = pct(turns, 99);
    sum.makespan_s = last;
    sum.jobs_per_s = last > 0 ? double(sum.completed) / last : 0.0;
    // union of the jobs' device intervals
    std::vector<std::pair<double, double>> iv;
    for (int64_t j = 0; j < n; ++j)
      if (res[j].status == SCHED_OK && res[j].t_end > res[j].t_start)
        iv.emplace_back(res[j].t_start, res[j].t_end);
    std::sort(iv.begin(), iv.end());
    double busy = 0.0, a = 0.0, b = -1.0;
    for (const auto &x : iv) {
      if (x.first > b) {
        if (b > a) busy += b - a;
        a = x.first;
        b = x.second;
      } else if (x.second > b) {
        b = x.second;
      }
    }
    if (b > a) busy += b - a;
    sum.dev_busy_s = busy;
  }
};

}  // namespace

extern "C" int sched_serve(sched_ctx_t *c, int64_t n, const sched_job_desc_t *jobs,
                           const sched_serve_opts_t *opts, sched_job_result_t *results,
                           sched_serve_summary_t *summary) {
  if (!c || n < 0 || (n > 0 && (!jobs || !results)) || !opts || c->shared()) return SCHED_E_INVALID;
  std::unique_lock<CtxLock> lk(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (n > c->jb.max_jobs || opts->max_placed < 0) return SCHED_E_INVALID;
  for (int64_t i = 0; i < n; ++i)
    if (jobs[i].demand <= 0 || jobs[i].kind < 0 || jobs[i].kind > SCHED_JOB_HIST ||
        (i > 0 && jobs[i].arrival_s < jobs[i - 1].arrival_s))
      return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  // tenant charges live in the slab's per-tenant counters (tenants = jobs,
  // quotas = reservations); a context without a slab gets a small one
  if (!c->slab) {
    if (int rc = sched_slab_init(c, 13 << 20, c->jb.max_jobs)) return rc;
  } else if (!sched_slab_quota_is_reservation(c)) {
    return SCHED_E_INVALID;
  }
  lk.unlock();
  if (int rc = sched_reset(c)) return rc;
  lk.lock();
  // jobs 0..n-1 are the serving run's jobs (priorities are uploaded by init)
  if (c->sh->n_jobs < n) c->sh->n_jobs = int32_t(n);
  for (int64_t i = 0; i < n; ++i) results[i] = sched_job_result_t{};
  Serve s{};
  s.sum.tuned_from_cache = -1;
  s.c = c;
  s.J = jobs;
  s.n = n;
  s.o = *opts;
  s.res = results;
  int rc = s.init();
  if (rc == SCHED_OK) rc = opts->mode == SCHED_SERVE_VIRTUAL ? s.run_virtual() : s.run_realtime();
  if (rc == SCHED_OK) rc = s.collect();
  s.summarize();
  s.sum.wall_s = s.host_now();
  s.fini();
  c->sh->stats.violations += s.sum.violations;
  if (summary) *summary = s.sum;
  return rc;
}
