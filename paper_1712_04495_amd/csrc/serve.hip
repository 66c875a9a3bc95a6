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
#include <map>
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

__global__ void k_digest(const uint32_t *__restrict__ w, int64_t n, unsigned long long *out) {
  unsigned long long s = 0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    s += w[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
  if ((threadIdx.x & (WAVE - 1)) == 0 && s) add_relaxed(out, s);
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}

int64_t rup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Buffer bytes a job allocates; must not exceed its declared demand.
int64_t job_bytes(const sched_job_desc_t &j) {
  switch (j.kind) {
    case SCHED_JOB_TRIAD: return 3 * rup(4 * j.size, 4096);
    case SCHED_JOB_GEMM: return 2 * rup(2 * j.size * j.size, 4096) + rup(4 * j.size * j.size, 4096);
    case SCHED_JOB_HIST: return rup(4 * j.size, 4096) + rup(4 * SCHED_HIST_BINS, 4096);
    default: return -1;
  }
}

int grid_of(int64_t n, int cap) {
  int64_t g = (n + 255) / 256;
  return int(std::max<int64_t>(1, std::min<int64_t>(g, cap)));
}

struct Running {
  int32_t job;          // -1 for a batch
  int32_t batch;        // index into batch_jobs, -1 for a single job
  uint64_t off, len;    // arena range (len 0: none)
  hipEvent_t ev_start, ev_end;
  hipStream_t stream;
};

// Device memory of the admitted jobs: one allocation of the scheduler's
// capacity, carved on the host best fit with coalescing of free neighbours
// (4 KiB granules).  Admission keeps the sum of the live demands within the
// capacity; a job whose demand fits but finds no contiguous range waits
// until a running job ends (when nothing runs the arena is one free range,
// so every admitted job eventually gets its memory).  A range returns to the
// arena only when its job's completion has been observed.
class Arena {
 public:
  char *base = nullptr;
  uint64_t size = 0;
  bool alloc(uint64_t len, uint64_t *off) {
    auto it = by_len.lower_bound(len);
    if (it == by_len.end()) return false;
    const uint64_t L = it->first, o = it->second;
    by_len.erase(it);
    by_off.erase(o);
    if (L > len) put(o + len, L - len);
    *off = o;
    return true;
  }
  void release(uint64_t off, uint64_t len) {
    auto nx = by_off.lower_bound(off);
    if (nx != by_off.end() && off + len == nx->first) {
      drop_len(nx->second, nx->first);
      len += nx->second;
      nx = by_off.erase(nx);
    }
    if (nx != by_off.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        drop_len(pv->second, pv->first);
        off = pv->first;
        len += pv->second;
        by_off.erase(pv);
      }
    }
    put(off, len);
  }
  void reset() {
    by_off.clear();
    by_len.clear();
    if (size) put(0, size);
  }

 private:
  std::map<uint64_t, uint64_t> by_off;       // offset -> length
  std::multimap<uint64_t, uint64_t> by_len;  // length -> offset
  void put(uint64_t off, uint64_t len) {
    by_off.emplace(off, len);
    by_len.emplace(len, off);
  }
  void drop_len(uint64_t len, uint64_t off) {
    auto r = by_len.equal_range(len);
    for (auto it = r.first; it != r.second; ++it)
      if (it->second == off) {
        by_len.erase(it);
        return;
      }
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
  Arena arena;
  std::deque<int32_t> deferred;  // admitted, waiting for a contiguous range

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
    if (o.mode == SCHED_SERVE_REALTIME) {
      arena.size = uint64_t(rup(c->capacity, 4096));
      SCHED_HIP_TRY(hipMalloc(&arena.base, arena.size));
      arena.reset();
    }
    SCHED_HIP_TRY(hipMalloc(&d_digest, sizeof(unsigned long long) * std::max<int64_t>(n, 1)));
    k_zero_u64<<<grid_of(n, 1024), 256, 0, stream_ctl>>>(d_digest, n);
    SCHED_HIP_TRY(hipGetLastError());
    h_cap = std::max<int64_t>(n, 1);
    SCHED_HIP_TRY(hipHostMalloc(&h_job, sizeof(int32_t) * h_cap, hipHostMallocDefault));
    SCHED_HIP_TRY(hipHostMalloc(&h_dem, sizeof(int64_t) * h_cap, hipHostMallocDefault));
    SCHED_HIP_TRY(hipHostMalloc(&h_adm, sizeof(int32_t) * h_cap, hipHostMallocDefault));
    SCHED_HIP_TRY(hipMalloc(&d_job, sizeof(int32_t) * h_cap));
    SCHED_HIP_TRY(hipMalloc(&d_dem, sizeof(int64_t) * h_cap));
    SCHED_HIP_TRY(hipHostMalloc(&h_rel, sizeof(int32_t) * h_cap, hipHostMallocDefault));
    SCHED_HIP_TRY(hipMalloc(&d_rel, sizeof(int32_t) * h_cap));
    // priorities of jobs 0..n-1
    for (int64_t i = 0; i < n; ++i) h_job[i] = J[i].priority;
    SCHED_HIP_TRY(hipMemcpyAsync(c->d_prio_of_job, h_job, sizeof(int32_t) * n, hipMemcpyHostToDevice,
                                 stream_ctl));
    if (o.batch_small && !o.serial) {
      beng = new BatchEngine();
      if (int rc = batch_init(*beng, c->device, 8192)) return rc;
      if (int rc = batch_autotune(*beng, o.tune_cache, bstream)) return rc;
      sum.tuned_block = beng->block;
      sum.tuned_chunk = beng->chunk;
      sum.tuned_per_cu = beng->per_cu;
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
    if (arena.base) (void)hipFree(arena.base);
    arena.base = nullptr;
    if (bstream) (void)hipStreamDestroy(bstream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (d_digest) (void)hipFree(d_digest);
    if (h_job) (void)hipHostFree(h_job);
    if (h_dem) (void)hipHostFree(h_dem);
    if (h_adm) (void)hipHostFree(h_adm);
    if (d_job) (void)hipFree(d_job);
    if (d_dem) (void)hipFree(d_dem);
    if (h_rel) (void)hipHostFree(h_rel);
    if (d_rel) (void)hipFree(d_rel);
    if (beng) {
      batch_free(*beng);
      delete beng;
    }
  }

  int64_t demand_of(int64_t j) const { return o.serial ? c->capacity : J[j].demand; }

  // Request intake: appends k staged (job, demand) pairs to the queue.
  int enqueue(int64_t k) {
    if (k == 0) return SCHED_OK;
    if (c->tail_h - c->head_h + k > c->q.capacity) return SCHED_E_NOMEM;
    SCHED_HIP_TRY(hipMemcpyAsync(d_job, h_job, sizeof(int32_t) * k, hipMemcpyHostToDevice, stream_ctl));
    SCHED_HIP_TRY(hipMemcpyAsync(d_dem, h_dem, sizeof(int64_t) * k, hipMemcpyHostToDevice, stream_ctl));
    if (int rc = adm_enqueue(c->eng, c->q, c->tail_h, k, d_job, d_dem, c->d_prio_of_job, c->seq_next,
                             stream_ctl))
      return rc;
    c->seq_next += k;
    c->tail_h += k;
    return SCHED_OK;
  }

  int release(int64_t k) {
    if (k == 0) return SCHED_OK;
    SCHED_HIP_TRY(hipMemcpyAsync(d_rel, h_rel, sizeof(int32_t) * k, hipMemcpyHostToDevice, stream_ctl));
    k_release_list<<<grid_of(k, 64), 256, 0, stream_ctl>>>(c->eng.d_ctl, c->jb, d_rel, k);
    SCHED_HIP_TRY(hipGetLastError());
    return SCHED_OK;
  }

  // One admission pass; the admitted job ids (queue order) land in h_adm.
  int pass(int64_t *n_adm) {
    sched_pass_result_t pr{};
    if (int rc = sched_run_pass_locked(c, stream_ctl, &pr)) return rc;
    const int64_t A = pr.admitted;
    if (A > 0) {
      SCHED_HIP_TRY(hipMemcpyAsync(h_adm, c->q.adm_job, sizeof(int32_t) * A, hipMemcpyDeviceToHost,
                                   stream_ctl));
      SCHED_HIP_TRY(hipStreamSynchronize(stream_ctl));
    }
    sum.passes += 1;
    sum.peak_used = std::max<int64_t>(sum.peak_used, c->used_h);
    *n_adm = A;
    return SCHED_OK;
  }

  // Buffers and work of one job on stream s.  Returns the allocation so the
  // caller can free it after completion (stream-ordered free is enqueued
  // here as well).
  int launch_single(int32_t j, hipStream_t s, Running *r) {
    const sched_job_desc_t &d = J[j];
    r->job = j;
    r->batch = -1;
    r->stream = s;
    const int64_t bytes = job_bytes(d);
    if (bytes < 0 || bytes > d.demand) return SCHED_E_INVALID;
    const uint64_t len = uint64_t(rup(std::max<int64_t>(bytes, 1), 4096));
    uint64_t off = 0;
    const double ta = host_now();
    const bool got = arena.alloc(len, &off);
    sum.host_alloc_s += host_now() - ta;
    if (!got) return SCHED_NOT_READY;  // no contiguous range yet: the caller defers
    r->off = off;
    r->len = len;
    r->ev_start = take_event();
    r->ev_end = take_event();
    SCHED_HIP_TRY(hipEventRecord(r->ev_start, s));
    char *p = arena.base + off;
    unsigned long long *dg = d_digest + j;
    if (d.kind == SCHED_JOB_TRIAD) {
      const int64_t n4 = rup(4 * d.size, 4096);
      float *a = (float *)p, *b = (float *)(p + n4), *cc = (float *)(p + 2 * n4);
      if (int rc = sched_triad_fill(b, cc, d.size, d.seed, s)) return rc;
      if (int rc = sched_triad(a, b, cc, 3.0f, d.size, o.iters, s)) return rc;
      if (o.digest) k_digest<<<grid_of(d.size, 2048), 256, 0, s>>>((const uint32_t *)a, d.size, dg);
    } else if (d.kind == SCHED_JOB_GEMM) {
      const int64_t N = d.size, ab = rup(2 * N * N, 4096);
      uint16_t *A = (uint16_t *)p, *B = (uint16_t *)(p + ab);
      float *C = (float *)(p + 2 * ab);
      if (int rc = sched_gemm_fill(A, N, N, 2 * d.seed, s)) return rc;
      if (int rc = sched_gemm_fill(B, N, N, 2 * d.seed + 1, s)) return rc;
      if (int rc = sched_gemm_bf16(A, B, C, N, N, N, s)) return rc;
      if (o.digest) k_digest<<<grid_of(N * N, 2048), 256, 0, s>>>((const uint32_t *)C, N * N, dg);
    } else {
      const int64_t kb = rup(4 * d.size, 4096);
      uint32_t *keys = (uint32_t *)p, *bins = (uint32_t *)(p + kb);
      if (int rc = sched_hist_fill(keys, d.size, d.seed, s)) return rc;
      if (int rc = sched_hist(keys, d.size, SCHED_HIST_BINS - 1, bins, s)) return rc;
      if (o.digest) k_digest<<<1, 256, 0, s>>>(bins, SCHED_HIST_BINS, dg);
    }
    SCHED_HIP_TRY(hipGetLastError());
    SCHED_HIP_TRY(hipEventRecord(r->ev_end, s));
    return SCHED_OK;
  }

  // Small triads admitted together: one arena, one persistent launch.
  int launch_batch(const std::vector<int32_t> &jobs, Running *r) {
    r->job = -1;
    r->batch = int32_t(batch_jobs.size());
    r->stream = bstream;
    uint64_t total = 0;
    for (int32_t j : jobs) total += uint64_t(job_bytes(J[j]));  // whole pages per array
    uint64_t off = 0;
    const double ta = host_now();
    const bool got = arena.alloc(std::max<uint64_t>(total, 4096), &off);
    sum.host_alloc_s += host_now() - ta;
    if (!got) return SCHED_NOT_READY;
    r->off = off;
    r->len = std::max<uint64_t>(total, 4096);
    r->ev_start = take_event();
    r->ev_end = take_event();
    SCHED_HIP_TRY(hipEventRecord(r->ev_start, bstream));
    std::vector<BatchDesc> ds;
    ds.reserve(jobs.size());
    char *p = arena.base + off;
    for (int32_t j : jobs) {
      const int64_t n4 = rup(4 * J[j].size, 4096);
      ds.push_back(BatchDesc{(float *)p, (float *)(p + n4), (float *)(p + 2 * n4), J[j].size,
                             J[j].seed, o.iters, 0, d_digest + j});
      res[j].batched = 1;
      p += job_bytes(J[j]);
    }
    // the pinned table is rewritten only when no batch is in flight
    if (int rc = batch_fill(*beng, ds, beng->chunk)) return rc;
    if (int rc = batch_launch(*beng, bstream, o.use_graph != 0)) return rc;
    SCHED_HIP_TRY(hipEventRecord(r->ev_end, bstream));
    batch_running = true;
    sum.batches += 1;
    sum.batched_jobs += int64_t(jobs.size());
    batch_jobs.push_back(jobs);
    return SCHED_OK;
  }

  int launch_admitted(int64_t A, double now) {
    for (int64_t i = 0; i < A; ++i) {
      const int32_t j = h_adm[i];
      res[j].t_admit = now;
      if (beng && J[j].kind == SCHED_JOB_TRIAD && J[j].demand < o.small_bytes) {
        pending_small.push_back(j);
        continue;
      }
      if (!deferred.empty()) {  // keep admission order behind jobs already waiting
        deferred.push_back(j);
        continue;
      }
      if (int rc = start_single(j)) return rc;
    }
    if (int rc = maybe_launch_batch()) return rc;
    sum.max_running = std::max<int64_t>(sum.max_running, cur_running);
    return SCHED_OK;
  }

  // The job stream with the least expected backlog: the sum of the nominal
  // durations of the jobs still in flight on it (ties in round-robin order).
  // Streams run their jobs in order, so a short job placed behind a long one
  // would hold its reservation until the long one ends.
  size_t pick_stream() const {
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
    double t = 0.0;
    for (const Running &r : inflight[si])
      if (r.job >= 0) t += J[r.job].vdur_s;
    return t;
  }

  // Launches admitted job j, or defers it while no contiguous range fits.
  int start_single(int32_t j) {
    Running r{};
    const size_t si = pick_stream();
    const int rc = launch_single(j, streams[si], &r);
    if (rc == SCHED_NOT_READY) {
      deferred.push_back(j);
      sum.deferred += 1;
      return SCHED_OK;
    }
    if (rc) return rc;
    ++next_stream;
    inflight[si].push_back(r);
    cur_running += 1;
    return SCHED_OK;
  }

  // Deferred jobs, oldest first, as long as ranges fit.
  int launch_deferred() {
    while (!deferred.empty()) {
      const int32_t j = deferred.front();
      Running r{};
      const size_t si = pick_stream();
      const int rc = launch_single(j, streams[si], &r);
      if (rc == SCHED_NOT_READY) break;
      if (rc) return rc;
      deferred.pop_front();
      ++next_stream;
      inflight[si].push_back(r);
      cur_running += 1;
    }
    sum.max_running = std::max<int64_t>(sum.max_running, cur_running);
    return SCHED_OK;
  }

  int maybe_launch_batch() {
    if (!beng || batch_running || pending_small.empty()) return SCHED_OK;
    // as many of the waiting small jobs as one contiguous range holds
    size_t k = std::min<size_t>(pending_small.size(), size_t(beng->max_desc));
    Running r{};
    std::vector<int32_t> take;
    for (;;) {
      take.assign(pending_small.begin(), pending_small.begin() + k);
      const int rc = launch_batch(take, &r);
      if (rc == SCHED_OK) break;
      if (rc != SCHED_NOT_READY) return rc;
      if (k == 1) return SCHED_OK;  // retried after the next completion
      k /= 2;
    }
    pending_small.erase(pending_small.begin(), pending_small.begin() + k);
    inflight.back().push_back(r);
    cur_running += int64_t(take.size());
    sum.max_running = std::max<int64_t>(sum.max_running, cur_running);
    return SCHED_OK;
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
        if (r.len) arena.release(r.off, r.len);
        ev_free.push_back(r.ev_start);
        ev_free.push_back(r.ev_end);
        q.pop_front();
      }
    }
    return k;
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
        if (d > c->capacity || job_bytes(J[ai]) < 0 || job_bytes(J[ai]) > J[ai].demand) {
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
        if (int rc = release(r)) return rc;
        changed = true;
      }
      double t2 = host_now();
      sum.host_poll_s += t2 - t1;
      if (r)
        if (int rc = launch_deferred()) return rc;
      if (int rc = maybe_launch_batch()) return rc;
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
        res[a].t_start = t;
        pq.emplace(t + J[a].vdur_s, 0, int64_t(a));
      }
    }
    return SCHED_OK;
  }

  void summarize() {
    std::vector<double> waits, turns;
    double last = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (res[j].status != SCHED_OK) continue;
      waits.push_back(res[j].t_admit - res[j].t_arrive);
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
  if (!c || n < 0 || (n > 0 && (!jobs || !results)) || !opts) return SCHED_E_INVALID;
  std::unique_lock<std::mutex> lk(c->mu);
  if (int rc = sched_settle_reset_locked(c)) return rc;
  if (n > c->jb.max_jobs) return SCHED_E_INVALID;
  for (int64_t i = 0; i < n; ++i)
    if (jobs[i].demand <= 0 || jobs[i].kind < 0 || jobs[i].kind > SCHED_JOB_HIST ||
        (i > 0 && jobs[i].arrival_s < jobs[i - 1].arrival_s))
      return SCHED_E_INVALID;
  SCHED_HIP_TRY(hipSetDevice(c->device));
  lk.unlock();
  if (int rc = sched_reset(c)) return rc;
  lk.lock();
  // jobs 0..n-1 are the serving run's jobs (priorities are uploaded by init)
  if (c->n_jobs < n) c->n_jobs = int32_t(n);
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
  if (rc == SCHED_OK && opts->digest && n > 0) {
    std::vector<unsigned long long> dg(n);
    if (hipMemcpy(dg.data(), s.d_digest, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost) ==
        hipSuccess)
      for (int64_t i = 0; i < n; ++i) results[i].digest = dg[i];
    else
      rc = SCHED_E_INTERNAL;
  }
  s.summarize();
  s.sum.wall_s = s.host_now();
  s.fini();
  c->stats.violations += s.sum.violations;
  if (summary) *summary = s.sum;
  return rc;
}
