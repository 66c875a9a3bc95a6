// Queue order for the priority policies (Sec. V, Policies 3 and 4): before a
// pass, the live queue [head, tail) is stably sorted by priority (lower value
// first).  Within one priority the previous order is kept, and since older
// entries of a class always precede newer arrivals, that order is arrival
// order: the pass then walks the queue in (priority, arrival) order.
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "runtime.h"

using namespace schedk;

namespace {

__global__ void k_prio_gather(QueueArrays q, int64_t head, int64_t n, int32_t *keys, int64_t *idx) {
  const int64_t mask = q.capacity - 1;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    keys[i] = q.prio[(head + i) & mask];
    idx[i] = i;
  }
}

// tmp <- queue entries in sorted order
__global__ void k_prio_permute(QueueArrays q, int64_t head, int64_t n, const int64_t *order,
                               int64_t *t_dem, int32_t *t_job, int32_t *t_prio, int64_t *t_seq) {
  const int64_t mask = q.capacity - 1;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t src = (head + order[i]) & mask;
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

struct PrioTmp {
  int32_t *keys_in, *keys_out, *t_job, *t_prio;
  int64_t *idx_in, *idx_out, *t_dem, *t_seq;
  void *cub;
  size_t cub_bytes;
  int64_t cap;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

int sched_priority_reorder_locked(sched_ctx *c, hipStream_t s) {
  const int64_t n = c->tail_h - c->head_h;
  if (n <= 1) return SCHED_OK;
  size_t cub_bytes = 0;
  SCHED_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, cub_bytes, (int32_t *)nullptr,
                                                   (int32_t *)nullptr, (int64_t *)nullptr,
                                                   (int64_t *)nullptr, int(n), 0, 32, s));
  const size_t need = 4 * align256(sizeof(int32_t) * n) + 4 * align256(sizeof(int64_t) * n) +
                      align256(cub_bytes);
  if (c->prio_tmp_bytes < need) {
    if (c->prio_tmp) (void)hipFree(c->prio_tmp);
    c->prio_tmp = nullptr;
    c->prio_tmp_bytes = 0;
    SCHED_HIP_TRY(hipMalloc(&c->prio_tmp, need));
    c->prio_tmp_bytes = need;
  }
  char *p = (char *)c->prio_tmp;
  auto take = [&](size_t bytes) {
    char *r = p;
    p += align256(bytes);
    return r;
  };
  PrioTmp t;
  t.keys_in = (int32_t *)take(sizeof(int32_t) * n);
  t.keys_out = (int32_t *)take(sizeof(int32_t) * n);
  t.t_job = (int32_t *)take(sizeof(int32_t) * n);
  t.t_prio = (int32_t *)take(sizeof(int32_t) * n);
  t.idx_in = (int64_t *)take(sizeof(int64_t) * n);
  t.idx_out = (int64_t *)take(sizeof(int64_t) * n);
  t.t_dem = (int64_t *)take(sizeof(int64_t) * n);
  t.t_seq = (int64_t *)take(sizeof(int64_t) * n);
  t.cub = take(cub_bytes);
  const int grid = int(std::min<int64_t>((n + 255) / 256, 2048));
  k_prio_gather<<<grid, 256, 0, s>>>(c->q, c->head_h, n, t.keys_in, t.idx_in);
  SCHED_HIP_TRY(hipGetLastError());
  size_t cb = cub_bytes;
  SCHED_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(t.cub, cb, t.keys_in, t.keys_out, t.idx_in,
                                                   t.idx_out, int(n), 0, 32, s));
  k_prio_permute<<<grid, 256, 0, s>>>(c->q, c->head_h, n, t.idx_out, t.t_dem, t.t_job, t.t_prio,
                                      t.t_seq);
  SCHED_HIP_TRY(hipGetLastError());
  k_prio_store<<<grid, 256, 0, s>>>(c->q, c->head_h, n, t.t_dem, t.t_job, t.t_prio, t.t_seq);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}
