// Batched execution of small admitted jobs in one persistent launch.
//
// Launch and synchronisation costs dominate jobs of a few MiB (a 4 MiB triad
// moves its data in a few microseconds).  Admitted small jobs are described
// in a table; one persistent grid pulls (job, chunk) work items from an
// atomic counter and runs every step of the job's chunk: input fill, the
// triad sweeps and the result digest.  Each thread handles the same elements
// in every step, so a chunk needs no synchronisation between steps.
//
// The launch is a HIP graph captured once per (block, chunk) shape: a staging
// kernel copies the descriptor table from pinned host memory to the device
// and clears the work counter (a kernel, not a memset node), then the
// persistent kernel runs.  Replays only rewrite the pinned table.  Block and
// chunk sizes come from a small autotuner that times the candidates on the
// device and caches the winner in a JSON file.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "batch.h"
#include "common.h"

namespace schedk {

namespace {

__device__ __forceinline__ uint64_t splitmix(uint64_t s0, uint64_t i) {
  uint64_t z = s0 + (i + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Copies the table (header + descriptors + item offsets) from pinned host
// memory and resets the work counter.
__global__ void k_batch_stage(const BatchTable *__restrict__ host, BatchTable *__restrict__ dev) {
  const int n = host->n_desc;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    dev->n_desc = n;
    dev->n_items = host->n_items;
    dev->chunk = host->chunk;
    dev->map = host->map;
    dev->need = host->need;
    dev->work = 0;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dev->desc[i] = host->desc[i];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x)
    dev->item_off[i] = host->item_off[i];
}

// A work item is `chunk` elements of one job, chunk a divisor of 16384, so
// the item lies inside one 64 KiB window of each of its arrays (which start
// at 4 KiB boundaries): the item resolves its three windows once (pages.h)
// and every step below addresses through them.
__global__ void k_batch_run(BatchTable *__restrict__ t) {
  __shared__ long long s_item;
  __shared__ uint32_t sdir[PG_DIR];
  const int64_t n_items = t->n_items;
  const int n_desc = t->n_desc;
  const int64_t chunk = t->chunk;
  const PageMap m = t->map;
  const int64_t mapped = pm_pages(m);
  if (mapped < t->need) return;  // the placement failed: nothing is mapped
  const PgView v = pg_view(m, sdir, mapped);
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned long long it = add_relaxed(&t->work, 1ULL);
      s_item = it < (unsigned long long)n_items ? (long long)it : -1;
    }
    __syncthreads();
    const long long item = s_item;
    __syncthreads();
    if (item < 0) break;
    // the job owning this item: largest j with item_off[j] <= item
    int lo = 0, hi = n_desc;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (t->item_off[mid] <= item) lo = mid;
      else hi = mid;
    }
    const BatchDesc d = t->desc[lo];
    const int64_t e0 = (item - t->item_off[lo]) * chunk;
    const int64_t e1 = e0 + chunk < d.n ? e0 + chunk : d.n;
    const uint64_t s0 = d.seed << 32;
    const uint64_t wbase = uint64_t(4 * e0) & ~uint64_t(PG_BYTES - 1), end = uint64_t(4 * d.n);
    const uint32_t b0 = uint32_t(uint64_t(4 * e0) - wbase);
    const PgWin A = pg_win(v, d.oa + wbase, d.oa + end), B = pg_win(v, d.ob + wbase, d.ob + end),
                C = pg_win(v, d.oc + wbase, d.oc + end);
    // input fill (same element -> same thread in every step below)
    for (int64_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) {
      const uint32_t byte = b0 + 4 * uint32_t(i - e0);
      const uint64_t h = splitmix(s0, uint64_t(i));
      *reinterpret_cast<float *>(B.at(byte)) = 1.0f + float(h & 0xFFFF) * (1.0f / 65536.0f);
      *reinterpret_cast<float *>(C.at(byte)) = 1.0f + float((h >> 16) & 0xFFFF) * (1.0f / 65536.0f);
    }
    for (int it = 0; it < d.iters; ++it) {
      for (int64_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) {
        const uint32_t byte = b0 + 4 * uint32_t(i - e0);
        *reinterpret_cast<float *>(A.at(byte)) = *reinterpret_cast<const float *>(B.at(byte)) +
                                                 3.0f * *reinterpret_cast<const float *>(C.at(byte));
      }
    }
    unsigned long long dg = 0;
    if (d.digest)
      for (int64_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) {
        const uint32_t byte = b0 + 4 * uint32_t(i - e0);
        dg += digest_term(uint64_t(i), *reinterpret_cast<const uint32_t *>(A.at(byte)));
      }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dg += __shfl_xor(dg, off, WAVE);
    if (d.digest && (threadIdx.x & (WAVE - 1)) == 0 && dg) add_relaxed(d.digest, dg);
  }
}

}  // namespace

int batch_init(BatchEngine &b, int device, int max_desc) {
  b.device = device;
  b.max_desc = max_desc;
  const size_t bytes = BatchTable::bytes_for(max_desc);
  SCHED_HIP_TRY(hipHostMalloc(&b.h_table, bytes, hipHostMallocMapped));
  SCHED_HIP_TRY(hipHostGetDevicePointer((void **)&b.h_table_dev, b.h_table, 0));
  SCHED_HIP_TRY(hipMalloc(&b.d_table, bytes));
  BatchTable::layout(b.h_table, max_desc);
  // the device copy keeps its own pointers into device memory
  BatchTable tmp;
  BatchTable::layout_at(&tmp, (char *)b.d_table, max_desc);
  SCHED_HIP_TRY(hipMemcpy(b.d_table, &tmp, sizeof(BatchTable), hipMemcpyHostToDevice));
  // and the host copy's pointers as the device sees them
  BatchTable::layout_at(b.h_table, (char *)b.h_table_dev, max_desc);
  int cus = 0;
  SCHED_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  b.cus = cus;
  return SCHED_OK;
}

void batch_free(BatchEngine &b) {
  for (auto &g : b.graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  b.graphs.clear();
  if (b.h_table) (void)hipHostFree(b.h_table);
  if (b.d_table) (void)hipFree(b.d_table);
  b.h_table = nullptr;
  b.d_table = nullptr;
}

static int launch_direct(BatchEngine &b, int block, int grid, hipStream_t s) {
  k_batch_stage<<<std::max(1, std::min(64, b.max_desc / 256 + 1)), 256, 0, s>>>(b.h_table_dev,
                                                                               b.d_table);
  SCHED_HIP_TRY(hipGetLastError());
  k_batch_run<<<grid, block, 0, s>>>(b.d_table);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

static int graph_for(BatchEngine &b, int block, int grid, hipStream_t s, hipGraphExec_t *out) {
  for (auto &g : b.graphs)
    if (g.block == block && g.grid == grid) {
      *out = g.exec;
      return SCHED_OK;
    }
  BatchGraph g;
  g.block = block;
  g.grid = grid;
  SCHED_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = launch_direct(b, block, grid, s);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &graph);
  if (rc) return rc;
  SCHED_HIP_TRY(e);
  g.graph = graph;
  SCHED_HIP_TRY(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
  b.graphs.push_back(g);
  *out = g.exec;
  return SCHED_OK;
}

// Fills the pinned table from descriptors; chunk in elements.
int batch_fill(BatchEngine &b, const std::vector<BatchDesc> &descs, int64_t chunk, const PageMap &map,
               int64_t need) {
  if ((int)descs.size() > b.max_desc) return SCHED_E_INVALID;
  // a work item inside one 64 KiB window of each array: see k_batch_run
  if (chunk <= 0 || chunk > PG_BYTES / 4 || (PG_BYTES / 4) % chunk) return SCHED_E_INVALID;
  for (const BatchDesc &d : descs)
    if ((d.oa | d.ob | d.oc) & 4095) return SCHED_E_INVALID;
  BatchTable *t = b.h_table;
  t->n_desc = int(descs.size());
  t->chunk = chunk;
  t->map = map;
  t->need = need;
  int64_t acc = 0;
  BatchDesc *hd = (BatchDesc *)((char *)t + BatchTable::desc_offset());
  int64_t *ho = (int64_t *)((char *)t + BatchTable::off_offset(b.max_desc));
  for (size_t i = 0; i < descs.size(); ++i) {
    hd[i] = descs[i];
    ho[i] = acc;
    acc += (descs[i].n + chunk - 1) / chunk;
  }
  ho[descs.size()] = acc;
  t->n_items = acc;
  return SCHED_OK;
}

int batch_launch(BatchEngine &b, hipStream_t s, bool use_graph) {
  const int block = b.block > 0 ? b.block : 256;
  const int grid = b.cus * (b.per_cu > 0 ? b.per_cu : 4);
  if (!use_graph) return launch_direct(b, block, grid, s);
  hipGraphExec_t exec = nullptr;
  if (int rc = graph_for(b, block, grid, s, &exec)) return rc;
  SCHED_PROF_LAUNCH_GRAPH("k_batch_graph", s, hipGraphLaunch(exec, s));
  return SCHED_OK;
}

// Autotuner: times each (block, chunk) candidate on a synthetic batch of
// `n_jobs` triads of `job_elems` elements and keeps the fastest.  The result
// is cached in `cache_path` (JSON) when given.
int batch_autotune(BatchEngine &b, const char *cache_path, hipStream_t s) {
  if (cache_path && *cache_path) {
    FILE *f = fopen(cache_path, "r");
    if (f) {
      int blk = 0, per = 0;
      long long ch = 0;
      char buf[512] = {0};
      size_t nr = fread(buf, 1, sizeof(buf) - 1, f);
      fclose(f);
      buf[nr] = 0;
      const char *pb = strstr(buf, "\"block\":"), *pc = strstr(buf, "\"chunk\":"),
                 *pp = strstr(buf, "\"per_cu\":");
      if (pb && pc && pp && sscanf(pb, "\"block\": %d", &blk) == 1 &&
          sscanf(pc, "\"chunk\": %lld", &ch) == 1 && sscanf(pp, "\"per_cu\": %d", &per) == 1 &&
          blk > 0 && per > 0 && ch > 0 && ch <= PG_BYTES / 4 && (PG_BYTES / 4) % ch == 0) {
        b.block = blk;
        b.chunk = ch;
        b.per_cu = per;
        b.tuned = true;
        b.from_cache = true;
        return SCHED_OK;
      }
    }
  }
  const int n_jobs = std::min(b.max_desc, 256);
  const int64_t job_elems = (4 << 20) / 12;  // 4 MiB triads
  const int64_t arr = (job_elems * 4 + 4095) / 4096 * 4096;
  char *arena = nullptr;
  unsigned long long *dig = nullptr;
  SCHED_HIP_TRY(hipMalloc(&arena, 3 * arr * n_jobs));
  SCHED_HIP_TRY(hipMalloc(&dig, sizeof(unsigned long long) * n_jobs));
  PgIdentity idm;
  if (int rc = pg_identity(arena, 3 * arr * n_jobs, s, &idm)) return rc;
  const int64_t need = (3 * arr * n_jobs + PG_BYTES - 1) / PG_BYTES;
  std::vector<BatchDesc> ds(n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    const uint64_t base = uint64_t(i) * 3 * arr;
    ds[i] = BatchDesc{base, base + arr, base + 2 * arr, job_elems, uint64_t(i + 1), 10, 0, dig + i};
  }
  const int blocks[] = {256, 512, 1024};
  const int64_t chunks[] = {1 << 12, 1 << 13, 1 << 14};  // divisors of a 64 KiB window
  const int pers[] = {2, 4, 8};
  double best = 1e30;
  hipEvent_t e0, e1;
  SCHED_HIP_TRY(hipEventCreate(&e0));
  SCHED_HIP_TRY(hipEventCreate(&e1));
  for (int blk : blocks)
    for (int64_t ch : chunks)
      for (int per : pers) {
        if (blk * per > 2048) continue;  // at most 32 waves per CU
        b.block = blk;
        b.per_cu = per;
        if (int rc = batch_fill(b, ds, ch, idm.map, need)) return rc;
        if (int rc = batch_launch(b, s, false)) return rc;  // warm
        SCHED_HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r)
          if (int rc = batch_launch(b, s, false)) return rc;
        SCHED_HIP_TRY(hipEventRecord(e1, s));
        SCHED_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0;
        SCHED_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          b.chunk = ch;
          b.best_block = blk;
          b.best_per_cu = per;
        }
      }
  b.block = b.best_block;
  b.per_cu = b.best_per_cu;
  b.tuned = true;
  b.from_cache = false;
  b.tune_ms = best / 3;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  pg_identity_free(&idm);
  (void)hipFree(arena);
  (void)hipFree(dig);
  if (cache_path && *cache_path) {
    FILE *f = fopen(cache_path, "w");
    if (f) {
      fprintf(f,
              "{\"block\": %d, \"chunk\": %lld, \"per_cu\": %d, \"batch_ms\": %.4f, "
              "\"probe\": \"%d triads x %lld fp32 x 3 arrays, 10 sweeps\"}\n",
              b.block, (long long)b.chunk, b.per_cu, b.tune_ms, n_jobs, (long long)job_elems);
      fclose(f);
    }
  }
  return SCHED_OK;
}

}  // namespace schedk
