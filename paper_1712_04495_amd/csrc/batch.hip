// Batched execution of small admitted jobs in persistent launches.
//
// Launch and synchronisation costs dominate jobs of a few MiB (a 4 MiB triad
// moves its data in a few microseconds, a 512^3 GEMM is 0.27 GFLOP).
// Admitted small jobs of every kind are described in a table, and persistent
// grids pull (job, item) work from atomic counters.  A triad's item is a
// chunk on which it runs every step of the job -- input fill, the sweeps and
// the result digest -- with each thread on the same elements in every step,
// so the chunk needs no synchronisation.  Histograms and GEMMs have steps
// whose items read what other items wrote (bins zeroed before they are
// counted into, operands filled before the multiply, the output complete
// before its digest).  Those steps are separate phases (batch.h), one launch
// each, so ordering and visibility come from the kernel boundaries rather
// than from device-wide flags and cache write-backs inside one launch.
//
// The launches form a HIP graph captured once per shape: a staging kernel
// copies the descriptor table from pinned host memory to the device and
// clears the work counters (a kernel, not a memset node), then the phase
// launches run (phases 1 and 2 only when the batch has a histogram or a
// GEMM).  Replays only rewrite the pinned table.  The shapes come from a
// small autotuner that times candidates on the device and caches the winners
// in a JSON file: block size, workgroups per CU and chunk of the streaming
// phase; GEMM tile edge and workgroups per CU of phase 1.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "batch.h"
#include "common.h"

namespace schedk {

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int P12_THREADS = 256;  // phases 1 and 2: four waves
constexpr int GLR = 72;           // bf16 per LDS row of a GEMM k-tile (64 + 8: no bank aliasing)
constexpr int P2_PER_CU = 4;

// Copies the table (header, descriptors, item offsets of every phase) from
// pinned host memory and resets the work counters.
__global__ void k_batch_stage(const BatchTable *__restrict__ host, BatchTable *__restrict__ dev) {
  const int n = host->n_desc;
  const int stride = host->stride;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    dev->n_desc = n;
    dev->chunk = host->chunk;
    for (int p = 0; p < BATCH_PHASES; ++p) {
      dev->n_items[p] = host->n_items[p];
      dev->work[p] = 0;
    }
    dev->map = host->map;
    dev->need = host->need;
    dev->tile = host->tile;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dev->desc[i] = host->desc[i];
  for (int p = 0; p < BATCH_PHASES; ++p)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x)
      dev->item_off[p * stride + i] = host->item_off[p * stride + i];
}

// The job owning work item x of a phase: the largest j with off[j] <= x
// (jobs without items in the phase have off[j] == off[j + 1]).
__device__ __forceinline__ int job_of(const int64_t *__restrict__ off, int n, int64_t x) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Pulls the items of phase p until none is left and runs f(desc, item index
// within the job's share of the phase) with the whole workgroup.  The two
// barriers around the claim also separate one item's LDS use from the next.
template <typename F>
__device__ __forceinline__ void pull_items(BatchTable *__restrict__ t, int p, long long *s_item,
                                           F f) {
  const int64_t n_items = t->n_items[p];
  const int64_t *off = t->item_off + int64_t(p) * t->stride;
  const int n_desc = t->n_desc;
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned long long it = add_relaxed(&t->work[p], 1ULL);
      *s_item = it < (unsigned long long)n_items ? (long long)it : -1;
    }
    __syncthreads();
    const long long item = *s_item;
    __syncthreads();
    if (item < 0) break;
    const int j = job_of(off, n_desc, item);
    const BatchDesc d = t->desc[j];
    f(d, int64_t(item) - off[j]);
  }
}

__device__ __forceinline__ void add_digest(const BatchDesc &d, unsigned long long dg) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dg += __shfl_xor(dg, off, WAVE);
  if (d.digest && (threadIdx.x & (WAVE - 1)) == 0 && dg) add_relaxed(d.digest, dg);
}

// ---- phase 0 ----------------------------------------------------------------
// A triad chunk of `chunk` elements (a divisor of 16384), which lies inside
// one 64 KiB window of each of its arrays (they start at 4 KiB boundaries):
// the chunk resolves its three windows once (pages.h), every step below
// addresses through them, and each thread keeps its elements in every step.
__device__ __forceinline__ void triad_item(const PgView &v, const BatchDesc &d, int64_t q,
                                           int64_t chunk) {
  const int64_t e0 = q * chunk;
  const int64_t e1 = e0 + chunk < d.n ? e0 + chunk : d.n;
  const uint64_t s0 = d.seed << 32;
  const uint64_t wbase = uint64_t(4 * e0) & ~uint64_t(PG_BYTES - 1), end = uint64_t(4 * d.n);
  const uint32_t b0 = uint32_t(uint64_t(4 * e0) - wbase);
  const PgWin A = pg_win(v, d.o0 + wbase, d.o0 + end), B = pg_win(v, d.o1 + wbase, d.o1 + end),
              C = pg_win(v, d.o2 + wbase, d.o2 + end);
  for (int64_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) {
    const uint32_t byte = b0 + 4 * uint32_t(i - e0);
    const uint64_t h = splitmix_at(s0, uint64_t(i));
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
  add_digest(d, dg);
}

// The 4096 bins of a histogram (16 KiB from a 4 KiB boundary: one window).
__device__ __forceinline__ PgWin bins_win(const PgView &v, const BatchDesc &d) {
  return pg_win(v, d.o1, d.o1 + 4 * uint64_t(SCHED_HIST_BINS));
}

__device__ __forceinline__ void hist_zero(const PgView &v, const BatchDesc &d) {
  const PgWin W = bins_win(v, d);
  for (int b = threadIdx.x; b < SCHED_HIST_BINS; b += blockDim.x)
    *reinterpret_cast<uint32_t *>(W.at(4 * b)) = 0;
}

// Page q of the GEMM operands (pages of A, then pages of B^T): element i of
// an operand is (low byte of SplitMix64 output i - 128) / 64 in bf16, A from
// state (2 seed) << 32 and B^T from (2 seed + 1) << 32.
__device__ __forceinline__ void gemm_fill_page(const PgView &v, const BatchDesc &d, int64_t q) {
  const int64_t P = 2 * d.n * d.n / PG_BYTES;  // pages per operand
  const int op = q >= P ? 1 : 0;
  const int64_t pq = q - op * P;
  char *base = v.addr((op ? d.o1 : d.o0) + uint64_t(pq) * PG_BYTES);
  const uint64_t s0 = (2 * d.seed + uint64_t(op)) << 32;
  const uint64_t e0 = uint64_t(pq) * (PG_BYTES / 2);
  for (int w = threadIdx.x; w < PG_BYTES / 16; w += blockDim.x) {
    u32x4 x;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      uint32_t pair = 0;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const uint64_t z = splitmix_at(s0, e0 + 8 * uint64_t(w) + 2 * e + hh);
        const float f = (float(int(z & 0xFF)) - 128.0f) * (1.0f / 64.0f);
        pair |= (__float_as_uint(f) >> 16) << (16 * hh);  // exact: 8 significant bits
      }
      x[e] = pair;
    }
    *reinterpret_cast<u32x4 *>(base + 16 * w) = x;
  }
}

__global__ void k_batch_p0(BatchTable *__restrict__ t) {
  __shared__ long long s_item;
  __shared__ uint32_t sdir[PG_DIR];
  const PageMap m = t->map;
  const int64_t mapped = pm_pages(m);
  if (mapped < t->need) return;  // the placement failed: nothing is mapped
  const PgView v = pg_view(m, sdir, mapped);
  const int64_t chunk = t->chunk;
  pull_items(t, 0, &s_item, [&](const BatchDesc &d, int64_t q) {
    if (d.kind == SCHED_JOB_TRIAD) triad_item(v, d, q, chunk);
    else if (d.kind == SCHED_JOB_HIST) hist_zero(v, d);
    else gemm_fill_page(v, d, q);
  });
}

// ---- phase 1 ----------------------------------------------------------------
// A histogram chunk: the keys are generated (key i = low 32 bits of
// SplitMix64 output i), stored to the job's key array, counted in LDS and the
// nonzero counts added to the bins.
__device__ __forceinline__ void hist_chunk(const PgView &v, const BatchDesc &d, int64_t q,
                                           int64_t chunk, uint32_t *h) {
  for (int b = threadIdx.x; b < SCHED_HIST_BINS; b += P12_THREADS) h[b] = 0;
  __syncthreads();
  const int64_t e0 = q * chunk;
  const int64_t e1 = e0 + chunk < d.n ? e0 + chunk : d.n;
  const uint64_t s0 = d.seed << 32;
  const uint64_t wbase = uint64_t(4 * e0) & ~uint64_t(PG_BYTES - 1);
  const uint32_t b0 = uint32_t(uint64_t(4 * e0) - wbase);
  const PgWin K = pg_win(v, d.o0 + wbase, d.o0 + uint64_t(4 * d.n));
  for (int64_t i = e0 + threadIdx.x; i < e1; i += P12_THREADS) {
    const uint32_t key = uint32_t(splitmix_at(s0, uint64_t(i)));
    *reinterpret_cast<uint32_t *>(K.at(b0 + 4 * uint32_t(i - e0))) = key;
    atomicAdd(&h[key & (SCHED_HIST_BINS - 1)], 1u);
  }
  __syncthreads();
  const PgWin W = bins_win(v, d);
  for (int b = threadIdx.x; b < SCHED_HIST_BINS; b += P12_THREADS) {
    const uint32_t c = h[b];
    if (c) atomicAdd(reinterpret_cast<uint32_t *>(W.at(4 * b)), c);
  }
}

// Output tile q (row-major over the (N / T)^2 tiles) of C = A B^T, N x N x N:
// four waves, each a (T/2) x (T/2) block of 32 x 32 MFMA blocks; k-tiles of
// 64 staged through one LDS stage with the next k-tile's loads in registers.
// Operand and output rows each lie in one page (the arrays start at page
// boundaries and 2N, 4N divide the page size), so every row is translated
// once, into a table in LDS.  The MFMA operands and the k order are those of
// the single-job kernel, so the result is bit-identical to it.
template <int T>
__device__ __forceinline__ void gemm_tile(const PgView &v, const BatchDesc &d, int64_t q, char *smem) {
  constexpr int MB = T / 64;  // 32 x 32 blocks per wave and dimension
  constexpr int LJ = T / 32;  // 16-byte loads per thread, operand and k-tile
  uint16_t *sA = reinterpret_cast<uint16_t *>(smem);
  uint16_t *sB = sA + T * GLR;
  char **srow = reinterpret_cast<char **>(sB + T * GLR);
  const int64_t N = d.n, tn = N / T;
  const int64_t m0 = (q / tn) * T, n0 = (q % tn) * T;
  const int tid = threadIdx.x;
  for (int r = tid; r < 3 * T; r += P12_THREADS) {
    uint64_t off;
    if (r < T) off = d.o0 + uint64_t(m0 + r) * uint64_t(2 * N);
    else if (r < 2 * T) off = d.o1 + uint64_t(n0 + r - T) * uint64_t(2 * N);
    else off = d.o2 + uint64_t(m0 + r - 2 * T) * uint64_t(4 * N);
    srow[r] = v.addr(off);
  }
  __syncthreads();
  const int lr = tid >> 3, c8 = (tid & 7) * 8;
  const char *pa[LJ], *pb[LJ];
  u32x4 ra[LJ], rb[LJ];
#pragma unroll
  for (int j = 0; j < LJ; ++j) {
    pa[j] = srow[lr + 32 * j] + 2 * c8;
    pb[j] = srow[T + lr + 32 * j] + 2 * c8;
    ra[j] = *reinterpret_cast<const u32x4 *>(pa[j]);
    rb[j] = *reinterpret_cast<const u32x4 *>(pb[j]);
  }
#pragma unroll
  for (int j = 0; j < LJ; ++j) {
    *reinterpret_cast<u32x4 *>(sA + (lr + 32 * j) * GLR + c8) = ra[j];
    *reinterpret_cast<u32x4 *>(sB + (lr + 32 * j) * GLR + c8) = rb[j];
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * (T / 2), wn = (wave & 1) * (T / 2);
  const int frow = lane & 31, fk = (lane >> 5) * 8;
  f32x16 acc[MB][MB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < MB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  const int nk = int(N / 64);
  for (int kb = 0; kb < nk; ++kb) {
    if (kb + 1 < nk) {
#pragma unroll
      for (int j = 0; j < LJ; ++j) {
        ra[j] = *reinterpret_cast<const u32x4 *>(pa[j] + (kb + 1) * 128);
        rb[j] = *reinterpret_cast<const u32x4 *>(pb[j] + (kb + 1) * 128);
      }
    }
#pragma unroll
    for (int ks = 0; ks < 64; ks += 16) {
      bf16x8 fa[MB], fb[MB];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        fa[i] = *reinterpret_cast<const bf16x8 *>(sA + (wm + 32 * i + frow) * GLR + ks + fk);
        fb[i] = *reinterpret_cast<const bf16x8 *>(sB + (wn + 32 * i + frow) * GLR + ks + fk);
      }
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < MB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (kb + 1 < nk) {
#pragma unroll
      for (int j = 0; j < LJ; ++j) {
        *reinterpret_cast<u32x4 *>(sA + (lr + 32 * j) * GLR + c8) = ra[j];
        *reinterpret_cast<u32x4 *>(sB + (lr + 32 * j) * GLR + c8) = rb[j];
      }
    }
    __syncthreads();
  }
  // D layout of a 32 x 32 block: lane -> column (lane & 31); register r ->
  // row 8 (r / 4) + 4 (lane / 32) + (r % 4)
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      float *crow = reinterpret_cast<float *>(srow[2 * T + row]);
#pragma unroll
      for (int j = 0; j < MB; ++j) crow[n0 + wn + 32 * j + (lane & 31)] = acc[i][j][r];
    }
}

template <int T>
constexpr int p1_lds() {
  return 4 * SCHED_HIST_BINS > 2 * T * GLR * 2 + 3 * T * 8 ? 4 * SCHED_HIST_BINS
                                                          : 2 * T * GLR * 2 + 3 * T * 8;
}

template <int T>
__global__ __launch_bounds__(P12_THREADS) void k_batch_p1(BatchTable *__restrict__ t) {
  __shared__ long long s_item;
  __shared__ uint32_t sdir[PG_DIR];
  __shared__ __attribute__((aligned(16))) char smem[p1_lds<T>()];
  const PageMap m = t->map;
  const int64_t mapped = pm_pages(m);
  if (mapped < t->need) return;
  const PgView v = pg_view(m, sdir, mapped);
  const int64_t chunk = t->chunk;
  pull_items(t, 1, &s_item, [&](const BatchDesc &d, int64_t q) {
    if (d.kind == SCHED_JOB_HIST) hist_chunk(v, d, q, chunk, reinterpret_cast<uint32_t *>(smem));
    else if (d.kind == SCHED_JOB_GEMM) gemm_tile<T>(v, d, q, smem);
  });
}

// ---- phase 2 ----------------------------------------------------------------
// Digests of the histograms' bins (one item) and of the GEMMs' C (one item
// per page), plus each GEMM's sampled entries: sample k is written by the
// item of the page that holds it.
__global__ __launch_bounds__(P12_THREADS) void k_batch_p2(BatchTable *__restrict__ t) {
  __shared__ long long s_item;
  __shared__ uint32_t sdir[PG_DIR];
  const PageMap m = t->map;
  const int64_t mapped = pm_pages(m);
  if (mapped < t->need) return;
  const PgView v = pg_view(m, sdir, mapped);
  pull_items(t, 2, &s_item, [&](const BatchDesc &d, int64_t q) {
    unsigned long long dg = 0;
    if (d.kind == SCHED_JOB_HIST) {
      const PgWin W = bins_win(v, d);
      for (int b = threadIdx.x; b < SCHED_HIST_BINS; b += P12_THREADS)
        dg += digest_term(uint64_t(b), *reinterpret_cast<const uint32_t *>(W.at(4 * b)));
    } else if (d.kind == SCHED_JOB_GEMM) {
      const char *base = v.addr(d.o2 + uint64_t(q) * PG_BYTES);
      const uint64_t i0 = uint64_t(q) * (PG_BYTES / 4);
      for (int w = threadIdx.x; w < PG_BYTES / 16; w += P12_THREADS) {
        const u32x4 x = *reinterpret_cast<const u32x4 *>(base + 16 * w);
#pragma unroll
        for (int e = 0; e < 4; ++e) dg += digest_term(i0 + 4 * uint64_t(w) + e, x[e]);
      }
      if (threadIdx.x < GEMM_SAMPLES && d.samples) {
        const uint64_t p = splitmix_at((d.seed << 32) ^ SAMPLE_KEY, uint64_t(threadIdx.x)) %
                           uint64_t(d.n * d.n);
        if ((p >> (PG_SHIFT - 2)) == uint64_t(q))
          d.samples[threadIdx.x] =
              *reinterpret_cast<const float *>(base + 4 * (p & uint64_t(PG_BYTES / 4 - 1)));
      }
    }
    add_digest(d, dg);
  });
}

}  // namespace

int batch_init(BatchEngine &b, int device, int max_desc) {
  b.device = device;
  b.max_desc = max_desc;
  const size_t bytes = BatchTable::bytes_for(max_desc);
  SCHED_HIP_TRY(hipHostMalloc(&b.h_table, bytes, hipHostMallocMapped));
  SCHED_HIP_TRY(hipHostGetDevicePointer((void **)&b.h_table_dev, b.h_table, 0));
  SCHED_HIP_TRY(hipMalloc(&b.d_table, bytes));
  // the device copy keeps its own pointers into device memory
  BatchTable tmp{};
  BatchTable::layout_at(&tmp, (char *)b.d_table, max_desc);
  SCHED_HIP_TRY(hipMemcpy(b.d_table, &tmp, sizeof(BatchTable), hipMemcpyHostToDevice));
  // and the host copy's pointers as the device sees them
  memset(b.h_table, 0, sizeof(BatchTable));
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

static int launch_direct(BatchEngine &b, const BatchGraph &sh, hipStream_t s) {
  k_batch_stage<<<std::max(1, std::min(64, b.max_desc / 256 + 1)), 256, 0, s>>>(b.h_table_dev,
                                                                               b.d_table);
  SCHED_HIP_TRY(hipGetLastError());
  k_batch_p0<<<sh.grid, sh.block, 0, s>>>(b.d_table);
  SCHED_HIP_TRY(hipGetLastError());
  if (sh.phases > 1) {
    if (sh.tile == 64) k_batch_p1<64><<<sh.grid1, P12_THREADS, 0, s>>>(b.d_table);
    else k_batch_p1<128><<<sh.grid1, P12_THREADS, 0, s>>>(b.d_table);
    SCHED_HIP_TRY(hipGetLastError());
    k_batch_p2<<<b.cus * P2_PER_CU, P12_THREADS, 0, s>>>(b.d_table);
    SCHED_HIP_TRY(hipGetLastError());
  }
  return SCHED_OK;
}

static int graph_for(BatchEngine &b, const BatchGraph &sh, hipStream_t s, hipGraphExec_t *out) {
  for (auto &g : b.graphs)
    if (g.block == sh.block && g.grid == sh.grid && g.tile == sh.tile && g.grid1 == sh.grid1 &&
        g.phases == sh.phases) {
      *out = g.exec;
      return SCHED_OK;
    }
  BatchGraph g = sh;
  SCHED_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = launch_direct(b, sh, s);
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

// Fills the pinned table from descriptors (chunk in elements) and counts
// each job's work items per phase:
//   triad      ceil(n / chunk) | -                       | -
//   histogram  1 (zero bins)   | ceil(n / chunk)          | 1 (digest)
//   GEMM       pages of A, B^T | (N / tile)^2 tiles       | pages of C (digest)
// (no digest items for a job without a digest).
int batch_fill(BatchEngine &b, const std::vector<BatchDesc> &descs, int64_t chunk, const PageMap &map,
               int64_t need) {
  if ((int)descs.size() > b.max_desc) return SCHED_E_INVALID;
  // a streaming item inside one 64 KiB window of each array: see triad_item
  if (chunk <= 0 || chunk > PG_BYTES / 4 || (PG_BYTES / 4) % chunk) return SCHED_E_INVALID;
  if (b.tile != 64 && b.tile != 128) return SCHED_E_INVALID;
  BatchTable *t = b.h_table;
  const int stride = b.max_desc + 1;
  BatchDesc *hd = (BatchDesc *)((char *)t + BatchTable::desc_offset());
  int64_t *ho = (int64_t *)((char *)t + BatchTable::off_offset(b.max_desc));
  int64_t acc[BATCH_PHASES] = {0, 0, 0};
  bool later = false;
  for (size_t i = 0; i < descs.size(); ++i) {
    BatchDesc d = descs[i];
    if (((d.o0 | d.o1 | d.o2) & 4095) || d.n < 0) return SCHED_E_INVALID;
    int64_t it[BATCH_PHASES] = {0, 0, 0};
    const bool dig = d.digest != nullptr;
    switch (d.kind) {
      case SCHED_JOB_TRIAD:
        if (d.iters < 0) return SCHED_E_INVALID;
        it[0] = (d.n + chunk - 1) / chunk;
        break;
      case SCHED_JOB_HIST:
        it[0] = 1;
        it[1] = (d.n + chunk - 1) / chunk;
        it[2] = dig ? 1 : 0;
        break;
      case SCHED_JOB_GEMM: {
        const int64_t N = d.n;
        // every operand and output row inside one page, whole pages per array
        if (N < 256 || N < b.tile || N > PG_BYTES / 4 || (N & (N - 1)) ||
            ((d.o0 | d.o1 | d.o2) & (PG_BYTES - 1)))
          return SCHED_E_INVALID;
        it[0] = 2 * (2 * N * N / PG_BYTES);
        it[1] = (N / b.tile) * (N / b.tile);
        it[2] = dig ? 4 * N * N / PG_BYTES : 0;
        break;
      }
      default: return SCHED_E_INVALID;
    }
    for (int p = 0; p < BATCH_PHASES; ++p) {
      if (it[p] > INT_MAX) return SCHED_E_INVALID;
      d.items[p] = int32_t(it[p]);
      ho[p * stride + int(i)] = acc[p];
      acc[p] += it[p];
    }
    later = later || it[1] > 0 || it[2] > 0;
    hd[i] = d;
  }
  for (int p = 0; p < BATCH_PHASES; ++p) {
    ho[p * stride + int(descs.size())] = acc[p];
    t->n_items[p] = acc[p];
  }
  t->n_desc = int(descs.size());
  t->stride = stride;
  t->chunk = chunk;
  t->map = map;
  t->need = need;
  t->tile = b.tile;
  b.phases = later ? BATCH_PHASES : 1;
  return SCHED_OK;
}

int batch_launch(BatchEngine &b, hipStream_t s, bool use_graph) {
  BatchGraph sh;
  sh.block = b.block > 0 ? b.block : 256;
  sh.grid = b.cus * (b.per_cu > 0 ? b.per_cu : 4);
  sh.phases = b.phases;
  // the phase-1 shape only matters to batches that have the phase
  sh.tile = sh.phases > 1 ? b.tile : 0;
  sh.grid1 = sh.phases > 1 ? b.cus * std::max(1, b.per_cu1) : 0;
  if (!use_graph) return launch_direct(b, sh, s);
  hipGraphExec_t exec = nullptr;
  if (int rc = graph_for(b, sh, s, &exec)) return rc;
  SCHED_PROF_LAUNCH_GRAPH("k_batch_graph", s, hipGraphLaunch(exec, s));
  return SCHED_OK;
}

namespace {

// Device time of `reps` launches of the filled table (after one warm-up).
int time_batch(BatchEngine &b, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, float *ms) {
  if (int rc = batch_launch(b, s, false)) return rc;
  SCHED_HIP_TRY(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r)
    if (int rc = batch_launch(b, s, false)) return rc;
  SCHED_HIP_TRY(hipEventRecord(e1, s));
  SCHED_HIP_TRY(hipEventSynchronize(e1));
  SCHED_HIP_TRY(hipEventElapsedTime(ms, e0, e1));
  return SCHED_OK;
}

bool read_cache(BatchEngine &b, const char *path) {
  FILE *f = fopen(path, "r");
  if (!f) return false;
  int blk = 0, per = 0, tile = 0, per1 = 0;
  long long ch = 0;
  char buf[768] = {0};
  size_t nr = fread(buf, 1, sizeof(buf) - 1, f);
  fclose(f);
  buf[nr] = 0;
  const char *pb = strstr(buf, "\"block\":"), *pc = strstr(buf, "\"chunk\":"),
             *pp = strstr(buf, "\"per_cu\":"), *pt = strstr(buf, "\"gemm_tile\":"),
             *p1 = strstr(buf, "\"gemm_per_cu\":");
  if (!(pb && pc && pp && pt && p1 && sscanf(pb, "\"block\": %d", &blk) == 1 &&
        sscanf(pc, "\"chunk\": %lld", &ch) == 1 && sscanf(pp, "\"per_cu\": %d", &per) == 1 &&
        sscanf(pt, "\"gemm_tile\": %d", &tile) == 1 &&
        sscanf(p1, "\"gemm_per_cu\": %d", &per1) == 1))
    return false;
  if (blk <= 0 || blk > 1024 || blk % WAVE || per <= 0 || ch <= 0 || ch > PG_BYTES / 4 ||
      (PG_BYTES / 4) % ch || (tile != 64 && tile != 128) || per1 <= 0 || per1 > 16)
    return false;
  b.block = blk;
  b.chunk = ch;
  b.per_cu = per;
  b.tile = tile;
  b.per_cu1 = per1;
  return true;
}

}  // namespace

// Autotuner.  Streaming phase: each (block, chunk, workgroups per CU)
// candidate on a synthetic batch of 4 MiB triads.  Phase 1: each (GEMM tile
// edge, workgroups per CU) candidate on a synthetic batch of small GEMMs
// (8 each of N = 256, 512, 1024; the whole three-launch batch is timed).
// The fastest of each is kept and cached in `cache_path` (JSON) when given.
int batch_autotune(BatchEngine &b, const char *cache_path, hipStream_t s) {
  if (cache_path && *cache_path && read_cache(b, cache_path)) {
    b.tuned = true;
    b.from_cache = true;
    return SCHED_OK;
  }
  hipEvent_t e0, e1;
  SCHED_HIP_TRY(hipEventCreate(&e0));
  SCHED_HIP_TRY(hipEventCreate(&e1));
  // -- streaming phase
  {
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
      ds[i] = BatchDesc{base, base + arr, base + 2 * arr, job_elems, uint64_t(i + 1), 10,
                        SCHED_JOB_TRIAD, dig + i, nullptr, {0, 0, 0}, 0};
    }
    const int blocks[] = {256, 512, 1024};
    const int64_t chunks[] = {1 << 12, 1 << 13, 1 << 14};  // divisors of a 64 KiB window
    const int pers[] = {2, 4, 8};
    double best = 1e30;
    for (int blk : blocks)
      for (int64_t ch : chunks)
        for (int per : pers) {
          if (blk * per > 2048) continue;  // at most 32 waves per CU
          b.block = blk;
          b.per_cu = per;
          if (int rc = batch_fill(b, ds, ch, idm.map, need)) return rc;
          float ms = 0;
          if (int rc = time_batch(b, s, e0, e1, 3, &ms)) return rc;
          if (ms < best) {
            best = ms;
            b.chunk = ch;
            b.best_block = blk;
            b.best_per_cu = per;
          }
        }
    b.block = b.best_block;
    b.per_cu = b.best_per_cu;
    b.tune_ms = best / 3;
    pg_identity_free(&idm);
    (void)hipFree(arena);
    (void)hipFree(dig);
  }
  // -- phase 1: GEMM tiles
  {
    const int64_t Ns[] = {256, 512, 1024};
    std::vector<BatchDesc> ds;
    uint64_t base = 0;
    for (int64_t N : Ns)
      for (int k = 0; k < 8; ++k) {
        const uint64_t ab = uint64_t(2 * N * N);
        ds.push_back(BatchDesc{base, base + ab, base + 2 * ab, N, uint64_t(ds.size() + 1), 0,
                               SCHED_JOB_GEMM, nullptr, nullptr, {0, 0, 0}, 0});
        base += 2 * ab + uint64_t(4 * N * N);
      }
    char *arena = nullptr;
    unsigned long long *dig = nullptr;
    SCHED_HIP_TRY(hipMalloc(&arena, base));
    SCHED_HIP_TRY(hipMalloc(&dig, sizeof(unsigned long long) * ds.size()));
    for (size_t i = 0; i < ds.size(); ++i) ds[i].digest = dig + i;
    PgIdentity idm;
    if (int rc = pg_identity(arena, int64_t(base), s, &idm)) return rc;
    const int64_t need = int64_t(base / PG_BYTES);
    const int tiles[] = {64, 128};
    const int pers[] = {1, 2, 4};
    double best = 1e30;
    int best_tile = 128, best_per = 2;
    for (int tile : tiles)
      for (int per : pers) {
        b.tile = tile;
        b.per_cu1 = per;
        if (int rc = batch_fill(b, ds, b.chunk, idm.map, need)) return rc;
        float ms = 0;
        if (int rc = time_batch(b, s, e0, e1, 3, &ms)) return rc;
        if (ms < best) {
          best = ms;
          best_tile = tile;
          best_per = per;
        }
      }
    b.tile = best_tile;
    b.per_cu1 = best_per;
    b.tune_gemm_ms = best / 3;
    pg_identity_free(&idm);
    (void)hipFree(arena);
    (void)hipFree(dig);
  }
  b.tuned = true;
  b.from_cache = false;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (cache_path && *cache_path) {
    FILE *f = fopen(cache_path, "w");
    if (f) {
      fprintf(f,
              "{\"block\": %d, \"chunk\": %lld, \"per_cu\": %d, \"batch_ms\": %.4f, "
              "\"gemm_tile\": %d, \"gemm_per_cu\": %d, \"gemm_batch_ms\": %.4f, "
              "\"probe\": \"256 triads x 4 MiB, 10 sweeps; 8 GEMMs each of N = 256, 512, 1024\"}\n",
              b.block, (long long)b.chunk, b.per_cu, b.tune_ms, b.tile, b.per_cu1, b.tune_gemm_ms);
      fclose(f);
    }
  }
  return SCHED_OK;
}

}  // namespace schedk
