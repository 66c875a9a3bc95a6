// Page tier of the device sub-allocator: the memory the serving loop gives
// its tenants.
//
// Admission (Sec. V) only guarantees that the declared demands of the running
// jobs add up to at most the capacity; with one contiguous range per job, an
// admitted job could still find no range wide enough.  Here a job's buffers
// live in a logical address space of its own, mapped page by page onto a
// device pool of 64 KiB pages, so any set of pages will do and placing an
// admitted job cannot fail for lack of contiguity.
//
//   * The pool's free pages are a stack of page numbers; a placement pops the
//     pages it needs, a release pushes them back.  Pop and push positions come
//     from one counter of pages in use, charged by compare-and-swap so that a
//     request that does not fit never disturbs the counter.
//   * Each placement slot has a directory of PG_DIR entries.  A placement of
//     at most PG_DIR pages stores its page numbers in the directory itself; a
//     larger one stores node numbers there, each node a block of PG_NODE page
//     numbers from a node pool managed like the page pool.  Up to
//     PG_DIR * PG_NODE pages (64 GiB) per placement.
//   * Buffers inside a logical space start at 4 KiB boundaries; a tenant
//     kernel translates a logical offset with one or two loads (directory,
//     then node), at most once per 4 KiB it touches, since 4 KiB never
//     straddles a page.
// The bytes a job's buffers take (each buffer rounded up to 4 KiB) are charged
// to the job against its admitted reservation -- the itemised use of
// Sec. III-B -- with the slab's per-tenant counters.  Physically a placement
// also holds the unused rest of its last page, so the pool is one page per
// slot larger than the capacity admission hands out.
#pragma once

#include "common.h"

namespace schedk {

constexpr int PG_SHIFT = 16;
constexpr int64_t PG_BYTES = int64_t(1) << PG_SHIFT;   // 64 KiB pages
constexpr int PG_DIR = 1024;                           // directory entries per slot
constexpr int PG_NODE_SHIFT = 10;
constexpr int PG_NODE = 1 << PG_NODE_SHIFT;            // page numbers per node
constexpr int64_t PG_MAX_PAGES = int64_t(PG_DIR) * PG_NODE;

// Per-slot record, written by the placement kernel and read by the tenant
// kernels of the placement (pages == 0: nothing is mapped, the kernels do
// nothing) and by the release kernel.
struct PlaceRec {
  int64_t pages;      // logical pages mapped
  int64_t bytes;      // bytes charged over all jobs of the placement
  int32_t nodes;      // nodes taken (0: direct)
  int32_t status;     // 0 placed; 1 over quota; 2 pool exhausted; 3 node pool
                      // exhausted; 5 invalid request; 6 released / never placed
};

// What a tenant kernel receives by value.
struct PageMap {
  char *pool;
  const uint32_t *dir;     // the slot's directory
  const uint32_t *nodes;   // node pool
  const PlaceRec *rec;     // the slot's record
  int32_t direct;          // pages <= PG_DIR: the directory holds page numbers
  int32_t pad;
};

// Page tables do not change while a placement's kernels run, so they are
// read through the constant address space: a wave-uniform lookup becomes a
// scalar load.
typedef const __attribute__((address_space(4))) uint32_t cst_u32;

__device__ __forceinline__ uint32_t pm_page(const PageMap &m, uint64_t lp) {
  cst_u32 *dir = (cst_u32 *)m.dir;
  if (m.direct) return dir[lp];
  const uint32_t node = dir[lp >> PG_NODE_SHIFT];
  return ((cst_u32 *)m.nodes)[uint64_t(node) * PG_NODE + (lp & (PG_NODE - 1))];
}

// The same lookup when the kind of table is known at compile time (no
// branch, so independent lookups issue back to back).
template <bool DIRECT>
__device__ __forceinline__ char *pm_addr_t(const PageMap &m, uint64_t off) {
  cst_u32 *dir = (cst_u32 *)m.dir;
  const uint64_t lp = off >> PG_SHIFT;
  uint32_t pg;
  if constexpr (DIRECT) {
    pg = dir[lp];
  } else {
    pg = ((cst_u32 *)m.nodes)[uint64_t(dir[lp >> PG_NODE_SHIFT]) * PG_NODE + (lp & (PG_NODE - 1))];
  }
  return m.pool + (uint64_t(pg) << PG_SHIFT) + (off & (PG_BYTES - 1));
}

// Device address of logical offset `off` (the page must be mapped).
__device__ __forceinline__ char *pm_addr(const PageMap &m, uint64_t off) {
  return m.pool + (uint64_t(pm_page(m, off >> PG_SHIFT)) << PG_SHIFT) + (off & (PG_BYTES - 1));
}

// Logical pages the placement has mapped (0 after a failed placement).
__device__ __forceinline__ int64_t pm_pages(const PageMap &m) {
  return __hip_atomic_load(&m.rec->pages, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- windows: the fast path of the streaming kernels ----------------------
// A kernel copies the placement's directory (at most PG_DIR entries) into LDS
// once; then a 64 KiB window of an array that starts at a 4 KiB boundary
// covers at most two pages, so its two bases are resolved once per window
// (directory from LDS, plus one node load for a placement of more than
// PG_DIR pages) and every access inside it is a compare and an add.
typedef const __attribute__((address_space(3))) uint32_t lds_u32;

struct PgView {
  lds_u32 *sdir;          // LDS copy of the directory
  const uint32_t *nodes;
  char *pool;
  int32_t direct;
  __device__ __forceinline__ uint32_t page(uint64_t lp) const {
    if (direct) return sdir[lp];
    const uint32_t node = sdir[lp >> PG_NODE_SHIFT];
    return nodes[uint64_t(node) * PG_NODE + (lp & (PG_NODE - 1))];
  }
  __device__ __forceinline__ char *addr(uint64_t off) const {
    return pool + (uint64_t(page(off >> PG_SHIFT)) << PG_SHIFT) + (off & (PG_BYTES - 1));
  }
};

// Loads the directory entries a placement of `pages` pages uses; the whole
// workgroup calls it (it ends with a barrier).  sdir: a __shared__ array of
// PG_DIR entries.
__device__ __forceinline__ PgView pg_view(const PageMap &m, uint32_t *sdir, int64_t pages) {
  const int64_t e = m.direct ? pages : (pages + PG_NODE - 1) >> PG_NODE_SHIFT;
  for (int64_t i = threadIdx.x; i < e && i < PG_DIR; i += blockDim.x) sdir[i] = m.dir[i];
  __syncthreads();
  return PgView{(lds_u32 *)sdir, m.nodes, m.pool, m.direct};
}

// The physical runs behind logical bytes [off, off + 64 KiB) of an array
// that starts at a 4 KiB boundary and ends at logical offset `end`: bytes
// below `split` at b0, the rest at b1.  The second page is looked up only if
// the array reaches it.  `split` is a multiple of 4 KiB, so each 4 KiB unit
// of the window lies in one run: unit(q) is the same for every thread.
struct PgWin {
  char *b0, *b1;
  uint32_t split;
  __device__ __forceinline__ char *at(uint32_t byte) const {
    return byte < split ? b0 + byte : b1 + (byte - split);
  }
  __device__ __forceinline__ char *unit(uint32_t q) const {
    const uint32_t byte = q << 12;
    return byte < split ? b0 + byte : b1 + (byte - split);
  }
};
__device__ __forceinline__ PgWin pg_win(const PgView &v, uint64_t off, uint64_t end) {
  const uint32_t in = uint32_t(off & (PG_BYTES - 1));
  PgWin w;
  w.b0 = v.addr(off);
  w.split = uint32_t(PG_BYTES) - in;
  const uint64_t next = (off >> PG_SHIFT) + 1;
  w.b1 = in && (next << PG_SHIFT) < end ? v.pool + (uint64_t(v.page(next)) << PG_SHIFT) : w.b0 + w.split;
  return w;
}

// Position-keyed digest of 32-bit words: sum over i of (s_i | 1) * w_i mod
// 2^64, where s_i is output i of SplitMix64 (Steele, Lea, Flood 2014) whose
// state starts at DIGEST_KEY.  Every multiplier is odd, so changing any one
// word changes the digest, and moving a word to another position changes it
// unless the two multipliers collide.
constexpr uint64_t DIGEST_KEY = 0x6A09E667F3BCC908ULL;

__device__ __forceinline__ uint64_t splitmix_at(uint64_t s0, uint64_t i) {
  uint64_t z = s0 + (i + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t digest_term(uint64_t i, uint32_t w) {
  return (splitmix_at(DIGEST_KEY, i) | 1ULL) * uint64_t(w);
}

// Sampled GEMM entries reported by the serving loop: entry k (0 <= k <
// GEMM_SAMPLES) is C's element (SplitMix64 output k for state
// (seed << 32) ^ SAMPLE_KEY) mod N^2, in row-major order.
constexpr uint64_t SAMPLE_KEY = 0xBB67AE8584CAA73BULL;
constexpr int GEMM_SAMPLES = 8;

// ---- host side ----------------------------------------------------------
// One placement request (device-readable): slot, logical pages to map, and
// the jobs it charges, entries [job_off, job_off + n_jobs) of the parallel
// job / byte lists passed beside it.
struct PgReq {
  int32_t slot;
  int32_t n_jobs;
  int64_t pages;
  int64_t job_off;
};

struct PgCounters {
  int64_t pages_used, nodes_used, charged, violations, placed, released, over_admitted,
      peak_pages, pool_pages;
};

// A page table mapping a contiguous buffer onto itself.
struct PgIdentity {
  PageMap map;
  uint32_t *dir = nullptr, *nodes = nullptr;
  PlaceRec *rec = nullptr;
};

int pg_identity(char *base, int64_t bytes, hipStream_t s, PgIdentity *out);
void pg_identity_free(PgIdentity *m);

// Paged tenant work (tenants.hip); offsets are logical byte offsets inside
// the placement mapped by m, each a multiple of 4096.
int pgt_triad_fill(const PageMap &m, uint64_t off_b, uint64_t off_c, int64_t n, uint64_t seed,
                   hipStream_t s);
int pgt_triad(const PageMap &m, uint64_t off_a, uint64_t off_b, uint64_t off_c, float sc,
              int64_t n, int32_t iters, hipStream_t s);
int pgt_hist_fill(const PageMap &m, uint64_t off_keys, int64_t n, uint64_t seed, hipStream_t s);
int pgt_hist(const PageMap &m, uint64_t off_keys, int64_t n, uint32_t mask, uint64_t off_bins,
             hipStream_t s);
int pgt_gemm_fill(const PageMap &m, uint64_t off, int64_t rows, int64_t K, uint64_t seed,
                  hipStream_t s);
// N x N x N, N a power of two in [256, 16384]; A, B, C at page boundaries.
int pgt_gemm(const PageMap &m, uint64_t off_a, uint64_t off_b, uint64_t off_c, int64_t N,
             hipStream_t s);
// *out += position-keyed digest of n 32-bit words at off.
int pgt_digest(const PageMap &m, uint64_t off, int64_t n, unsigned long long *out, hipStream_t s);
// out[k] = C[p_k] for the GEMM_SAMPLES sampled positions of the job's seed.
int pgt_gemm_samples(const PageMap &m, uint64_t off_c, int64_t N, uint64_t seed, float *out,
                     hipStream_t s);

}  // namespace schedk
