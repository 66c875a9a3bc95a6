// Synthetic tenant jobs that the co-scheduler runs side by side:
//   * STREAM triad a = b + s*c in fp32 (HBM streaming);
//   * histogram of uint32 keys into 4096 bins (HBM streaming + LDS atomics);
//   * C = A * B^T with bf16 inputs and fp32 accumulation on MFMA (the one
//     dense contraction).
// Input contents are generated on the device from SplitMix64 (Steele, Lea,
// Flood 2014): output i of the generator whose state starts at s0 is the
// finaliser applied to s0 + (i + 1) * golden-gamma.
#include <algorithm>

#include "common.h"
#include "pages.h"
#include "prof.h"

using namespace schedk;

namespace {

__device__ __forceinline__ uint64_t splitmix(uint64_t s0, uint64_t i) {
  uint64_t z = s0 + (i + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

int grid_cap(int64_t items, int threads, int cap) {
  int64_t g = (items + threads - 1) / threads;
  return int(std::max<int64_t>(1, std::min<int64_t>(g, cap)));
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------- triad
__global__ void k_triad_fill(float *__restrict__ b, float *__restrict__ c, int64_t n, uint64_t s0) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const uint64_t h = splitmix(s0, uint64_t(i));
    b[i] = 1.0f + float(h & 0xFFFF) * (1.0f / 65536.0f);
    c[i] = 1.0f + float((h >> 16) & 0xFFFF) * (1.0f / 65536.0f);
  }
}

// 16-byte vectors, non-temporal.  Each workgroup streams a contiguous chunk
// of TRIAD_U x 256 vectors (all loads of a chunk in flight before its
// stores); the launch covers the array with one chunk per workgroup (the
// loop only runs again when the grid had to be capped).  Measured on 1 GiB
// arrays this beats a grid-stride layout by ~25 %, and on 2 GiB arrays one
// chunk per workgroup streams ~4 % faster than a grid capped at 32768
// workgroups looping over chunks (6.0 vs 5.8 TB/s).  The scalar tail (n % 4)
// is done by the first threads.
constexpr int TRIAD_U = 4;
__global__ __launch_bounds__(256) void k_triad(float *__restrict__ a, const float *__restrict__ b,
                                               const float *__restrict__ c, float s, int64_t n) {
  const int64_t nv = n >> 2;
  const f32x4 *__restrict__ b4 = reinterpret_cast<const f32x4 *>(b);
  const f32x4 *__restrict__ c4 = reinterpret_cast<const f32x4 *>(c);
  f32x4 *__restrict__ a4 = reinterpret_cast<f32x4 *>(a);
  constexpr int64_t CH = 256 * TRIAD_U;
  for (int64_t base = blockIdx.x * CH; base < nv; base += int64_t(gridDim.x) * CH) {
    f32x4 x[TRIAD_U], y[TRIAD_U];
#pragma unroll
    for (int u = 0; u < TRIAD_U; ++u) {
      const int64_t i = base + u * 256 + threadIdx.x;
      if (i < nv) {
        x[u] = __builtin_nontemporal_load(b4 + i);
        y[u] = __builtin_nontemporal_load(c4 + i);
      }
    }
#pragma unroll
    for (int u = 0; u < TRIAD_U; ++u) {
      const int64_t i = base + u * 256 + threadIdx.x;
      if (i < nv) __builtin_nontemporal_store(x[u] + s * y[u], a4 + i);
    }
  }
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t < (n & 3)) {
    const int64_t j = (nv << 2) + t;
    a[j] = b[j] + s * c[j];
  }
}

// --------------------------------------------------------------- histogram
__global__ void k_hist_fill(uint32_t *__restrict__ keys, int64_t n, uint64_t s0) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    keys[i] = uint32_t(splitmix(s0, uint64_t(i)));
}

// Two sub-histograms per workgroup (waves 0 and 2 share one, 1 and 3 the
// other): 32 KiB of LDS, so three workgroups fit a CU.  Over 2^29 keys, three
// workgroups per CU stream at 6.9 TB/s, against 6.1 TB/s with one
// sub-histogram per wave (64 KiB, two workgroups per CU); four or more per
// CU are slower again.
constexpr int HIST_THREADS = 256;
constexpr int HIST_COPIES = 2;
constexpr int HIST_PER_CU = 3;

__global__ __launch_bounds__(HIST_THREADS) void k_hist(const uint32_t *__restrict__ keys, int64_t n,
                                                       uint32_t mask, uint32_t *__restrict__ bins) {
  __shared__ uint32_t h[HIST_COPIES][SCHED_HIST_BINS];
  for (int i = threadIdx.x; i < HIST_COPIES * SCHED_HIST_BINS; i += HIST_THREADS)
    (&h[0][0])[i] = 0;
  __syncthreads();
  uint32_t *mine = h[(threadIdx.x / 64) % HIST_COPIES];
  const int64_t nv = n >> 2;
  const u32x4 *__restrict__ k4 = reinterpret_cast<const u32x4 *>(keys);
  const int64_t stride = int64_t(gridDim.x) * HIST_THREADS;
  int64_t i = blockIdx.x * int64_t(HIST_THREADS) + threadIdx.x;
  // four 16-byte loads in flight per lane before their sixteen LDS updates
  for (; i + 3 * stride < nv; i += 4 * stride) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(k4 + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      atomicAdd(&mine[v[u].x & mask], 1u);
      atomicAdd(&mine[v[u].y & mask], 1u);
      atomicAdd(&mine[v[u].z & mask], 1u);
      atomicAdd(&mine[v[u].w & mask], 1u);
    }
  }
  for (; i < nv; i += stride) {
    const u32x4 v = __builtin_nontemporal_load(k4 + i);
    atomicAdd(&mine[v.x & mask], 1u);
    atomicAdd(&mine[v.y & mask], 1u);
    atomicAdd(&mine[v.z & mask], 1u);
    atomicAdd(&mine[v.w & mask], 1u);
  }
  const int64_t t = blockIdx.x * int64_t(HIST_THREADS) + threadIdx.x;
  if (t < (n & 3)) atomicAdd(&mine[keys[(nv << 2) + t] & mask], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < SCHED_HIST_BINS; b += HIST_THREADS) {
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < HIST_COPIES; ++k) s += h[k][b];
    if (s) atomicAdd(&bins[b], s);
  }
}

__global__ void k_zero_u32(uint32_t *p, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// -------------------------------------------------------------------- GEMM
__global__ void k_gemm_fill(uint16_t *__restrict__ x, int64_t rows, int64_t K, uint64_t s0) {
  const int64_t n = rows * K;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const uint64_t h = splitmix(s0, uint64_t(i));
    const float v = (float(int(h & 0xFF)) - 128.0f) * (1.0f / 64.0f);
    x[i] = uint16_t(__float_as_uint(v) >> 16);  // exact: v has 8 significant bits
  }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BN = 128, BK = 64;
constexpr int GT = 256;            // 4 waves, 2 x 2, each 64 x 64
constexpr int LDS_ROW = BK + 8;    // bf16 per LDS row: 144 B, breaks bank aliasing

// Each thread moves 4 x 16 B of A and 4 x 16 B of B per BK step: rows r =
// (tid >> 3) + 32 j, columns (tid & 7) * 8 .. +8.
struct Stage {
  u32x4 r0, r1, r2, r3;
};
__device__ __forceinline__ Stage g2r(const uint16_t *__restrict__ src, int64_t ld, int64_t row0,
                                     int64_t k0) {
  const int c = (threadIdx.x & 7) * 8;
  const uint16_t *p = src + (row0 + (threadIdx.x >> 3)) * ld + k0 + c;
  Stage s;
  s.r0 = *reinterpret_cast<const u32x4 *>(p);
  s.r1 = *reinterpret_cast<const u32x4 *>(p + 32 * ld);
  s.r2 = *reinterpret_cast<const u32x4 *>(p + 64 * ld);
  s.r3 = *reinterpret_cast<const u32x4 *>(p + 96 * ld);
  return s;
}
__device__ __forceinline__ void r2s(uint16_t *dst, const Stage &s) {
  const int c = (threadIdx.x & 7) * 8;
  uint16_t *p = dst + (threadIdx.x >> 3) * LDS_ROW + c;
  *reinterpret_cast<u32x4 *>(p) = s.r0;
  *reinterpret_cast<u32x4 *>(p + 32 * LDS_ROW) = s.r1;
  *reinterpret_cast<u32x4 *>(p + 64 * LDS_ROW) = s.r2;
  *reinterpret_cast<u32x4 *>(p + 96 * LDS_ROW) = s.r3;
}

// C[m][n] = sum_k A[m][k] * Bt[n][k]; M % 128 == N % 128 == K % 64 == 0.
// Blocks are ordered so that consecutive workgroups (spread over the XCDs)
// walk a column of C tiles, sharing the B^T panel through the MALL.
__global__ __launch_bounds__(GT) void k_gemm_bf16(const uint16_t *__restrict__ A,
                                                  const uint16_t *__restrict__ Bt,
                                                  float *__restrict__ C, int64_t M, int64_t N,
                                                  int64_t K) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][BM * LDS_ROW];
  __shared__ __attribute__((aligned(16))) uint16_t sB[2][BN * LDS_ROW];
  const int64_t tiles_m = M / BM;
  const int64_t bm = blockIdx.x % tiles_m, bn = blockIdx.x / tiles_m;
  const int64_t m0 = bm * BM, n0 = bn * BN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  Stage ra = g2r(A, K, m0, 0);
  Stage rb = g2r(Bt, K, n0, 0);
  r2s(sA[0], ra);
  r2s(sB[0], rb);
  __syncthreads();

  const int nk = int(K / BK);
  // operand fragment: row (lane & 31), k offset (lane >> 5) * 8 within a 16-wide k step
  const int frow = lane & 31, fk = (lane >> 5) * 8;
  for (int kb = 0; kb < nk; ++kb) {
    const int cur = kb & 1;
    if (kb + 1 < nk) {
      ra = g2r(A, K, m0, int64_t(kb + 1) * BK);
      rb = g2r(Bt, K, n0, int64_t(kb + 1) * BK);
    }
    const uint16_t *a_s = sA[cur];
    const uint16_t *b_s = sB[cur];
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf16x8 fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fa[i] = *reinterpret_cast<const bf16x8 *>(a_s + (wm + 32 * i + frow) * LDS_ROW + ks + fk);
        fb[i] = *reinterpret_cast<const bf16x8 *>(b_s + (wn + 32 * i + frow) * LDS_ROW + ks + fk);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (kb + 1 < nk) {
      r2s(sA[cur ^ 1], ra);
      r2s(sB[cur ^ 1], rb);
    }
    __syncthreads();
  }
  // D layout of a 32 x 32 block: lane -> column (lane & 31); register r -> row
  // 8 * (r / 4) + 4 * (lane / 32) + (r % 4).
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t col = n0 + wn + 32 * j + (lane & 31);
        C[row * N + col] = acc[i][j][r];
      }
}

// 256 x 256 x 64 block tile in 8 waves, two per SIMD, each owning 64 x 128
// of C (2 x 4 MFMA blocks of 32 x 32, 128 fp32 accumulators per lane).
//   * Operands go from HBM straight into LDS: buffer loads with the LDS flag
//     move 16 B per lane, one wave instruction filling 1 KiB of LDS (8 rows of
//     64 bf16).  The lane that fills chunk position p of row r fetches global
//     chunk p ^ ((r >> 1) & 7), so a fragment read (32 rows, one chunk each,
//     16 lanes per LDS cycle) touches 16 distinct 16-B bank groups.
//   * Two LDS stages (128 KiB).  One barrier per k-tile, placed before its
//     last k-step: the next tile's first fragments are read during that step,
//     and right after the barrier the stage just finished is refilled with
//     tile t + 2, its eight loads interleaved with the step's eight MFMAs.  A
//     load thus has a whole k-tile to land; each wave waits for its own loads
//     before the barrier, which publishes them to the other waves.
//   * Inside a k-tile, the fragment reads of step s + 1 alternate with the
//     MFMAs of step s.
// Blocks are dealt to the 8 XCDs round robin (block b runs on XCD b % 8);
// when the tile grid allows, XCD x gets a band of tile columns and walks it in
// groups of 8 tile rows, so the 32 workgroups an XCD runs at a time share
// their A and B k-slices in that XCD's L2.
constexpr int BM2 = 256, BN2 = 256;
constexpr int GT2 = 512;           // 8 waves
constexpr int ROW2 = BK;           // bf16 per LDS row: 128 B, unpadded (swizzled)
constexpr int N_XCD = 8, GROUP_ROWS = 8;
constexpr int BUF_RSRC_DW3 = 0x00020000;  // raw buffer, 32-bit dword format

typedef __attribute__((address_space(3))) void lds_void;

// PAGED: the operands live in a page-mapped placement (pages.h) at logical
// offsets oa, ob, oc instead of at A, Bt, C.  Every operand row then lies in
// one page (the host checks that 2K and 4N divide the page size and that the
// three arrays start at page boundaries), so each of the tile's 256 A rows,
// 256 B rows and 256 C rows is translated once, by one thread, into a table
// in LDS; the loads become global loads with the LDS flag from per-lane
// 64-bit addresses, the rest of the kernel is unchanged.
template <bool PAGED>
__global__ __launch_bounds__(GT2, 1) void k_gemm_bf16_256(const uint16_t *__restrict__ A,
                                                          const uint16_t *__restrict__ Bt,
                                                          float *__restrict__ C, int64_t M,
                                                          int64_t N, int64_t K, PageMap pm,
                                                          int64_t need, uint64_t oa, uint64_t ob,
                                                          uint64_t oc) {
  __shared__ __attribute__((aligned(1024))) uint16_t sA0[BM2 * ROW2];
  __shared__ __attribute__((aligned(1024))) uint16_t sA1[BM2 * ROW2];
  __shared__ __attribute__((aligned(1024))) uint16_t sB0[BN2 * ROW2];
  __shared__ __attribute__((aligned(1024))) uint16_t sB1[BN2 * ROW2];
  __shared__ char *s_row[PAGED ? BM2 + BN2 : 1];
  if constexpr (PAGED) {
    if (pm_pages(pm) < need) return;  // the placement failed: nothing is mapped
  }
  const int64_t tiles_m = M / BM2, tiles_n = N / BN2;
  const int64_t b = blockIdx.x;
  int64_t bm, bn;
  if (tiles_m % GROUP_ROWS == 0 && tiles_n % N_XCD == 0) {
    const int64_t bw = tiles_n / N_XCD;  // tile columns per XCD
    const int64_t x = b % N_XCD, q = b / N_XCD;
    const int64_t g = q / (GROUP_ROWS * bw), w = q % (GROUP_ROWS * bw);
    bm = g * GROUP_ROWS + w % GROUP_ROWS;
    bn = x * bw + w / GROUP_ROWS;
  } else {
    bm = b % tiles_m;
    bn = b / tiles_m;
  }
  const int64_t m0 = bm * BM2, n0 = bn * BN2;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 128;
  const int frow = lane & 31, half = lane >> 5, sw = (frow >> 1) & 7;

  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  // One buffer resource per 256-row operand panel (the host guarantees its
  // byte size fits the 32-bit range); lane offsets are fixed, the k advance
  // rides in the scalar offset.
  const int nk = int(K / BK);
  // (PAGED: unused resources over no memory)
  const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc(
      PAGED ? nullptr : (void *)(A + m0 * K), 0, PAGED ? 0 : int(BM2 * K * 2), BUF_RSRC_DW3);
  const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc(
      PAGED ? nullptr : (void *)(Bt + n0 * K), 0, PAGED ? 0 : int(BN2 * K * 2), BUF_RSRC_DW3);
  int voff[4];
  const char *gA[4], *gB[4];  // PAGED: per-lane addresses of the rows this lane loads
  if constexpr (!PAGED) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 8 * (wave + 8 * j) + (lane >> 3);  // wave instruction j fills rows 8G .. 8G + 7
      voff[j] = (r * int(K) + ((lane & 7) ^ ((r >> 1) & 7)) * 8) * 2;
    }
  } else {
    const int t = threadIdx.x;
    s_row[t] = t < BM2 ? pm_addr(pm, oa + uint64_t(m0 + t) * uint64_t(K) * 2)
                       : pm_addr(pm, ob + uint64_t(n0 + t - BM2) * uint64_t(K) * 2);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 8 * (wave + 8 * j) + (lane >> 3);
      const int cb = ((lane & 7) ^ ((r >> 1) & 7)) * 16;
      gA[j] = s_row[r] + cb;
      gB[j] = s_row[BM2 + r] + cb;
    }
  }
  auto fill = [&](__amdgpu_buffer_rsrc_t rs, const char *const *g, uint16_t *stage, int kbyte) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (!PAGED)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)(stage + (wave + 8 * j) * 8 * ROW2),
                                                 16, voff[j], kbyte, 0, 0);
      else
        __builtin_amdgcn_global_load_lds((const void *)(g[j] + kbyte),
                                         (lds_void *)(stage + (wave + 8 * j) * 8 * ROW2), 16, 0, 0);
    }
  };
  bf16x8 fa[2][2], fb[2][4];
  auto frag = [&](bf16x8 *xa, bf16x8 *xb, const uint16_t *a_s, const uint16_t *b_s, int step) {
    const int p = ((2 * step + half) ^ sw) * 8;
#pragma unroll
    for (int i = 0; i < 2; ++i)
      xa[i] = *reinterpret_cast<const bf16x8 *>(a_s + (wm + 32 * i + frow) * ROW2 + p);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      xb[j] = *reinterpret_cast<const bf16x8 *>(b_s + (wn + 32 * j + frow) * ROW2 + p);
  };

  fill(rsA, gA, sA0, 0);
  fill(rsB, gB, sB0, 0);
  if (nk > 1) {
    fill(rsA, gA, sA1, BK * 2);
    fill(rsB, gB, sB1, BK * 2);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  frag(fa[0], fb[0], sA0, sB0, 0);

  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1;
    uint16_t *a_s = cur ? sA1 : sA0, *b_s = cur ? sB1 : sB0;
    const uint16_t *a_n = cur ? sA0 : sA1, *b_n = cur ? sB0 : sB1;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int p = s & 1;
      if (s < 3) {
        frag(fa[p ^ 1], fb[p ^ 1], a_s, b_s, s + 1);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[p][i], fb[p][j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);         // one MFMA
          if (q < 6) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
        }
        __builtin_amdgcn_sched_barrier(0);
      } else {
        // this wave's loads of tile t + 1 must have landed before the barrier
        // publishes them; the memory clobber also keeps every LDS read of
        // tile t on this side of the barrier
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        frag(fa[p ^ 1], fb[p ^ 1], a_n, b_n, 0);  // on the last tile: unused reads of the idle stage
        // stage `cur` is free now; past the end the loads repeat the last
        // tile (in bounds) into it, which no one reads, so the block stays
        // branch free for the interleaving below
        const int kbyte = (t + 2 < nk ? t + 2 : nk - 1) * BK * 2;
        fill(rsA, gA, a_s, kbyte);
        fill(rsB, gB, b_s, kbyte);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[p][i], fb[p][j], acc[i][j], 0, 0, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);  // the six LDS reads first
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // one buffer load
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // no load may still target LDS at exit
  if constexpr (!PAGED) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int64_t col = n0 + wn + 32 * j + (lane & 31);
          __builtin_nontemporal_store(acc[i][j][r], C + row * N + col);
        }
  } else {
    __syncthreads();  // every lane has its A and B row addresses in registers
    if (threadIdx.x < BM2)
      s_row[threadIdx.x] = pm_addr(pm, oc + uint64_t(m0 + threadIdx.x) * uint64_t(N) * 4);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        float *crow = reinterpret_cast<float *>(s_row[rr]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          __builtin_nontemporal_store(acc[i][j][r], crow + n0 + wn + 32 * j + (lane & 31));
      }
  }
}


// ------------------------------------------------ paged tenant work (pages.h)
// Work is cut into 4 KiB units of each array (1024 words, 2048 bf16): a unit
// never straddles a page, so it is translated once.  The streaming kernels
// make each unit a buffer resource (see k_pg_triad).  Each kernel returns at
// once when the placement maps fewer than `need` pages (a failed placement
// maps none).
constexpr int64_t UNIT_W = 1024;  // 32-bit words per unit
constexpr int PGT_U = 4;          // vectors in flight per thread

__device__ __forceinline__ bool pg_ok(const PageMap &m, int64_t need) { return pm_pages(m) >= need; }

constexpr int BUF_NT = 2;  // buffer instruction aux: non-temporal
constexpr int64_t PGT_ONE_LAUNCH = 65536;  // workgroups of a triad job launched at once

template <bool DIRECT>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t unit_rsrc(const PageMap &m, uint64_t base,
                                                            int64_t o, int64_t bytes) {
  // a unit past the end maps unit 0 (always mapped) with an empty range
  const bool in = o < bytes;
  const int64_t valid = in ? ((bytes - o < 4096 ? bytes - o : 4096) & ~int64_t(15)) : 0;
  return __builtin_amdgcn_make_buffer_rsrc(pm_addr_t<DIRECT>(m, base + (in ? o : 0)), 0, int(valid),
                                           BUF_RSRC_DW3);
}

// Fills in the shape of the triad: workgroup g writes item g (PGT_U units of
// 4 KiB per array), thread t one 16-byte vector per unit.
template <bool DIRECT>
__global__ __launch_bounds__(256) void k_pg_triad_fill(PageMap m, int64_t need, uint64_t ob,
                                                       uint64_t oc, int64_t n, uint64_t s0) {
  if (pm_pages(m) < need) return;
  const int64_t bytes = 4 * n;
  const int64_t n_item = (bytes + PGT_U * 4096 - 1) / (PGT_U * 4096);
  const int tb = 16 * int(threadIdx.x);
  for (int64_t it = blockIdx.x; it < n_item; it += gridDim.x) {
#pragma unroll
    for (int u = 0; u < PGT_U; ++u) {
      const int64_t o = (it * PGT_U + u) << 12;
      const __amdgpu_buffer_rsrc_t rb = unit_rsrc<DIRECT>(m, ob, o, bytes);
      const __amdgpu_buffer_rsrc_t rc = unit_rsrc<DIRECT>(m, oc, o, bytes);
      f32x4 vb, vc;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint64_t h = splitmix(s0, uint64_t((o + tb) / 4 + e));
        vb[e] = 1.0f + float(h & 0xFFFF) * (1.0f / 65536.0f);
        vc[e] = 1.0f + float((h >> 16) & 0xFFFF) * (1.0f / 65536.0f);
      }
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, vb), rb, tb, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, vc), rc, tb, 0, 0);
    }
  }
  // the partial vector at the end
  const int64_t t0 = n & ~int64_t(3);
  if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
    const int64_t i = t0 + threadIdx.x;
    const uint64_t h = splitmix(s0, uint64_t(i));
    *reinterpret_cast<float *>(pm_addr(m, ob + uint64_t(i) * 4)) = 1.0f + float(h & 0xFFFF) * (1.0f / 65536.0f);
    *reinterpret_cast<float *>(pm_addr(m, oc + uint64_t(i) * 4)) =
        1.0f + float((h >> 16) & 0xFFFF) * (1.0f / 65536.0f);
  }
}

// a = b + s * c in the shape of k_triad: workgroup g streams item g, 16 KiB
// (PGT_U units of 4 KiB) of each array, thread t one 16-byte vector per unit.
// A launch may cover several sweeps: workgroup g then takes item g % n_item
// of sweep g / n_item.  Workgroups are dispatched in order, so the sweeps
// stream one after the other as separate launches would; a sweep rewrites
// the same values, so where two overlap at their boundary they agree.
// A unit never straddles a page, so each unit is one buffer resource whose
// base comes from a uniform (scalar) lookup -- all twelve of an item issued
// back to back -- and whose range stops at the array's last whole vector:
// lanes past it read zero and their stores are dropped, so no lane branches.
// The partial vector at the end is done elementwise.
template <bool DIRECT>
__global__ __launch_bounds__(256) void k_pg_triad(PageMap m, int64_t need, uint64_t oa, uint64_t ob,
                                                  uint64_t oc, float s, int64_t n) {
  if (pm_pages(m) < need) return;
  const int64_t bytes = 4 * n;
  const int64_t n_item = (bytes + PGT_U * 4096 - 1) / (PGT_U * 4096);
  const int tb = 16 * int(threadIdx.x);
  {
    const int64_t it = int64_t(blockIdx.x % uint32_t(n_item));  // n_item <= the grid < 2^31
    __amdgpu_buffer_rsrc_t ra[PGT_U], rb[PGT_U], rc[PGT_U];
#pragma unroll
    for (int u = 0; u < PGT_U; ++u) {
      const int64_t o = (it * PGT_U + u) << 12;
      ra[u] = unit_rsrc<DIRECT>(m, oa, o, bytes);
      rb[u] = unit_rsrc<DIRECT>(m, ob, o, bytes);
      rc[u] = unit_rsrc<DIRECT>(m, oc, o, bytes);
    }
    u32x4 x[PGT_U], y[PGT_U];
#pragma unroll
    for (int u = 0; u < PGT_U; ++u) {
      x[u] = __builtin_amdgcn_raw_buffer_load_b128(rb[u], tb, 0, BUF_NT);
      y[u] = __builtin_amdgcn_raw_buffer_load_b128(rc[u], tb, 0, BUF_NT);
    }
#pragma unroll
    for (int u = 0; u < PGT_U; ++u) {
      const f32x4 r = __builtin_bit_cast(f32x4, x[u]) + s * __builtin_bit_cast(f32x4, y[u]);
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, r), ra[u], tb, 0, BUF_NT);
    }
  }
  const int64_t t0 = n & ~int64_t(3);
  if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
    const uint64_t o = uint64_t(t0 + threadIdx.x) * 4;
    *reinterpret_cast<float *>(pm_addr(m, oa + o)) =
        *reinterpret_cast<const float *>(pm_addr(m, ob + o)) +
        s * *reinterpret_cast<const float *>(pm_addr(m, oc + o));
  }
}

template <bool DIRECT>
__global__ __launch_bounds__(256) void k_pg_hist_fill(PageMap m, int64_t need, uint64_t ok_,
                                                      int64_t n, uint64_t s0) {
  if (pm_pages(m) < need) return;
  const int64_t bytes = 4 * n;
  const int64_t n_item = (bytes + PGT_U * 4096 - 1) / (PGT_U * 4096);
  const int tb = 16 * int(threadIdx.x);
  for (int64_t it = blockIdx.x; it < n_item; it += gridDim.x) {
#pragma unroll
    for (int u = 0; u < PGT_U; ++u) {
      const int64_t o = (it * PGT_U + u) << 12;
      const __amdgpu_buffer_rsrc_t rk = unit_rsrc<DIRECT>(m, ok_, o, bytes);
      u32x4 k;
#pragma unroll
      for (int e = 0; e < 4; ++e) k[e] = uint32_t(splitmix(s0, uint64_t((o + tb) / 4 + e)));
      __builtin_amdgcn_raw_buffer_store_b128(k, rk, tb, 0, 0);
    }
  }
  const int64_t t0 = n & ~int64_t(3);
  if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
    const int64_t i = t0 + threadIdx.x;
    *reinterpret_cast<uint32_t *>(pm_addr(m, ok_ + uint64_t(i) * 4)) = uint32_t(splitmix(s0, uint64_t(i)));
  }
}

__global__ void k_pg_zero(PageMap m, int64_t need, uint64_t off, int64_t n_words) {
  if (!pg_ok(m, need)) return;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n_words;
       i += int64_t(gridDim.x) * blockDim.x)
    *reinterpret_cast<uint32_t *>(pm_addr(m, off + uint64_t(i) * 4)) = 0;
}

// Same LDS scheme as k_hist: a capped grid walks items of PGT_U units of
// keys (one 16-byte vector per thread per unit, buffer resources over the
// units as in the triad, so a lane past the end reads nothing it counts);
// the partial vector at the end elementwise.
template <bool DIRECT>
__global__ __launch_bounds__(HIST_THREADS) void k_pg_hist(PageMap m, int64_t need, uint64_t ok_,
                                                          int64_t n, uint32_t mask, uint64_t ob) {
  __shared__ uint32_t h[HIST_COPIES][SCHED_HIST_BINS];
  if (pm_pages(m) < need) return;
  for (int i = threadIdx.x; i < HIST_COPIES * SCHED_HIST_BINS; i += HIST_THREADS)
    (&h[0][0])[i] = 0;
  __syncthreads();
  uint32_t *mine = h[(threadIdx.x / 64) % HIST_COPIES];
  const int64_t bytes = 4 * n;
  const int64_t n_item = (bytes + PGT_U * 4096 - 1) / (PGT_U * 4096);
  const int tb = 16 * int(threadIdx.x);
  const int64_t full = bytes & ~int64_t(15);  // bytes of whole vectors
  for (int64_t it = blockIdx.x; it < n_item; it += gridDim.x) {
    __amdgpu_buffer_rsrc_t rk[PGT_U];
#pragma unroll
    for (int u = 0; u < PGT_U; ++u) rk[u] = unit_rsrc<DIRECT>(m, ok_, (it * PGT_U + u) << 12, bytes);
    u32x4 x[PGT_U];
#pragma unroll
    for (int u = 0; u < PGT_U; ++u) x[u] = __builtin_amdgcn_raw_buffer_load_b128(rk[u], tb, 0, BUF_NT);
#pragma unroll
    for (int u = 0; u < PGT_U; ++u) {
      if (((it * PGT_U + u) << 12) + tb + 16 <= full) {
        atomicAdd(&mine[x[u].x & mask], 1u);
        atomicAdd(&mine[x[u].y & mask], 1u);
        atomicAdd(&mine[x[u].z & mask], 1u);
        atomicAdd(&mine[x[u].w & mask], 1u);
      }
    }
  }
  const int64_t t0 = n & ~int64_t(3);
  if (blockIdx.x == 0 && threadIdx.x < (n & 3))
    atomicAdd(&mine[*reinterpret_cast<const uint32_t *>(pm_addr(m, ok_ + uint64_t(t0 + threadIdx.x) * 4)) &
                    mask],
              1u);
  __syncthreads();
  for (int b = threadIdx.x; b < SCHED_HIST_BINS; b += HIST_THREADS) {
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < HIST_COPIES; ++k) sum += h[k][b];
    if (sum) atomicAdd(reinterpret_cast<uint32_t *>(pm_addr(m, ob + uint64_t(b) * 4)), sum);
  }
}

// bf16 operand of n elements: items of PGT_U units (2048 elements each),
// thread t one 16-byte vector (8 elements) per unit.
template <bool DIRECT>
__global__ __launch_bounds__(256) void k_pg_gemm_fill(PageMap m, int64_t need, uint64_t off,
                                                      int64_t n, uint64_t s0) {
  if (pm_pages(m) < need) return;
  const int64_t bytes = 2 * n;
  const int64_t n_item = (bytes + PGT_U * 4096 - 1) / (PGT_U * 4096);
  const int tb = 16 * int(threadIdx.x);
  for (int64_t it = blockIdx.x; it < n_item; it += gridDim.x) {
#pragma unroll
    for (int u = 0; u < PGT_U; ++u) {
      const int64_t o = (it * PGT_U + u) << 12;
      const __amdgpu_buffer_rsrc_t rx = unit_rsrc<DIRECT>(m, off, o, bytes);
      u32x4 w;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uint32_t pair = 0;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const uint64_t z = splitmix(s0, uint64_t((o + tb) / 2 + 2 * e + hh));
          const float f = (float(int(z & 0xFF)) - 128.0f) * (1.0f / 64.0f);
          pair |= (__float_as_uint(f) >> 16) << (16 * hh);
        }
        w[e] = pair;
      }
      __builtin_amdgcn_raw_buffer_store_b128(w, rx, tb, 0, 0);
    }
  }
  // elements of the partial vector at the end
  const int64_t t0 = n & ~int64_t(7);
  if (blockIdx.x == 0 && threadIdx.x < (n & 7)) {
    const int64_t i = t0 + threadIdx.x;
    const uint64_t z = splitmix(s0, uint64_t(i));
    const float f = (float(int(z & 0xFF)) - 128.0f) * (1.0f / 64.0f);
    *reinterpret_cast<uint16_t *>(pm_addr(m, off + uint64_t(i) * 2)) = uint16_t(__float_as_uint(f) >> 16);
  }
}

// *out += sum over words i of (s_i | 1) * w_i (pages.h); one atomic per wave.
__global__ __launch_bounds__(256) void k_pg_digest(PageMap m, int64_t need, uint64_t off,
                                                   int64_t n, unsigned long long *out) {
  if (!pg_ok(m, need)) return;
  const int64_t units = (n + UNIT_W - 1) / UNIT_W;
  unsigned long long acc = 0;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const uint32_t *w = reinterpret_cast<const uint32_t *>(pm_addr(m, off + uint64_t(u) * 4096));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = q * 256 + threadIdx.x;
      const int64_t i = u * UNIT_W + k;
      if (i < n) acc += digest_term(uint64_t(i), w[k]);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
  if ((threadIdx.x & (WAVE - 1)) == 0 && acc) atomicAdd(out, acc);
}

__global__ void k_pg_gemm_samples(PageMap m, int64_t need, uint64_t oc, int64_t N, uint64_t seed,
                                  float *out) {
  const int k = threadIdx.x;
  if (k >= GEMM_SAMPLES) return;
  if (!pg_ok(m, need)) {
    out[k] = __int_as_float(0x7fc00000);  // NaN: nothing was computed
    return;
  }
  const uint64_t p = splitmix_at((seed << 32) ^ SAMPLE_KEY, uint64_t(k)) % uint64_t(N * N);
  out[k] = *reinterpret_cast<const float *>(pm_addr(m, oc + p * 4));
}
}  // namespace

extern "C" int sched_triad_fill(float *b, float *c, int64_t n, uint64_t seed, sched_stream_t st) {
  if (n < 0 || (n > 0 && (!b || !c))) return SCHED_E_INVALID;
  if (n == 0) return SCHED_OK;
  k_triad_fill<<<grid_cap(n, 256, 8192), 256, 0, (hipStream_t)st>>>(b, c, n, seed << 32);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

extern "C" int sched_triad(float *a, const float *b, const float *c, float s, int64_t n, int32_t iters,
                           sched_stream_t st) {
  if (n < 0 || iters < 0 || (n > 0 && (!a || !b || !c))) return SCHED_E_INVALID;
  if ((uintptr_t(a) | uintptr_t(b) | uintptr_t(c)) & 15) return SCHED_E_INVALID;
  if (n == 0) return SCHED_OK;
  const int grid = grid_cap((n + 3) / 4, 256 * TRIAD_U, 1 << 30);
  for (int32_t it = 0; it < iters; ++it) {
    SCHED_PROF_LAUNCH("k_triad", (hipStream_t)st,
                      (k_triad<<<grid, 256, 0, (hipStream_t)st>>>(a, b, c, s, n)));
    SCHED_HIP_TRY(hipGetLastError());
  }
  return SCHED_OK;
}

extern "C" int sched_hist_fill(uint32_t *keys, int64_t n, uint64_t seed, sched_stream_t st) {
  if (n < 0 || (n > 0 && !keys)) return SCHED_E_INVALID;
  if (n == 0) return SCHED_OK;
  k_hist_fill<<<grid_cap(n, 256, 8192), 256, 0, (hipStream_t)st>>>(keys, n, seed << 32);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

extern "C" int sched_hist(const uint32_t *keys, int64_t n, uint32_t mask, uint32_t *bins,
                          sched_stream_t st) {
  if (n < 0 || !bins || (n > 0 && !keys) || mask >= SCHED_HIST_BINS) return SCHED_E_INVALID;
  if (uintptr_t(keys) & 15) return SCHED_E_INVALID;
  k_zero_u32<<<4, 256, 0, (hipStream_t)st>>>(bins, SCHED_HIST_BINS);
  SCHED_HIP_TRY(hipGetLastError());
  if (n == 0) return SCHED_OK;
  SCHED_PROF_LAUNCH("k_hist", (hipStream_t)st,
                    (k_hist<<<grid_cap((n + 3) / 4, HIST_THREADS * 16, 256 * HIST_PER_CU), HIST_THREADS, 0,
                              (hipStream_t)st>>>(keys, n, mask, bins)));
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

extern "C" int sched_gemm_fill(uint16_t *x, int64_t rows, int64_t K, uint64_t seed, sched_stream_t st) {
  if (rows < 0 || K < 0 || (rows * K > 0 && !x)) return SCHED_E_INVALID;
  if (rows * K == 0) return SCHED_OK;
  k_gemm_fill<<<grid_cap(rows * K, 256, 8192), 256, 0, (hipStream_t)st>>>(x, rows, K, seed << 32);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

extern "C" int sched_gemm_bf16(const uint16_t *A, const uint16_t *Bt, float *C, int64_t M, int64_t N,
                               int64_t K, sched_stream_t st) {
  if (M <= 0 || N <= 0 || K <= 0 || !A || !Bt || !C) return SCHED_E_INVALID;
  if (M % BM || N % BN || K % BK) return SCHED_E_INVALID;
  if ((uintptr_t(A) | uintptr_t(Bt)) & 15) return SCHED_E_INVALID;
  // the 256-tile kernel addresses a 256-row operand panel with 32-bit buffer
  // offsets: 256 * K * 2 bytes must stay below 2^31
  if (M % BM2 == 0 && N % BN2 == 0 && K < (int64_t(1) << 22)) {
    const int64_t blocks = (M / BM2) * (N / BN2);
    if (blocks > 0x7fffffff) return SCHED_E_INVALID;
    SCHED_PROF_LAUNCH("k_gemm_bf16", (hipStream_t)st,
                      (k_gemm_bf16_256<false><<<int(blocks), GT2, 0, (hipStream_t)st>>>(
                          A, Bt, C, M, N, K, PageMap{}, 0, 0, 0, 0)));
    SCHED_HIP_TRY(hipGetLastError());
    return SCHED_OK;
  }
  const int64_t blocks = (M / BM) * (N / BN);
  if (blocks > 0x7fffffff) return SCHED_E_INVALID;
  SCHED_PROF_LAUNCH("k_gemm_bf16", (hipStream_t)st,
                    (k_gemm_bf16<<<int(blocks), GT, 0, (hipStream_t)st>>>(A, Bt, C, M, N, K)));
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

// ---------------------------------------------------------- paged wrappers
namespace schedk {

namespace {
int64_t pages_to(uint64_t off, int64_t bytes) {
  return bytes > 0 ? int64_t((off + uint64_t(bytes) - 1) >> PG_SHIFT) + 1 : 0;
}
int units_grid(int64_t units, int per, int cap) {
  return int(std::max<int64_t>(1, std::min<int64_t>((units + per - 1) / per, cap)));
}
bool off_ok(uint64_t off) { return (off & 4095) == 0; }
}  // namespace

int pgt_triad_fill(const PageMap &m, uint64_t ob, uint64_t oc, int64_t n, uint64_t seed,
                   hipStream_t s) {
  if (n <= 0) return n == 0 ? SCHED_OK : SCHED_E_INVALID;
  if (!off_ok(ob) || !off_ok(oc)) return SCHED_E_INVALID;
  const int64_t need = std::max(pages_to(ob, 4 * n), pages_to(oc, 4 * n));
  const int grid = units_grid((4 * n + PGT_U * 4096 - 1) / (PGT_U * 4096), 1, 1 << 30);
  if (m.direct)
    k_pg_triad_fill<true><<<grid, 256, 0, s>>>(m, need, ob, oc, n, seed << 32);
  else
    k_pg_triad_fill<false><<<grid, 256, 0, s>>>(m, need, ob, oc, n, seed << 32);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int pgt_triad(const PageMap &m, uint64_t oa, uint64_t ob, uint64_t oc, float sc, int64_t n,
              int32_t iters, hipStream_t s) {
  if (n < 0 || iters < 0 || !off_ok(oa) || !off_ok(ob) || !off_ok(oc)) return SCHED_E_INVALID;
  if (n == 0) return SCHED_OK;
  const int64_t need =
      std::max(pages_to(oa, 4 * n), std::max(pages_to(ob, 4 * n), pages_to(oc, 4 * n)));
  // Jobs up to PGT_ONE_LAUNCH workgroups in all (~100 MiB per array over 10
  // sweeps) run their sweeps in one launch (item-major inside a sweep, sweep
  // after sweep): there the launches, not the bytes, cost the time.  Larger
  // ones launch sweep by sweep, so that the admission kernels of the serving
  // loop, which share the device, get workgroup slots between long launches.
  const int64_t n_item = (4 * n + PGT_U * 4096 - 1) / (PGT_U * 4096);
  const bool one = n_item * iters <= PGT_ONE_LAUNCH;
  const int grid = int(one ? n_item * iters : n_item);
  for (int32_t it = 0; it < (one ? (iters > 0 ? 1 : 0) : iters); ++it) {
    if (m.direct)
      SCHED_PROF_LAUNCH("k_pg_triad", s,
                        (k_pg_triad<true><<<grid, 256, 0, s>>>(m, need, oa, ob, oc, sc, n)));
    else
      SCHED_PROF_LAUNCH("k_pg_triad", s,
                        (k_pg_triad<false><<<grid, 256, 0, s>>>(m, need, oa, ob, oc, sc, n)));
    SCHED_HIP_TRY(hipGetLastError());
  }
  return SCHED_OK;
}

int pgt_hist_fill(const PageMap &m, uint64_t ok_, int64_t n, uint64_t seed, hipStream_t s) {
  if (n < 0 || !off_ok(ok_)) return SCHED_E_INVALID;
  if (n == 0) return SCHED_OK;
  const int grid = units_grid((4 * n + PGT_U * 4096 - 1) / (PGT_U * 4096), 1, 1 << 30);
  if (m.direct)
    k_pg_hist_fill<true><<<grid, 256, 0, s>>>(m, pages_to(ok_, 4 * n), ok_, n, seed << 32);
  else
    k_pg_hist_fill<false><<<grid, 256, 0, s>>>(m, pages_to(ok_, 4 * n), ok_, n, seed << 32);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int pgt_hist(const PageMap &m, uint64_t ok_, int64_t n, uint32_t mask, uint64_t ob, hipStream_t s) {
  if (n < 0 || mask >= SCHED_HIST_BINS || !off_ok(ok_) || !off_ok(ob)) return SCHED_E_INVALID;
  const int64_t need_b = pages_to(ob, 4 * SCHED_HIST_BINS);
  k_pg_zero<<<4, 256, 0, s>>>(m, need_b, ob, SCHED_HIST_BINS);
  SCHED_HIP_TRY(hipGetLastError());
  if (n == 0) return SCHED_OK;
  const int64_t need = std::max(need_b, pages_to(ok_, 4 * n));
  const int grid = units_grid((4 * n + PGT_U * 4096 - 1) / (PGT_U * 4096), 1, 256 * HIST_PER_CU);
  if (m.direct)
    SCHED_PROF_LAUNCH("k_pg_hist", s,
                      (k_pg_hist<true><<<grid, HIST_THREADS, 0, s>>>(m, need, ok_, n, mask, ob)));
  else
    SCHED_PROF_LAUNCH("k_pg_hist", s,
                      (k_pg_hist<false><<<grid, HIST_THREADS, 0, s>>>(m, need, ok_, n, mask, ob)));
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int pgt_gemm_fill(const PageMap &m, uint64_t off, int64_t rows, int64_t K, uint64_t seed,
                  hipStream_t s) {
  const int64_t n = rows * K;
  if (rows < 0 || K < 0 || !off_ok(off)) return SCHED_E_INVALID;
  if (n == 0) return SCHED_OK;
  const int grid = units_grid((2 * n + PGT_U * 4096 - 1) / (PGT_U * 4096), 1, 1 << 30);
  if (m.direct)
    k_pg_gemm_fill<true><<<grid, 256, 0, s>>>(m, pages_to(off, 2 * n), off, n, seed << 32);
  else
    k_pg_gemm_fill<false><<<grid, 256, 0, s>>>(m, pages_to(off, 2 * n), off, n, seed << 32);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int pgt_gemm(const PageMap &m, uint64_t oa, uint64_t ob, uint64_t oc, int64_t N, hipStream_t s) {
  // each operand row inside one page: 2N and 4N divide the page size, and
  // the arrays start at page boundaries
  if (N < BM2 || N > (PG_BYTES / 4) || (N & (N - 1)) || ((oa | ob | oc) & (PG_BYTES - 1)))
    return SCHED_E_INVALID;
  const int64_t need = std::max(pages_to(oa, 2 * N * N),
                                std::max(pages_to(ob, 2 * N * N), pages_to(oc, 4 * N * N)));
  const int64_t blocks = (N / BM2) * (N / BN2);
  SCHED_PROF_LAUNCH("k_gemm_bf16_paged", s,
                    (k_gemm_bf16_256<true><<<int(blocks), GT2, 0, s>>>(nullptr, nullptr, nullptr, N,
                                                                       N, N, m, need, oa, ob, oc)));
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int pgt_digest(const PageMap &m, uint64_t off, int64_t n, unsigned long long *out, hipStream_t s) {
  if (n < 0 || !off_ok(off) || !out) return SCHED_E_INVALID;
  if (n == 0) return SCHED_OK;
  k_pg_digest<<<units_grid((n + UNIT_W - 1) / UNIT_W, 1, 2048), 256, 0, s>>>(
      m, pages_to(off, 4 * n), off, n, out);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

int pgt_gemm_samples(const PageMap &m, uint64_t oc, int64_t N, uint64_t seed, float *out,
                     hipStream_t s) {
  if (N <= 0 || !off_ok(oc) || !out) return SCHED_E_INVALID;
  k_pg_gemm_samples<<<1, 64, 0, s>>>(m, pages_to(oc, 4 * N * N), oc, N, seed, out);
  SCHED_HIP_TRY(hipGetLastError());
  return SCHED_OK;
}

}  // namespace schedk
