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
#include "prof.h"

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

__global__ __launch_bounds__(GT2, 1) void k_gemm_bf16_256(const uint16_t *__restrict__ A,
                                                          const uint16_t *__restrict__ Bt,
                                                          float *__restrict__ C, int64_t M,
                                                          int64_t N, int64_t K) {
  __shared__ __attribute__((aligned(1024))) uint16_t sA0[BM2 * ROW2];
  __shared__ __attribute__((aligned(1024))) uint16_t sA1[BM2 * ROW2];
  __shared__ __attribute__((aligned(1024))) uint16_t sB0[BN2 * ROW2];
  __shared__ __attribute__((aligned(1024))) uint16_t sB1[BN2 * ROW2];
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
  const __amdgpu_buffer_rsrc_t rsA =
      __builtin_amdgcn_make_buffer_rsrc((void *)(A + m0 * K), 0, int(BM2 * K * 2), BUF_RSRC_DW3);
  const __amdgpu_buffer_rsrc_t rsB =
      __builtin_amdgcn_make_buffer_rsrc((void *)(Bt + n0 * K), 0, int(BN2 * K * 2), BUF_RSRC_DW3);
  int voff[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = 8 * (wave + 8 * j) + (lane >> 3);  // wave instruction j fills rows 8G .. 8G + 7
    voff[j] = (r * int(K) + ((lane & 7) ^ ((r >> 1) & 7)) * 8) * 2;
  }
  auto fill = [&](__amdgpu_buffer_rsrc_t rs, uint16_t *stage, int kbyte) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)(stage + (wave + 8 * j) * 8 * ROW2),
                                               16, voff[j], kbyte, 0, 0);
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

  fill(rsA, sA0, 0);
  fill(rsB, sB0, 0);
  if (nk > 1) {
    fill(rsA, sA1, BK * 2);
    fill(rsB, sB1, BK * 2);
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
        fill(rsA, a_s, kbyte);
        fill(rsB, b_s, kbyte);
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
                      (k_gemm_bf16_256<<<int(blocks), GT2, 0, (hipStream_t)st>>>(A, Bt, C, M, N, K)));
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
