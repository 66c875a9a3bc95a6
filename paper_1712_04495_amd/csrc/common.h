// Shared device/host helpers for the co-scheduler library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cosched.h"

#define SCHED_HIP_TRY(expr)                                    \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) {                                    \
      sched_note_hip_error(_e, #expr, __FILE__, __LINE__);     \
      return SCHED_E_INTERNAL;                                 \
    }                                                          \
  } while (0)

void sched_note_hip_error(hipError_t e, const char *what, const char *file, int line);

namespace schedk {

constexpr int WAVE = 64;

// ---- relaxed, agent-scope atomics (visible across all XCDs) --------------
template <typename T>
__device__ __forceinline__ T ld_relaxed(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T add_relaxed(T *p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T min_relaxed(T *p, T v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T max_relaxed(T *p, T v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Saturating add for non-negative values bounded by cap (cap < 2^62).
__device__ __forceinline__ int64_t sat_add(int64_t a, int64_t b, int64_t cap) {
  int64_t s = a + b;
  return s < cap ? s : cap;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// ---- wave-level primitives (64 lanes) ------------------------------------
__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}
__device__ __forceinline__ int64_t wave_min(int64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    int64_t u = __shfl_xor(v, off, WAVE);
    v = u < v ? u : v;
  }
  return v;
}
__device__ __forceinline__ int64_t wave_max(int64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    int64_t u = __shfl_xor(v, off, WAVE);
    v = u > v ? u : v;
  }
  return v;
}
// Inclusive saturating prefix over lanes in lane order.
__device__ __forceinline__ int64_t wave_incl_scan_sat(int64_t v, int64_t cap) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    int64_t u = __shfl_up(v, off, WAVE);
    if (lane >= off) v = sat_add(v, u, cap);
  }
  return v;
}
// DPP lane moves of a 64-bit value (both halves moved with the same control);
// lanes without a source, or outside row_mask, receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int64_t dpp_move64(int64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(v)), CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(uint64_t(v) >> 32)), CTRL, ROW_MASK,
                                             0xF, true);
  return int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}
// Inclusive saturating prefix with DPP: shifts by 1, 2, 4, 8 inside each row
// of 16 lanes, then lane 15 of rows 0/2 is broadcast into rows 1/3 and lane 31
// into rows 2/3 (the GFX9 row broadcasts).  All operands stay in VGPRs.
__device__ __forceinline__ int64_t wave_incl_scan_sat_dpp(int64_t v, int64_t cap) {
  v = sat_add(v, dpp_move64<0x111, 0xF>(v), cap);  // row_shr:1
  v = sat_add(v, dpp_move64<0x112, 0xF>(v), cap);  // row_shr:2
  v = sat_add(v, dpp_move64<0x114, 0xF>(v), cap);  // row_shr:4
  v = sat_add(v, dpp_move64<0x118, 0xF>(v), cap);  // row_shr:8
  v = sat_add(v, dpp_move64<0x142, 0xA>(v), cap);  // row_bcast:15 into rows 1, 3
  v = sat_add(v, dpp_move64<0x143, 0xC>(v), cap);  // row_bcast:31 into rows 2, 3
  return v;
}
// Inclusive plain prefix with the same DPP steps, for values small enough
// that the 64-lane total cannot overflow.
__device__ __forceinline__ int64_t wave_incl_scan_dpp(int64_t v) {
  v += dpp_move64<0x111, 0xF>(v);  // row_shr:1
  v += dpp_move64<0x112, 0xF>(v);  // row_shr:2
  v += dpp_move64<0x114, 0xF>(v);  // row_shr:4
  v += dpp_move64<0x118, 0xF>(v);  // row_shr:8
  v += dpp_move64<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_move64<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
  return v;
}
// 32-bit unsigned variants: saturating add (v_add_u32 with clamp) and the
// same DPP prefix steps.  A saturated prefix only ever stands for "more than
// any bound below 2^32 - 1", so comparisons against such a bound stay exact.
__device__ __forceinline__ uint32_t add_sat_u32(uint32_t a, uint32_t b) {
  return __builtin_elementwise_add_sat(a, b);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_move32(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, ROW_MASK, 0xF, true));
}
__device__ __forceinline__ uint32_t wave_incl_scan_sat32_dpp(uint32_t v) {
  v = add_sat_u32(v, dpp_move32<0x111, 0xF>(v));  // row_shr:1
  v = add_sat_u32(v, dpp_move32<0x112, 0xF>(v));  // row_shr:2
  v = add_sat_u32(v, dpp_move32<0x114, 0xF>(v));  // row_shr:4
  v = add_sat_u32(v, dpp_move32<0x118, 0xF>(v));  // row_shr:8
  v = add_sat_u32(v, dpp_move32<0x142, 0xA>(v));  // row_bcast:15 into rows 1, 3
  v = add_sat_u32(v, dpp_move32<0x143, 0xC>(v));  // row_bcast:31 into rows 2, 3
  return v;
}
__device__ __forceinline__ uint32_t wave_prev_lane32(uint32_t v) { return dpp_move32<0x138, 0xF>(v); }
// Value of the previous lane (0 for lane 0): wave_shr:1.
__device__ __forceinline__ int64_t wave_prev_lane64(int64_t v) { return dpp_move64<0x138, 0xF>(v); }
// Value of a uniform lane, read into scalar registers.
__device__ __forceinline__ int64_t read_lane64(int64_t v, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane(int(uint32_t(v)), lane);
  const uint32_t hi = __builtin_amdgcn_readlane(int(uint32_t(uint64_t(v) >> 32)), lane);
  return int64_t((uint64_t(hi) << 32) | lo);
}

// Inclusive plain prefix over lanes (no saturation).
__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    int64_t u = __shfl_up(v, off, WAVE);
    if (lane >= off) v += u;
  }
  return v;
}

// ---- block-level primitives; `red` is LDS of at least NW int64 -----------
template <int NT>
__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t *red) {
  constexpr int NW = NT / WAVE;
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}
template <int NT>
__device__ __forceinline__ int64_t block_min(int64_t v, int64_t *red) {
  constexpr int NW = NT / WAVE;
  v = wave_min(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  int64_t s = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) s = red[i] < s ? red[i] : s;
  return s;
}
template <int NT>
__device__ __forceinline__ int64_t block_max(int64_t v, int64_t *red) {
  constexpr int NW = NT / WAVE;
  v = wave_max(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  int64_t s = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) s = red[i] > s ? red[i] : s;
  return s;
}
// Exclusive saturating scan over threads in thread order; returns the
// exclusive prefix and writes the block total to *total.
template <int NT>
__device__ __forceinline__ int64_t block_excl_scan_sat(int64_t v, int64_t cap, int64_t *red,
                                                       int64_t *total) {
  constexpr int NW = NT / WAVE;
  const int w = threadIdx.x / WAVE;
  const int64_t incl = wave_incl_scan_sat(v, cap);
  int64_t wexcl = __shfl_up(incl, 1, WAVE);
  if (lane_id() == 0) wexcl = 0;
  __syncthreads();
  if (lane_id() == WAVE - 1) red[w] = incl;
  __syncthreads();
  int64_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    if (i < w) before = sat_add(before, red[i], cap);
    tot = sat_add(tot, red[i], cap);
  }
  *total = tot;
  return sat_add(before, wexcl, cap);
}
// Exclusive plain scan (no saturation).
template <int NT>
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *red, int64_t *total) {
  constexpr int NW = NT / WAVE;
  const int w = threadIdx.x / WAVE;
  const int64_t incl = wave_incl_scan(v);
  __syncthreads();
  if (lane_id() == WAVE - 1) red[w] = incl;
  __syncthreads();
  int64_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    if (i < w) before += red[i];
    tot += red[i];
  }
  *total = tot;
  return before + incl - v;
}

}  // namespace schedk
