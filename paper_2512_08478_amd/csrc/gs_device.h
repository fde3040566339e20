// Device helpers for wave64 (gfx950): lane queries, ballots, wave scans,
// DPP group sums and agent-scope atomic loads/stores for cross-workgroup
// look-back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// bits of lanes below this one
__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += shfl_u32(v, l ^ d);
  return v;
}

// x from another lane of the same 16-lane row by the DPP control CTRL
// (lanes whose source is outside the row read 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, true));
}

// Sum of v over each group of 8 lanes, left in the group's last lane (7,
// 15, ..., 63): DPP row shifts by 1, 2 and 4 accumulate the 8 lanes ending
// at each lane, and lanes shifted in from outside a 16-lane row read 0.
__device__ __forceinline__ float oct_sum_dpp(float v) {
  v += dpp_f32<0x111, 0xF>(v);  // row_shr:1
  v += dpp_f32<0x112, 0xF>(v);  // row_shr:2
  v += dpp_f32<0x114, 0xF>(v);  // row_shr:4
  return v;
}

// u32 from another lane by the DPP control CTRL; lanes of rows outside
// ROW_MASK, and lanes whose source lies outside their row, read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xF, true);
}

// Inclusive scan of u32 over the 64 lanes on the DPP paths (no LDS): row
// shifts by 1, 2, 4 and 8 scan each 16-lane row; row_bcast:15 then adds
// the total of rows 0 and 2 to rows 1 and 3, and row_bcast:31 adds the
// total of lanes 0-31 to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t v) {
  v += dpp_u32<0x111, 0xF>(v);  // row_shr:1
  v += dpp_u32<0x112, 0xF>(v);  // row_shr:2
  v += dpp_u32<0x114, 0xF>(v);  // row_shr:4
  v += dpp_u32<0x118, 0xF>(v);  // row_shr:8
  v += dpp_u32<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_u32<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) { return wave_incl_scan_dpp(v); }

// Inclusive max-scan of u32 over the 64 lanes, on the same DPP paths.
__device__ __forceinline__ uint32_t wave_incl_max_dpp(uint32_t v) {
  v = max(v, dpp_u32<0x111, 0xF>(v));
  v = max(v, dpp_u32<0x112, 0xF>(v));
  v = max(v, dpp_u32<0x114, 0xF>(v));
  v = max(v, dpp_u32<0x118, 0xF>(v));
  v = max(v, dpp_u32<0x142, 0xA>(v));
  v = max(v, dpp_u32<0x143, 0xC>(v));
  return v;
}

// The value of the next lower lane (0 for lane 0): DPP wave_shr:1.
__device__ __forceinline__ uint32_t wave_shr1(uint32_t v) { return dpp_u32<0x138, 0xF>(v); }

// Lanes of the wave whose `d` (BITS wide) equals this lane's, among `active`.
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
  uint64_t m = active;
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const uint64_t v = ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? v : ~v;
  }
  return m;
}

// Agent-scope (all XCDs) relaxed atomics for look-back status words.  The
// payload and its flag live in the same word, so no further ordering is
// needed.
__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// a*d - b*c with one rounding error (Kahan's fma method).
__device__ __forceinline__ float det2(float a, float b, float c, float d) {
  const float w = b * c;
  const float e = fmaf(-b, c, w);
  const float f = fmaf(a, d, -w);
  return f + e;
}

}  // namespace gs
