// Exclusive prefix sum of the per-Gaussian tile counts -> instance offsets
// and the instance total.  This replaces the atomic append of Algorithm 1
// (atomicAdd on a global count) with a deterministic compaction, so the
// instance order -- and with it the stable sort's permutation -- is unique.
//
// Single pass with decoupled look-back: each workgroup takes a partition
// index from an atomic ticket (so every partition it waits on has already
// started), scans 4096 counts locally, publishes its aggregate, and wave 0
// walks back over predecessors 64 at a time.
#include "gs_device.h"
#include "gs_internal.h"

namespace gs {
namespace {

constexpr uint64_t kScanAgg = 1ull << 32;
constexpr uint64_t kScanInc = 2ull << 32;

__global__ __launch_bounds__(kBlock) void k_scan_init(uint64_t* status, int parts,
                                                      uint32_t* ticket, uint32_t* total) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < parts) status[i] = 0;
  if (i == 0) {
    *ticket = 0;
    *total = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan(uint32_t* __restrict__ data, int n,
                                                 uint64_t* __restrict__ status,
                                                 uint32_t* __restrict__ ticket,
                                                 uint32_t* __restrict__ total) {
  __shared__ uint32_t s_part;
  __shared__ uint32_t s_wave[kBlock / 64];
  __shared__ uint32_t s_prefix;
  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  if (t == 0) s_part = atomicAdd(ticket, 1u);
  __syncthreads();
  const int part = (int)s_part;
  const int64_t base = (int64_t)part * kScanPart + (int64_t)t * kScanItems;

  uint32_t v[kScanItems];
  if (base + kScanItems <= n) {
    const uint4* src = reinterpret_cast<const uint4*>(data + base);
#pragma unroll
    for (int j = 0; j < kScanItems / 4; ++j) {
      const uint4 u = src[j];
      v[4 * j] = u.x; v[4 * j + 1] = u.y; v[4 * j + 2] = u.z; v[4 * j + 3] = u.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) v[j] = (base + j < n) ? data[base + j] : 0u;
  }
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) sum += v[j];
  const uint32_t incl = wave_incl_scan(sum);
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  uint32_t wave_off = 0, agg = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    const uint32_t x = s_wave[w];
    wave_off += (w < wave) ? x : 0u;
    agg += x;
  }

  if (wave == 0) {
    uint32_t excl = 0;
    if (part == 0) {
      if (lane == 0) st_agent64(&status[0], kScanInc | agg);
    } else {
      if (lane == 0) st_agent64(&status[part], kScanAgg | agg);
      int j = part - 1;
      while (true) {
        const int idx = j - lane;
        uint64_t s = idx >= 0 ? ld_agent64(&status[idx]) : kScanInc;
        while (ballot((s >> 32) == 0) != 0ull) {
          if ((s >> 32) == 0) s = ld_agent64(&status[idx]);
        }
        const uint64_t inc = ballot((s >> 32) == 2);
        if (inc) {
          const int first = __builtin_ctzll(inc);
          excl += wave_sum_u32(lane <= first ? (uint32_t)s : 0u);
          break;
        }
        excl += wave_sum_u32((uint32_t)s);
        j -= 64;
      }
      if (lane == 0) st_agent64(&status[part], kScanInc | (uint64_t)(excl + agg));
    }
    if (lane == 0) {
      s_prefix = excl;
      if ((int64_t)(part + 1) * kScanPart >= n) *total = excl + agg;
    }
  }
  __syncthreads();
  uint32_t run = s_prefix + wave_off + incl - sum;
  if (base + kScanItems <= n) {
    uint4* dst = reinterpret_cast<uint4*>(data + base);
#pragma unroll
    for (int j = 0; j < kScanItems / 4; ++j) {
      uint4 u;
      u.x = run; run += v[4 * j];
      u.y = run; run += v[4 * j + 1];
      u.z = run; run += v[4 * j + 2];
      u.w = run; run += v[4 * j + 3];
      dst[j] = u;
    }
  } else {
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      if (base + j < n) data[base + j] = run;
      run += v[j];
    }
  }
}

}  // namespace

ScanLayout scan_layout(int64_t n) {
  ScanLayout L;
  L.parts = (int)((n + kScanPart - 1) / kScanPart);
  L.status = 0;
  L.ticket = align_up((size_t)L.parts * 8, 256);
  L.bytes = L.ticket + 256;
  return L;
}

hipError_t launch_scan(int n, uint32_t* data, uint32_t* total, void* ws, const ScanLayout& L,
                       hipStream_t st) {
  char* w = static_cast<char*>(ws);
  uint64_t* status = reinterpret_cast<uint64_t*>(w + L.status);
  uint32_t* ticket = reinterpret_cast<uint32_t*>(w + L.ticket);
  const int init_blocks = (L.parts + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_scan_init, dim3(init_blocks > 0 ? init_blocks : 1), dim3(kBlock), 0, st,
                     status, L.parts, ticket, total);
  if (L.parts > 0)
    hipLaunchKernelGGL(k_scan, dim3(L.parts), dim3(kBlock), 0, st, data, n, status, ticket, total);
  return hipGetLastError();
}

}  // namespace gs
