// (tile, depth) key generation and the per-frame GPU radix sort
// (Algorithm 1, Radix Sort; Section 3.4).
//
// The sort is a stable least-significant-digit radix sort in the onesweep
// style: one histogram of every digit (fused into key generation), then one
// kernel per digit.  Each radix pass
//   1. takes a partition of 4096 keys by atomic ticket (every partition it
//      waits on has started),
//   2. ranks the keys of each wave with ballot-based digit matching (one
//      ballot per digit bit; equal digits keep index order, so the sort is
//      stable),
//   3. publishes its per-digit counts and looks back over earlier
//      partitions for their prefixes (one thread per digit),
//   4. stages the keys in LDS in sorted order and writes them out, so
//      consecutive threads write consecutive addresses of one digit run.
// All kernels read the instance count from device memory, so the pipeline
// runs without a host round trip.
#include "gs_device.h"
#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kHistMax = 2048;  // passes * bins upper bound (8 x 256, 10 x 128, 11 x 64)

// Zero the per-call sort state; count = min(total, capacity) and the
// capacity flag.
__global__ __launch_bounds__(kBlock) void k_sort_init(uint32_t* hist, int hist_len,
                                                      uint32_t* tickets, int passes,
                                                      uint32_t* lookback0, int lb_len,
                                                      uint32_t* ranges, int ranges_len,
                                                      uint32_t* count, const uint32_t* total_src,
                                                      uint32_t host_total, int64_t capacity,
                                                      uint32_t* status_flag) {
  const int stride = gridDim.x * kBlock;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < lb_len; i += stride) lookback0[i] = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < ranges_len; i += stride) ranges[i] = 0;
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < hist_len; i += kBlock) hist[i] = 0;
    if ((int)threadIdx.x < passes) tickets[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
      const uint32_t tot = total_src ? *total_src : host_total;
      const bool over = (int64_t)tot > capacity;
      *count = over ? (uint32_t)capacity : tot;
      if (status_flag) *status_flag = over ? 1u : 0u;
    }
  }
}

// Add one digit per lane to an LDS histogram with one atomic per distinct
// digit in the wave.
template <int BITS>
__device__ __forceinline__ void wave_hist_add(uint32_t* h, uint32_t d, bool valid) {
  const uint64_t active = ballot(valid);
  if (!active) return;
  const uint64_t peers = match_digit<BITS>(d, active);
  if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__builtin_popcountll(peers));
}

template <int BITS>
__device__ __forceinline__ void flush_hist(const uint32_t* s_hist, uint32_t* hist, int len) {
  for (int b = threadIdx.x; b < len; b += kBlock) {
    const uint32_t v = s_hist[b];
    if (v) atomicAdd(&hist[b], v);
  }
}

// Keys for every (visible Gaussian, tile of its rect), Gaussian-major and
// row-major within the rect; a block expands 256 Gaussians' instances with
// a binary search over their offsets, so big splats do not stall a thread.
template <int BITS>
__global__ __launch_bounds__(kBlock) void k_keygen(int n, const gs_splat* __restrict__ splats,
                                                   const uint32_t* __restrict__ offsets,
                                                   const uint32_t* __restrict__ total,
                                                   const uint32_t* __restrict__ count,
                                                   int tiles_x, int passes,
                                                   uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals,
                                                   uint32_t* __restrict__ hist) {
  constexpr int NB = 1 << BITS;
  __shared__ uint32_t s_off[kBlock + 1];
  __shared__ uint32_t s_lo[kBlock], s_hi[kBlock], s_depth[kBlock];
  __shared__ uint32_t s_hist[kHistMax];
  const int t = threadIdx.x;
  const uint32_t cnt = *count, tot = *total;
  for (int b = t; b < passes * NB; b += kBlock) s_hist[b] = 0;
  for (int chunk = blockIdx.x; chunk * kBlock < n; chunk += gridDim.x) {
    const int g0 = chunk * kBlock, g = g0 + t;
    __syncthreads();
    s_off[t] = g < n ? offsets[g] : tot;
    if (t == 0) s_off[kBlock] = (g0 + kBlock < n) ? offsets[g0 + kBlock] : tot;
    if (g < n) {
      const float4 r2 = reinterpret_cast<const float4*>(splats + g)[2];
      s_depth[t] = __float_as_uint(r2.y);
      s_lo[t] = __float_as_uint(r2.z);
      s_hi[t] = __float_as_uint(r2.w);
    }
    __syncthreads();
    const uint32_t begin = s_off[0], end = s_off[kBlock];
    for (uint32_t kk = begin; kk < end; kk += kBlock) {
      const uint32_t k = kk + t;
      const bool valid = k < end && k < cnt;
      uint64_t key = 0;
      if (valid) {
        int lo = 0, hi = kBlock - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= k) lo = mid; else hi = mid - 1;
        }
        const uint32_t local = k - s_off[lo];
        const uint32_t rl = s_lo[lo], rh = s_hi[lo];
        const uint32_t tx0 = rl & 0xFFFFu, ty0 = rl >> 16, tx1 = rh & 0xFFFFu;
        const uint32_t w = tx1 - tx0 + 1;
        const uint32_t ry = local / w;
        const uint32_t tile = (ty0 + ry) * (uint32_t)tiles_x + tx0 + (local - ry * w);
        key = ((uint64_t)tile << 32) | s_depth[lo];
        keys[k] = key;
        vals[k] = (uint32_t)(g0 + lo);
      }
      for (int p = 0; p < passes; ++p)
        wave_hist_add<BITS>(s_hist + p * NB, (uint32_t)(key >> (p * BITS)) & (NB - 1), valid);
    }
  }
  __syncthreads();
  flush_hist<BITS>(s_hist, hist, passes * NB);
}

// Digit histograms of an existing key array (for the stand-alone sort).
template <int BITS>
__global__ __launch_bounds__(kBlock) void k_histogram(int64_t n, const uint64_t* __restrict__ keys,
                                                      int passes, uint32_t* __restrict__ hist) {
  constexpr int NB = 1 << BITS;
  __shared__ uint32_t s_hist[kHistMax];
  for (int b = threadIdx.x; b < passes * NB; b += kBlock) s_hist[b] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    const uint64_t key = valid ? keys[i] : 0ull;
    for (int p = 0; p < passes; ++p)
      wave_hist_add<BITS>(s_hist + p * NB, (uint32_t)(key >> (p * BITS)) & (NB - 1), valid);
  }
  __syncthreads();
  flush_hist<BITS>(s_hist, hist, passes * NB);
}

template <int BITS>
__global__ __launch_bounds__(kBlock) void k_onesweep(const uint64_t* __restrict__ kin,
                                                     const uint32_t* __restrict__ vin,
                                                     uint64_t* __restrict__ kout,
                                                     uint32_t* __restrict__ vout,
                                                     const uint32_t* __restrict__ count, int shift,
                                                     const uint32_t* __restrict__ hist,
                                                     uint32_t* __restrict__ ticket,
                                                     uint32_t* __restrict__ lb,
                                                     uint32_t* __restrict__ lb_next) {
  constexpr int NB = 1 << BITS;
  constexpr int NW = kBlock / 64;
  __shared__ uint32_t s_whist[NW][NB];
  __shared__ uint32_t s_local[NB];
  __shared__ uint32_t s_gbase[NB];
  __shared__ uint64_t s_keys[kSortPart];
  __shared__ uint8_t s_dig[kSortPart];
  __shared__ uint32_t s_scan[2][NW];
  __shared__ uint32_t s_part;

  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  if (t == 0) s_part = atomicAdd(ticket, 1u);
  for (int b = t; b < NW * NB; b += kBlock) (&s_whist[0][0])[b] = 0;
  __syncthreads();
  const uint32_t part = s_part;
  const uint32_t n = *count;
  const uint32_t base = part * kSortPart;
  if (base >= n) return;
  for (int b = t; b < NB; b += kBlock) lb_next[part * NB + b] = 0;

  // warp-striped load: wave w owns keys [w*64*ITEMS, (w+1)*64*ITEMS)
  uint64_t k[kSortItems];
  uint32_t pos[kSortItems];
  const uint32_t wbase = base + wave * 64 * kSortItems + lane;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t idx = wbase + i * 64;
    k[i] = idx < n ? kin[idx] : ~0ull;  // past the end: last digit, ranked last
  }
  // wave-local ranks via digit matching
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t d = (uint32_t)(k[i] >> shift) & (NB - 1);
    const uint64_t peers = match_digit<BITS>(d, ~0ull);
    const uint32_t c = s_whist[wave][d];
    pos[i] = c + (uint32_t)__builtin_popcountll(peers & lt);
    if ((peers & lt) == 0) s_whist[wave][d] = c + (uint32_t)__builtin_popcountll(peers);
  }
  __syncthreads();

  // per digit: offsets of each wave, partition total, and global digit start
  uint32_t tot = 0, gcount = 0;
  if (t < NB) {
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t x = s_whist[w][t];
      s_whist[w][t] = run;
      run += x;
    }
    tot = run;
    gcount = hist[t];
    st_agent(&lb[part * NB + t], (part == 0 ? kLbFlagInc : kLbFlagAgg) | tot);
  }
  const uint32_t inc_tot = wave_incl_scan(tot);
  const uint32_t inc_g = wave_incl_scan(gcount);
  if (lane == 63) {
    s_scan[0][wave] = inc_tot;
    s_scan[1][wave] = inc_g;
  }
  __syncthreads();
  if (t < NB) {
    uint32_t off_tot = 0, off_g = 0;
    for (int w = 0; w < wave; ++w) {
      off_tot += s_scan[0][w];
      off_g += s_scan[1][w];
    }
    const uint32_t local = off_tot + inc_tot - tot;
    const uint32_t gstart = off_g + inc_g - gcount;
    uint32_t prefix = 0;
    if (part > 0) {
      int j = (int)part - 1;
      while (true) {
        const uint32_t s = ld_agent(&lb[j * NB + t]);
        if ((s & (kLbFlagAgg | kLbFlagInc)) == 0) continue;
        prefix += s & kLbValue;
        if (s & kLbFlagInc) break;
        --j;
      }
      st_agent(&lb[part * NB + t], kLbFlagInc | (prefix + tot));
    }
    s_local[t] = local;
    s_gbase[t] = gstart + prefix - local;
  }
  __syncthreads();

  // keys into LDS in partition-sorted order
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t d = (uint32_t)(k[i] >> shift) & (NB - 1);
    pos[i] += s_local[d] + s_whist[wave][d];
    s_keys[pos[i]] = k[i];
  }
  __syncthreads();
  for (int j = t; j < kSortPart; j += kBlock) {
    const uint64_t key = s_keys[j];
    const uint32_t d = (uint32_t)(key >> shift) & (NB - 1);
    s_dig[j] = (uint8_t)d;
    const uint32_t g = s_gbase[d] + j;
    if (g < n) kout[g] = key;
  }
  __syncthreads();
  uint32_t* s_vals = reinterpret_cast<uint32_t*>(s_keys);
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t idx = wbase + i * 64;
    s_vals[pos[i]] = idx < n ? vin[idx] : 0u;
  }
  __syncthreads();
  for (int j = t; j < kSortPart; j += kBlock) {
    const uint32_t g = s_gbase[s_dig[j]] + j;
    if (g < n) vout[g] = s_vals[j];
  }
}

__global__ __launch_bounds__(kBlock) void k_tile_ranges(int64_t capacity,
                                                        const uint32_t* __restrict__ count,
                                                        const uint64_t* __restrict__ keys,
                                                        uint32_t* __restrict__ ranges) {
  const uint32_t n = *count;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const uint32_t tile = (uint32_t)(keys[i] >> 32);
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != tile) ranges[2 * tile] = (uint32_t)i;
    if (i == (int64_t)n - 1 || (uint32_t)(keys[i + 1] >> 32) != tile) ranges[2 * tile + 1] = (uint32_t)(i + 1);
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) p[i] = v;
}

int stream_grid(int64_t items, int cap = 2048) {
  const int64_t b = (items + kBlock - 1) / kBlock;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

SortLayout sort_layout(int64_t capacity, int passes) {
  SortLayout L;
  const int64_t cap = capacity > 0 ? capacity : 1;
  L.parts = (int)((cap + kSortPart - 1) / kSortPart);
  size_t o = 0;
  L.keys_tmp = o; o = align_up(o + (size_t)cap * 8, 256);
  L.vals_tmp = o; o = align_up(o + (size_t)cap * 4, 256);
  L.keys_alt = o; o = align_up(o + (size_t)cap * 8, 256);
  L.vals_alt = o; o = align_up(o + (size_t)cap * 4, 256);
  L.hist = o; o = align_up(o + (size_t)kHistMax * 4, 256);
  L.tickets = o; o = align_up(o + (size_t)kMaxPasses * 4, 256);
  L.lookback = o; o = align_up(o + (size_t)2 * L.parts * 256 * 4, 256);
  L.flags = o; o = align_up(o + 4, 256);
  L.total = o; o = align_up(o + 4, 256);
  (void)passes;
  L.bytes = o;
  return L;
}

hipError_t launch_sort_init(const SortLayout& L, char* ws, int passes, int nbins,
                            uint32_t* tile_ranges, int tiles, uint32_t* status_flag,
                            const uint32_t* total_src, int64_t capacity, hipStream_t st) {
  // total_src == NULL: the count is `capacity` itself (stand-alone sort)
  const int lb_len = L.parts * nbins;
  const int ranges_len = tile_ranges ? 2 * tiles : 0;
  const int grid = stream_grid(lb_len > ranges_len ? lb_len : ranges_len, 512);
  hipLaunchKernelGGL(k_sort_init, dim3(grid), dim3(kBlock), 0, st,
                     reinterpret_cast<uint32_t*>(ws + L.hist), passes * nbins,
                     reinterpret_cast<uint32_t*>(ws + L.tickets), passes,
                     reinterpret_cast<uint32_t*>(ws + L.lookback), lb_len, tile_ranges,
                     ranges_len, reinterpret_cast<uint32_t*>(ws + L.total), total_src,
                     (uint32_t)capacity, capacity, status_flag);
  return hipGetLastError();
}

hipError_t launch_keygen(int n, const gs_splat* splats, const uint32_t* offsets,
                         const uint32_t* total, int64_t capacity, int tiles_x, int bits,
                         int passes, uint64_t* keys, uint32_t* vals, uint32_t* hist,
                         uint32_t* count, hipStream_t st) {
  (void)capacity;
  if (n == 0) return hipSuccess;
  const dim3 grid(stream_grid(n, 4096)), block(kBlock);
  switch (bits) {
    case 6: hipLaunchKernelGGL(k_keygen<6>, grid, block, 0, st, n, splats, offsets, total, count, tiles_x, passes, keys, vals, hist); break;
    case 7: hipLaunchKernelGGL(k_keygen<7>, grid, block, 0, st, n, splats, offsets, total, count, tiles_x, passes, keys, vals, hist); break;
    default: hipLaunchKernelGGL(k_keygen<8>, grid, block, 0, st, n, splats, offsets, total, count, tiles_x, passes, keys, vals, hist); break;
  }
  return hipGetLastError();
}

hipError_t launch_histogram(int64_t n, const uint64_t* keys, int bits, int passes,
                            uint32_t* hist, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 grid(stream_grid(n, 1024)), block(kBlock);
  switch (bits) {
    case 6: hipLaunchKernelGGL(k_histogram<6>, grid, block, 0, st, n, keys, passes, hist); break;
    case 7: hipLaunchKernelGGL(k_histogram<7>, grid, block, 0, st, n, keys, passes, hist); break;
    default: hipLaunchKernelGGL(k_histogram<8>, grid, block, 0, st, n, keys, passes, hist); break;
  }
  return hipGetLastError();
}

hipError_t launch_radix_passes(int64_t capacity, const uint32_t* count, int bits, int passes,
                               uint64_t* keys_a, uint32_t* vals_a, uint64_t* keys_b,
                               uint32_t* vals_b, uint64_t* keys_out, uint32_t* vals_out,
                               const uint32_t* hist, uint32_t* tickets, uint32_t* lookback,
                               hipStream_t st) {
  // keys_a: input; keys_b: scratch; the last pass lands in keys_out.
  const int nb = 1 << bits;
  const int parts = (int)((capacity + kSortPart - 1) / kSortPart);
  if (parts == 0) return hipSuccess;
  const uint64_t* kin = keys_a;
  const uint32_t* vin = vals_a;
  for (int p = 0; p < passes; ++p) {
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    uint64_t* kdst = to_out ? keys_out : keys_b;
    uint32_t* vdst = to_out ? vals_out : vals_b;
    uint32_t* lb = lookback + (size_t)(p & 1) * parts * 256;
    uint32_t* lb_next = lookback + (size_t)((p + 1) & 1) * parts * 256;
    const uint32_t* h = hist + p * nb;
    trace_mark(st, "radix_pass");
    switch (bits) {
      case 6: hipLaunchKernelGGL(k_onesweep<6>, dim3(parts), dim3(kBlock), 0, st, kin, vin, kdst, vdst, count, p * bits, h, tickets + p, lb, lb_next); break;
      case 7: hipLaunchKernelGGL(k_onesweep<7>, dim3(parts), dim3(kBlock), 0, st, kin, vin, kdst, vdst, count, p * bits, h, tickets + p, lb, lb_next); break;
      default: hipLaunchKernelGGL(k_onesweep<8>, dim3(parts), dim3(kBlock), 0, st, kin, vin, kdst, vdst, count, p * bits, h, tickets + p, lb, lb_next); break;
    }
    kin = kdst;
    vin = vdst;
  }
  return hipGetLastError();
}

hipError_t launch_tile_ranges(int64_t capacity, const uint32_t* count, const uint64_t* keys,
                              uint32_t* ranges, hipStream_t st) {
  if (capacity == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_ranges, dim3(stream_grid(capacity, 4096)), dim3(kBlock), 0, st,
                     capacity, count, keys, ranges);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(stream_grid(count, 1024)), dim3(kBlock), 0, st, p, v, count);
  return hipGetLastError();
}

}  // namespace gs
