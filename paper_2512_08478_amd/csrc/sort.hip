// (tile, depth) keys and the per-frame GPU radix sort (Algorithm 1, Radix
// Sort; Section 3.4).
//
// The sort is a stable least-significant-digit radix sort over the key
// tile << 32 | bits(float32 depth).  Its first passes work on the depth
// digits and its last passes on the tile digits.  Every (Gaussian, tile)
// instance of one Gaussian carries the same depth, so the depth passes give
// the same order whether they run before or after a Gaussian is expanded
// into its tiles: they run on the visible Gaussians (u32 depth keys), the
// instances are generated in that depth order (u32 tile keys), and the tile
// passes finish the sort.  The permutation is identical to sorting the
// 64-bit keys of the Gaussian-major instance list, with far fewer bytes.
//
// Each radix pass is onesweep-style: one digit histogram up front, then one
// kernel per digit in which a workgroup
//   1. takes a 4096-key partition by atomic ticket (every partition it waits
//      on has already started),
//   2. ranks the keys of each wave with ballot-based digit matching (one
//      ballot per digit bit; equal digits keep index order: stable),
//   3. publishes its per-digit counts and looks back over earlier
//      partitions, eight status words in flight per digit,
//   4. stages keys in LDS in sorted order and writes them out, so that
//      consecutive threads write consecutive addresses of one digit run.
// Counts are read from device memory, so no host round trip is needed.
#include "gs_device.h"
#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kHistMax = 2048;     // LDS histogram bins (passes x 2^bits)
constexpr int kLbWindow = 8;       // look-back status words in flight per digit

__global__ __launch_bounds__(kBlock) void k_sort_init(uint32_t* hist, int hist_len,
                                                      uint32_t* tickets, int ntickets,
                                                      uint32_t* lookback, int lb_len,
                                                      uint64_t* kg_status, int kg_len,
                                                      uint32_t* ranges, int ranges_len,
                                                      uint32_t* count, const uint32_t* total_src,
                                                      uint32_t host_total, int64_t capacity,
                                                      uint32_t* status_flag) {
  const int stride = gridDim.x * kBlock;
  const int i0 = blockIdx.x * kBlock + threadIdx.x;
  for (int i = i0; i < lb_len; i += stride) lookback[i] = 0;
  for (int i = i0; i < ranges_len; i += stride) ranges[i] = 0;
  for (int i = i0; i < kg_len; i += stride) kg_status[i] = 0;
  for (int i = i0; i < hist_len; i += stride) hist[i] = 0;
  if (i0 < ntickets) tickets[i0] = 0;
  if (i0 == 0) {
    const uint32_t tot = total_src ? *total_src : host_total;
    const bool over = (int64_t)tot > capacity;
    *count = over ? (uint32_t)capacity : tot;
    if (status_flag) *status_flag = over ? 1u : 0u;
  }
}

template <typename KeyT, int BITS>
__device__ __forceinline__ uint32_t digit_of(KeyT k, int shift) {
  return (uint32_t)(k >> shift) & ((1u << BITS) - 1);
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

// Digit histograms of `passes` digits of keys[0, n); global layout is 256
// bins per pass.  n comes from *count when count != NULL.
template <typename KeyT, int BITS>
__global__ __launch_bounds__(kBlock) void k_histogram(const KeyT* __restrict__ keys,
                                                      const uint32_t* __restrict__ count,
                                                      int64_t n_host, int passes,
                                                      uint32_t* __restrict__ hist) {
  constexpr int NB = 1 << BITS;
  __shared__ uint32_t s_hist[kHistMax];
  for (int b = threadIdx.x; b < passes * NB; b += kBlock) s_hist[b] = 0;
  __syncthreads();
  const int64_t n = count ? (int64_t)*count : n_host;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    const KeyT key = valid ? keys[i] : KeyT(0);
    for (int p = 0; p < passes; ++p)
      wave_hist_add<BITS>(s_hist + p * NB, digit_of<KeyT, BITS>(key, p * BITS), valid);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < passes * NB; b += kBlock) {
    const uint32_t v = s_hist[b];
    if (v) atomicAdd(&hist[(b / NB) * 256 + (b % NB)], v);
  }
}

// One radix pass.  kin/vin hold n pairs (n = *count); pairs are scattered to
// kout/vout by the digit at `shift`.  WRITE_KEYS = false skips the key
// stores of a last pass whose keys nobody reads.
template <typename KeyT, int BITS, bool WRITE_KEYS>
__global__ __launch_bounds__(kBlock) void k_onesweep(const KeyT* __restrict__ kin,
                                                     const uint32_t* __restrict__ vin,
                                                     KeyT* __restrict__ kout,
                                                     uint32_t* __restrict__ vout,
                                                     const uint32_t* __restrict__ count,
                                                     int64_t n_host, int shift,
                                                     const uint32_t* __restrict__ hist,
                                                     uint32_t* __restrict__ ticket,
                                                     uint32_t* __restrict__ lb,
                                                     uint32_t* __restrict__ lb_next) {
  constexpr int NB = 1 << BITS;
  constexpr int NW = kBlock / 64;
  __shared__ uint32_t s_whist[NW][NB];
  __shared__ uint32_t s_local[NB];
  __shared__ uint32_t s_gbase[NB];
  __shared__ KeyT s_keys[kSortPart];
  __shared__ uint8_t s_dig[kSortPart];
  __shared__ uint32_t s_scan[2][NW];
  __shared__ uint32_t s_part;

  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  if (t == 0) s_part = atomicAdd(ticket, 1u);
  for (int b = t; b < NW * NB; b += kBlock) (&s_whist[0][0])[b] = 0;
  __syncthreads();
  const uint32_t part = s_part;
  const uint32_t n = count ? *count : (uint32_t)n_host;
  const uint32_t base = part * kSortPart;
  if (base >= n) return;
  for (int b = t; b < NB; b += kBlock) lb_next[part * NB + b] = 0;

  // warp-striped load: wave w owns keys [w*64*ITEMS, (w+1)*64*ITEMS)
  KeyT k[kSortItems];
  uint32_t pos[kSortItems];
  const uint32_t wbase = base + wave * 64 * kSortItems + lane;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t idx = wbase + i * 64;
    k[i] = idx < n ? kin[idx] : ~KeyT(0);  // past the end: last digit, ranked last
  }
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t d = digit_of<KeyT, BITS>(k[i], shift);
    const uint64_t peers = match_digit<BITS>(d, ~0ull);
    const uint32_t c = s_whist[wave][d];
    pos[i] = c + (uint32_t)__builtin_popcountll(peers & lt);
    if ((peers & lt) == 0) s_whist[wave][d] = c + (uint32_t)__builtin_popcountll(peers);
  }
  __syncthreads();

  // per digit: offsets of each wave, partition total, global digit start
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
        uint32_t s[kLbWindow];
#pragma unroll
        for (int w = 0; w < kLbWindow; ++w)
          s[w] = (j - w >= 0) ? ld_agent(&lb[(j - w) * NB + t]) : kLbFlagInc;
        int used = 0;
        bool done = false;
#pragma unroll
        for (int w = 0; w < kLbWindow; ++w) {
          if (done || used < w) continue;  // stop at the first unpublished word
          if ((s[w] & (kLbFlagAgg | kLbFlagInc)) == 0) continue;
          prefix += s[w] & kLbValue;
          used = w + 1;
          if (s[w] & kLbFlagInc) done = true;
        }
        if (done) break;
        j -= used;
      }
      st_agent(&lb[part * NB + t], kLbFlagInc | (prefix + tot));
    }
    s_local[t] = local;
    s_gbase[t] = gstart + prefix - local;
  }
  __syncthreads();

#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t d = digit_of<KeyT, BITS>(k[i], shift);
    pos[i] += s_local[d] + s_whist[wave][d];
    s_keys[pos[i]] = k[i];
  }
  __syncthreads();
  for (int j = t; j < kSortPart; j += kBlock) {
    const KeyT key = s_keys[j];
    const uint32_t d = digit_of<KeyT, BITS>(key, shift);
    s_dig[j] = (uint8_t)d;
    if (WRITE_KEYS) {
      const uint32_t g = s_gbase[d] + j;
      if (g < n) kout[g] = key;
    }
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

// Instances in depth order.  Workgroup `part` (ticket order) takes 256
// Gaussians of the depth-sorted visible list, counts their tiles, gets the
// number of instances before it by decoupled look-back, and writes
// (tile id, Gaussian index) for each tile of each rect in row-major order;
// the expansion is spread over the workgroup with a binary search over the
// local offsets, so a large splat does not serialise one thread.
__global__ __launch_bounds__(kBlock) void k_keygen(const uint32_t* __restrict__ sorted_idx,
                                                   const uint32_t* __restrict__ vis_count,
                                                   const gs_splat* __restrict__ splats, int tiles_x,
                                                   const uint32_t* __restrict__ inst_count,
                                                   uint32_t* __restrict__ tkeys,
                                                   uint32_t* __restrict__ tvals,
                                                   uint64_t* __restrict__ status,
                                                   uint32_t* __restrict__ ticket) {
  __shared__ uint32_t s_part, s_prefix;
  __shared__ uint32_t s_off[kBlock + 1];
  __shared__ uint32_t s_lo[kBlock], s_hi[kBlock], s_g[kBlock];
  __shared__ uint32_t s_wave[kBlock / 64];
  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  if (t == 0) s_part = atomicAdd(ticket, 1u);
  __syncthreads();
  const uint32_t part = s_part, nvis = *vis_count, cap = *inst_count;
  const uint32_t base = part * kBlock;
  if (base >= nvis) return;
  const uint32_t j = base + t;
  uint32_t cnt = 0, g = 0, lo = 0, hi = 0;
  if (j < nvis) {
    g = sorted_idx[j];
    const float4 r2 = reinterpret_cast<const float4*>(splats + g)[2];
    lo = __float_as_uint(r2.z);
    hi = __float_as_uint(r2.w);
    cnt = ((hi & 0xFFFFu) - (lo & 0xFFFFu) + 1) * ((hi >> 16) - (lo >> 16) + 1);
  }
  s_g[t] = g;
  s_lo[t] = lo;
  s_hi[t] = hi;
  const uint32_t incl = wave_incl_scan(cnt);
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  uint32_t woff = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    woff += w < wave ? s_wave[w] : 0u;
    btot += s_wave[w];
  }
  s_off[t] = woff + incl - cnt;
  if (t == kBlock - 1) s_off[kBlock] = btot;
  if (wave == 0) {
    const uint32_t pre = wave_lookback(status, (int)part, btot);
    if (lane == 0) s_prefix = pre;
  }
  __syncthreads();
  const uint32_t prefix = s_prefix;
  for (uint32_t kk = 0; kk < btot; kk += kBlock) {
    const uint32_t k = kk + t;
    if (k < btot) {
      int a = 0, b = kBlock - 1;
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (s_off[mid] <= k) a = mid; else b = mid - 1;
      }
      const uint32_t local = k - s_off[a];
      const uint32_t rl = s_lo[a], rh = s_hi[a];
      const uint32_t tx0 = rl & 0xFFFFu, ty0 = rl >> 16, tx1 = rh & 0xFFFFu;
      const uint32_t w = tx1 - tx0 + 1;
      const uint32_t ry = local / w;
      const uint32_t gp = prefix + k;
      if (gp < cap) {
        tkeys[gp] = (ty0 + ry) * (uint32_t)tiles_x + tx0 + (local - ry * w);
        tvals[gp] = s_g[a];
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_tile_ranges(const uint32_t* __restrict__ count,
                                                        const uint32_t* __restrict__ tkeys,
                                                        uint32_t* __restrict__ ranges) {
  const uint32_t n = *count;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const uint32_t tile = tkeys[i];
    if (i == 0 || tkeys[i - 1] != tile) ranges[2 * tile] = (uint32_t)i;
    if (i == (int64_t)n - 1 || tkeys[i + 1] != tile) ranges[2 * tile + 1] = (uint32_t)(i + 1);
  }
}

// Optional 64-bit keys of the sorted list: tile << 32 | bits(float32 depth).
__global__ __launch_bounds__(kBlock) void k_compose_keys(const uint32_t* __restrict__ count,
                                                         const uint32_t* __restrict__ tkeys,
                                                         const uint32_t* __restrict__ values,
                                                         const gs_splat* __restrict__ splats,
                                                         uint64_t* __restrict__ keys) {
  const uint32_t n = *count;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const uint32_t d = __float_as_uint(splats[values[i]].depth);
    keys[i] = ((uint64_t)tkeys[i] << 32) | d;
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

template <typename KeyT, int BITS>
void histogram_t(const KeyT* keys, const uint32_t* count, int64_t n_grid, int passes,
                 uint32_t* hist, hipStream_t st) {
  hipLaunchKernelGGL((k_histogram<KeyT, BITS>), dim3(stream_grid(n_grid, 256)), dim3(kBlock), 0,
                     st, keys, count, n_grid, passes, hist);
}

template <typename KeyT, int BITS>
void onesweep_t(bool write_keys, int parts, const KeyT* kin, const uint32_t* vin, KeyT* kout,
                uint32_t* vout, const uint32_t* count, int64_t n_host, int shift,
                const uint32_t* hist, uint32_t* ticket, uint32_t* lb, uint32_t* lb_next,
                hipStream_t st) {
  if (write_keys)
    hipLaunchKernelGGL((k_onesweep<KeyT, BITS, true>), dim3(parts), dim3(kBlock), 0, st, kin, vin,
                       kout, vout, count, n_host, shift, hist, ticket, lb, lb_next);
  else
    hipLaunchKernelGGL((k_onesweep<KeyT, BITS, false>), dim3(parts), dim3(kBlock), 0, st, kin,
                       vin, kout, vout, count, n_host, shift, hist, ticket, lb, lb_next);
}

}  // namespace

SortLayout sort_layout(int64_t n, int64_t capacity) {
  SortLayout L;
  const int64_t nn = n > 0 ? n : 1, cap = capacity > 0 ? capacity : 1;
  const int64_t big = nn > cap ? nn : cap;
  L.parts = (int)((big + kSortPart - 1) / kSortPart);
  L.kg_parts = (int)((nn + kBlock - 1) / kBlock);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.dk[0] = take((size_t)nn * 4); L.dv[0] = take((size_t)nn * 4);
  L.dk[1] = take((size_t)nn * 4); L.dv[1] = take((size_t)nn * 4);
  L.tk[0] = take((size_t)cap * 4); L.tv[0] = take((size_t)cap * 4);
  L.tk[1] = take((size_t)cap * 4); L.tv[1] = take((size_t)cap * 4);
  L.tkf = take((size_t)cap * 4);
  L.hist = take((size_t)kMaxPassTotal * 256 * 4);
  L.tickets = take((size_t)kMaxPassTotal * 4);
  L.lookback = take((size_t)2 * L.parts * 256 * 4);
  L.kg_status = take((size_t)L.kg_parts * 8);
  L.count = take(4);
  L.bytes = o;
  return L;
}

SortLayout pairs_layout(int64_t n) {
  SortLayout L;
  const int64_t nn = n > 0 ? n : 1;
  L.parts = (int)((nn + kSortPart - 1) / kSortPart);
  L.kg_parts = 0;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.dk[0] = take((size_t)nn * 8);  // alternate key buffer (u64)
  L.dv[0] = take((size_t)nn * 4);  // alternate value buffer
  L.dk[1] = L.dv[1] = L.tk[0] = L.tv[0] = L.tk[1] = L.tv[1] = L.tkf = 0;
  L.hist = take((size_t)kMaxPassTotal * 256 * 4);
  L.tickets = take((size_t)kMaxPassTotal * 4);
  L.lookback = take((size_t)2 * L.parts * 256 * 4);
  L.kg_status = 0;
  L.count = take(4);
  L.bytes = o;
  return L;
}

hipError_t launch_sort_init(const SortLayout& L, char* ws, uint32_t* tile_ranges, int tiles,
                            uint32_t* status_flag, const uint32_t* total_src, int64_t capacity,
                            hipStream_t st) {
  const int lb_len = 2 * L.parts * 256;
  const int ranges_len = tile_ranges ? 2 * tiles : 0;
  int64_t most = lb_len > ranges_len ? lb_len : ranges_len;
  if (L.kg_parts > most) most = L.kg_parts;
  hipLaunchKernelGGL(k_sort_init, dim3(stream_grid(most, 1024)), dim3(kBlock), 0, st,
                     reinterpret_cast<uint32_t*>(ws + L.hist), kMaxPassTotal * 256,
                     reinterpret_cast<uint32_t*>(ws + L.tickets), kMaxPassTotal,
                     reinterpret_cast<uint32_t*>(ws + L.lookback), lb_len,
                     reinterpret_cast<uint64_t*>(ws + L.kg_status), L.kg_parts, tile_ranges,
                     ranges_len, reinterpret_cast<uint32_t*>(ws + L.count), total_src,
                     (uint32_t)capacity, capacity, status_flag);
  return hipGetLastError();
}

template <typename KeyT>
hipError_t launch_histogram(const KeyT* keys, const uint32_t* count, int64_t n_grid, int bits,
                            int passes, uint32_t* hist, hipStream_t st) {
  if (n_grid == 0 || passes == 0) return hipSuccess;
  switch (bits) {
    case 6: histogram_t<KeyT, 6>(keys, count, n_grid, passes, hist, st); break;
    case 7: histogram_t<KeyT, 7>(keys, count, n_grid, passes, hist, st); break;
    default: histogram_t<KeyT, 8>(keys, count, n_grid, passes, hist, st); break;
  }
  return hipGetLastError();
}
template hipError_t launch_histogram<uint32_t>(const uint32_t*, const uint32_t*, int64_t, int, int,
                                               uint32_t*, hipStream_t);
template hipError_t launch_histogram<uint64_t>(const uint64_t*, const uint32_t*, int64_t, int, int,
                                               uint32_t*, hipStream_t);

template <typename KeyT>
hipError_t launch_radix_passes(int64_t n_grid, const uint32_t* count, int bits, int passes,
                               int pass_base, const KeyT* kin, const uint32_t* vin, KeyT* k_alt,
                               uint32_t* v_alt, KeyT* k_out, uint32_t* v_out, bool last_keys,
                               uint32_t* hist, uint32_t* tickets, uint32_t* lookback, int lb_parts,
                               const char* label, hipStream_t st) {
  const int parts = (int)((n_grid + kSortPart - 1) / kSortPart);
  if (parts == 0 || passes == 0) return hipSuccess;
  const KeyT* ki = kin;
  const uint32_t* vi = vin;
  for (int p = 0; p < passes; ++p) {
    const int q = pass_base + p;  // global pass index: look-back buffer parity and ticket
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    KeyT* kd = to_out ? k_out : k_alt;
    uint32_t* vd = to_out ? v_out : v_alt;
    uint32_t* lb = lookback + (size_t)(q & 1) * lb_parts * 256;
    uint32_t* lb_next = lookback + (size_t)((q + 1) & 1) * lb_parts * 256;
    const bool wk = (p + 1 < passes) || last_keys;
    trace_mark(st, label);
    switch (bits) {
      case 6: onesweep_t<KeyT, 6>(wk, parts, ki, vi, kd, vd, count, n_grid, p * bits, hist + p * 256, tickets + q, lb, lb_next, st); break;
      case 7: onesweep_t<KeyT, 7>(wk, parts, ki, vi, kd, vd, count, n_grid, p * bits, hist + p * 256, tickets + q, lb, lb_next, st); break;
      default: onesweep_t<KeyT, 8>(wk, parts, ki, vi, kd, vd, count, n_grid, p * bits, hist + p * 256, tickets + q, lb, lb_next, st); break;
    }
    ki = kd;
    vi = vd;
  }
  return hipGetLastError();
}
template hipError_t launch_radix_passes<uint32_t>(int64_t, const uint32_t*, int, int, int,
                                                  const uint32_t*, const uint32_t*, uint32_t*,
                                                  uint32_t*, uint32_t*, uint32_t*, bool, uint32_t*,
                                                  uint32_t*, uint32_t*, int, const char*,
                                                  hipStream_t);
template hipError_t launch_radix_passes<uint64_t>(int64_t, const uint32_t*, int, int, int,
                                                  const uint64_t*, const uint32_t*, uint64_t*,
                                                  uint32_t*, uint64_t*, uint32_t*, bool, uint32_t*,
                                                  uint32_t*, uint32_t*, int, const char*,
                                                  hipStream_t);

hipError_t launch_keygen(int64_t n, const uint32_t* sorted_idx, const uint32_t* vis_count,
                         const gs_splat* splats, int tiles_x, const uint32_t* inst_count,
                         uint32_t* tkeys, uint32_t* tvals, uint64_t* status, uint32_t* ticket,
                         hipStream_t st) {
  const int parts = (int)((n + kBlock - 1) / kBlock);
  if (parts == 0) return hipSuccess;
  hipLaunchKernelGGL(k_keygen, dim3(parts), dim3(kBlock), 0, st, sorted_idx, vis_count, splats,
                     tiles_x, inst_count, tkeys, tvals, status, ticket);
  return hipGetLastError();
}

hipError_t launch_tile_ranges(int64_t capacity, const uint32_t* count, const uint32_t* tkeys,
                              uint32_t* ranges, hipStream_t st) {
  if (capacity == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_ranges, dim3(stream_grid(capacity, 4096)), dim3(kBlock), 0, st, count,
                     tkeys, ranges);
  return hipGetLastError();
}

hipError_t launch_compose_keys(int64_t capacity, const uint32_t* count, const uint32_t* tkeys,
                               const uint32_t* values, const gs_splat* splats, uint64_t* keys,
                               hipStream_t st) {
  if (capacity == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compose_keys, dim3(stream_grid(capacity, 4096)), dim3(kBlock), 0, st,
                     count, tkeys, values, splats, keys);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(stream_grid(count, 1024)), dim3(kBlock), 0, st, p, v, count);
  return hipGetLastError();
}

}  // namespace gs
