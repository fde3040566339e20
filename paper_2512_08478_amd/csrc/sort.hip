// (tile, depth) keys and the per-frame GPU radix sort (Algorithm 1, Radix
// Sort; Section 3.4).
//
// The sort is a stable least-significant-digit radix sort over the key
// tile << 32 | bits(float32 depth).  Its first passes work on the depth
// digits and its last passes on the tile digits.  Every (Gaussian, tile)
// instance of one Gaussian carries the same depth, so the depth passes give
// the same order whether they run before or after a Gaussian is expanded
// into its tiles: they run on the Gaussians (u32 depth keys; culled ones
// carry the largest key and sort last), the instances are generated in that
// depth order (u32 tile keys), and the tile passes finish the sort.  The
// permutation is identical to sorting the 64-bit keys of the Gaussian-major
// instance list, with far fewer bytes moved.
//
// A radix pass ranks the keys of each 4096-key partition in LDS: every wave
// ranks 64 keys at a time by ballot-based digit matching (one ballot per
// digit bit; equal digits keep index order, so the sort is stable), waves
// are stacked by per-wave digit counts, and the keys are staged in LDS in
// sorted order so that consecutive threads write consecutive addresses of
// one digit run.  The partition's global offsets per digit come from one of
// two schemes (gs_settings.sort_mode):
//   0  reduce-then-scan: an upsweep kernel writes every partition's digit
//      counts, a scan kernel turns them into per-partition offsets, and the
//      downsweep scatters.  No workgroup waits on another.
//   1  onesweep: one histogram up front, then a single kernel per digit that
//      publishes its counts and looks back over earlier partitions (eight
//      status words in flight per digit) with agent-scope atomics.  On an
//      8-XCD part every look-back round trip leaves the XCD's L2, so the
//      inclusive-prefix frontier advances one window per round trip.
// Counts are read from device memory, so no host round trip is needed.
#include "gs_device.h"
#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kHistMax = 2048;     // LDS histogram bins (passes x 2^bits)
constexpr int kMaxDigits = 512;    // digits of the widest (9-bit) pass
constexpr int kLbWindow = 8;       // look-back status words in flight per digit
constexpr int kKgItems = 4;        // sorted Gaussians per thread in the keygen
constexpr int kKgPart = kBlock * kKgItems;
constexpr int kRsMinParts = 384;   // reduce-then-scan passes aim for at least this many partitions

// Thread i0 of `stride` threads takes its share of the set-up.
__device__ __forceinline__ void sort_init_body(const SortInitK& I, int i0, int stride) {
  if (I.cls_count && i0 < kTileClasses) I.cls_count[i0] = 0;
  for (int i = i0; i < I.ranges_len; i += stride) I.ranges[i] = 0;
  if (i0 < I.ntickets) I.tickets[i0] = 0;
  if (i0 == 0) {
    const uint32_t tot = I.total_src ? *I.total_src : I.host_total;
    const bool over = (int64_t)tot > I.capacity;
    *I.count = over ? (uint32_t)I.capacity : tot;
    // total_src = counts: counts[1] visible, counts[2..3] their depth key range
    bool range_over = false;
    if (I.total_src && I.depth_bits > 0 && I.depth_bits < 32 && I.total_src[1] > 0)
      range_over = ((I.total_src[3] - I.total_src[2]) >> I.depth_bits) != 0u;
    if (I.status_flag) *I.status_flag = (over ? 1u : 0u) | (range_over ? 2u : 0u);
  }
}

__global__ __launch_bounds__(kBlock) void k_sort_init(SortInitK I, uint32_t* hist, int hist_len,
                                                      uint32_t* lookback, int lb_len) {
  const int stride = gridDim.x * kBlock;
  const int i0 = blockIdx.x * kBlock + threadIdx.x;
  for (int i = i0; i < lb_len; i += stride) lookback[i] = 0;
  for (int i = i0; i < hist_len; i += stride) hist[i] = 0;
  sort_init_body(I, i0, stride);
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

__device__ __forceinline__ uint32_t read_n(const uint32_t* count, int64_t n_host) {
  return count ? *count : (uint32_t)n_host;
}

// Block-wide exclusive scan of one u32 per thread (NT threads; s_tmp holds
// NT / 64 words).
template <int NT = kBlock>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(v);
  if (lane == 63) s_tmp[wave] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    off += w < wave ? s_tmp[w] : 0u;
    tot += s_tmp[w];
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

// ---------------------------------------------------------------- counting

// A key is sorted if it lies before the end and, in a dropping pass, is
// not the all-ones key (the depth key of a culled Gaussian).
template <typename KeyT>
__device__ __forceinline__ bool key_kept(KeyT k, uint32_t idx, uint32_t n, int drop) {
  return idx < n && !(drop && k == ~KeyT(0));
}

// Digit counts of one partition (kBlock * ITEMS keys) per workgroup,
// written partition-major into table[partition * NB + d], so one
// workgroup's counts are one contiguous row.  Counting needs no order.
// LDS atomics that hit one address in one instruction serialise, and the
// top digits of depth and tile keys cluster (a dense tile's instances
// share theirs), so each instruction first peels off the digits of its
// first two remaining lanes with a ballot each (one atomic adds the whole
// group), and the rest add one per lane into the sub-histogram of their
// 16-lane group (rows padded by one word, so the groups' copies of a digit
// sit in different banks).
template <typename KeyT, int BITS, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_rs_upsweep(const KeyT* __restrict__ kin,
                                                       const uint32_t* __restrict__ count,
                                                       int64_t n_host, int drop,
                                                       const uint32_t* __restrict__ kbase,
                                                       int shift, uint32_t* __restrict__ table,
                                                       SortInitK init) {
  constexpr int NB = 1 << BITS;
  constexpr int NS = kBlock / 16;  // sub-histograms
  constexpr int PART = kBlock * ITEMS;
  __shared__ uint32_t s_h[NS][NB + 1];
  const int t = threadIdx.x, lane = lane_id();
  if (init.active) sort_init_body(init, blockIdx.x * kBlock + t, gridDim.x * kBlock);
  const uint32_t n = read_n(count, n_host);
  const uint32_t base = blockIdx.x * PART;
  if (base >= n) return;
  for (int d = t; d < NS * (NB + 1); d += kBlock) (&s_h[0][0])[d] = 0;
  KeyT k[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t idx = base + i * kBlock + t;
    k[i] = idx < n ? kin[idx] : KeyT(0);
  }
  const KeyT kb = kbase ? (KeyT)*kbase : KeyT(0);
  __syncthreads();
  uint32_t* h = s_h[t >> 4];
  uint32_t* h0 = s_h[(t >> 6) * 4];  // the wave's first sub-histogram
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t d = digit_of<KeyT, BITS>(k[i] - kb, shift);
    uint64_t left = ballot(key_kept(k[i], base + i * kBlock + t, n, drop));
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (left) {
        const int first = __builtin_ctzll(left);
        const uint32_t dl = (uint32_t)__builtin_amdgcn_readlane((int)d, first);
        const uint64_t same = ballot(d == dl) & left;
        if (lane == first) atomicAdd(&h0[dl], (uint32_t)__builtin_popcountll(same));
        left &= ~same;
      }
    }
    if ((left >> lane) & 1ull) atomicAdd(&h[d], 1u);
  }
  __syncthreads();
  for (int d = t; d < NB; d += kBlock) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < NS; ++w) c += s_h[w][d];
    table[(size_t)blockIdx.x * NB + d] = c;
  }
}

// Exclusive scan of each row of a rows x P table in place (one workgroup
// per row); the row sums go to totals[row].
__global__ __launch_bounds__(kBlock) void k_row_scan(uint32_t* __restrict__ table, int P,
                                                     uint32_t* __restrict__ totals) {
  __shared__ uint32_t s_tmp[kBlock / 64];
  constexpr int IT = 16;
  uint32_t* row = table + (size_t)blockIdx.x * P;
  const int t = threadIdx.x;
  uint32_t carry = 0;
  for (int base = 0; base < P; base += kBlock * IT) {
    uint32_t v[IT];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const int idx = base + t * IT + j;
      v[j] = idx < P ? row[idx] : 0u;
      s += v[j];
    }
    uint32_t tot;
    uint32_t run = carry + block_excl_scan(s, s_tmp, &tot);
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const int idx = base + t * IT + j;
      if (idx < P) row[idx] = run;
      run += v[j];
    }
    carry += tot;
  }
  if (t == 0) totals[blockIdx.x] = carry;
}

// Per-digit exclusive prefix over the partitions of the partition-major
// count table (table[p * NB + d], p < the partitions that hold keys), in
// place; the digit sums go to totals[d].  Workgroup w owns the 4 digits
// [4w, 4w + 4): each thread reads the 16-byte slices of 16 consecutive
// rows per round, and the 4 digit columns are scanned side by side with
// DPP wave scans.
template <int NB, int PART>
__global__ __launch_bounds__(kBlock) void k_col_scan(uint32_t* __restrict__ table,
                                                     const uint32_t* __restrict__ count,
                                                     int64_t n_host,
                                                     uint32_t* __restrict__ totals) {
  constexpr int DG = 4, RPT = 16, NW = kBlock / 64;
  __shared__ uint32_t s_w[DG][NW];
  const uint32_t n = read_n(count, n_host);
  const int P = (int)((n + PART - 1) / PART);
  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  const int d0 = blockIdx.x * DG;
  uint32_t carry[DG];
#pragma unroll
  for (int k = 0; k < DG; ++k) carry[k] = 0;
  for (int r0 = 0; r0 < P; r0 += kBlock * RPT) {
    uint4 c[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = r0 + t * RPT + i;
      c[i] = row < P ? *reinterpret_cast<const uint4*>(table + (size_t)row * NB + d0)
                     : make_uint4(0u, 0u, 0u, 0u);
    }
    uint32_t s[DG] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      s[0] += c[i].x;
      s[1] += c[i].y;
      s[2] += c[i].z;
      s[3] += c[i].w;
    }
    uint32_t ex[DG];
#pragma unroll
    for (int k = 0; k < DG; ++k) {
      const uint32_t incl = wave_incl_scan_dpp(s[k]);
      if (lane == 63) s_w[k][wave] = incl;
      ex[k] = incl - s[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < DG; ++k) {
      uint32_t off = 0, tot = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint32_t x = s_w[k][w];
        off += w < wave ? x : 0u;
        tot += x;
      }
      ex[k] += off + carry[k];
      carry[k] += tot;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = r0 + t * RPT + i;
      if (row < P)
        *reinterpret_cast<uint4*>(table + (size_t)row * NB + d0) =
            make_uint4(ex[0], ex[1], ex[2], ex[3]);
      ex[0] += c[i].x;
      ex[1] += c[i].y;
      ex[2] += c[i].z;
      ex[3] += c[i].w;
    }
  }
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < DG; ++k) totals[d0 + k] = carry[k];
  }
}

// Digit histograms of `passes` digits of keys[0, n) for the onesweep mode
// (kept keys only); global layout is 256 bins per pass.
template <typename KeyT, int BITS>
__global__ __launch_bounds__(kBlock) void k_histogram(const KeyT* __restrict__ keys,
                                                      const uint32_t* __restrict__ count,
                                                      int64_t n_host, int drop,
                                                      const uint32_t* __restrict__ kbase,
                                                      int passes, uint32_t* __restrict__ hist) {
  constexpr int NB = 1 << BITS;
  __shared__ uint32_t s_hist[kHistMax];
  const int t = threadIdx.x;
  for (int b = t; b < passes * NB; b += kBlock) s_hist[b] = 0;
  __syncthreads();
  const uint32_t n = read_n(count, n_host);
  const KeyT kb = kbase ? (KeyT)*kbase : KeyT(0);
  for (uint32_t base = blockIdx.x * kSortPart; base < n; base += gridDim.x * kSortPart) {
    KeyT k[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const uint32_t idx = base + i * kBlock + t;
      k[i] = idx < n ? keys[idx] : KeyT(0);
    }
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const bool valid = key_kept(k[i], base + i * kBlock + t, n, drop);
      for (int p = 0; p < passes; ++p)
        wave_hist_add<BITS>(s_hist + p * NB, digit_of<KeyT, BITS>(k[i] - kb, p * BITS), valid);
    }
  }
  __syncthreads();
  for (int b = t; b < passes * NB; b += kBlock) {
    const uint32_t v = s_hist[b];
    if (v) atomicAdd(&hist[(b / NB) * 256 + (b % NB)], v);
  }
}

// ---------------------------------------------------------------- scatter

// Partition of workgroup b (b < P) in the reduce-then-scan downsweep.  The
// hardware deals workgroups to the 8 XCDs in turn (b % 8); XCD x is given
// the contiguous partitions [x q + min(x, r), ...) of P = 8 q + r, so the
// runs that neighbouring partitions write for one digit meet in one XCD's
// L2 instead of being split between two.
__device__ __forceinline__ uint32_t xcd_part(uint32_t b, uint32_t P) {
  const uint32_t q = P >> 3, r = P & 7u, x = b & 7u;
  return x * q + min(x, r) + (b >> 3);
}

// One radix pass.  kin/vin hold n pairs (vin == NULL: value = position);
// the kept pairs (drop != 0 drops the all-ones key) are scattered to
// kout/vout by the digit at `shift`.
// LOOKBACK = false: partitions dealt by xcd_part, offsets from the scanned
//   partition-major table (table[part * NB + d]) and the per-digit totals.
// LOOKBACK = true: partition by ticket, `totals` is this pass's global digit
//   histogram, offsets by decoupled look-back over lb.
// WRITE_KEYS = false skips the key stores of a last pass whose keys nobody
//   reads.
template <typename KeyT, int BITS, int ITEMS, bool WRITE_KEYS, bool LOOKBACK>
__global__ __launch_bounds__(kBlock) void k_radix_pass(
    const KeyT* __restrict__ kin, const uint32_t* __restrict__ vin, KeyT* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ count, int64_t n_host, int drop,
    const uint32_t* __restrict__ kbase, int shift, const uint32_t* __restrict__ table,
    const uint32_t* __restrict__ totals,
    uint32_t* __restrict__ ticket, uint32_t* __restrict__ lb, uint32_t* __restrict__ lb_next) {
  constexpr int NB = 1 << BITS;
  constexpr int NW = kBlock / 64;
  constexpr int PART = kBlock * ITEMS;
  __shared__ uint32_t s_whist[NW][NB];
  __shared__ uint32_t s_local[NB];
  __shared__ uint32_t s_gbase[NB];
  __shared__ KeyT s_keys[PART];
  __shared__ uint32_t s_vals[PART];
  __shared__ uint32_t s_scan[2][NW];
  __shared__ uint32_t s_part;

  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  const uint32_t n = read_n(count, n_host);
  uint32_t part;
  if (LOOKBACK) {
    if (t == 0) s_part = atomicAdd(ticket, 1u);
    for (int b = t; b < NW * NB; b += kBlock) (&s_whist[0][0])[b] = 0;
    __syncthreads();
    part = s_part;
    // the next pass's look-back words of every partition of the grid are
    // cleared, also by partitions that hold no keys in this pass: a later
    // pass may hold keys there (the depth passes after the first sort
    // fewer keys than it, the tile passes more)
    for (int b = t; b < NB; b += kBlock) lb_next[part * NB + b] = 0;
    if (part * PART >= n) return;
  } else {
    const uint32_t P = (n + PART - 1) / PART;
    if (blockIdx.x >= P) return;
    part = xcd_part(blockIdx.x, P);
    for (int b = t; b < NW * NB; b += kBlock) (&s_whist[0][0])[b] = 0;
  }
  const uint32_t base = part * PART;
  // this thread's digits' global totals and (reduce-then-scan) partition
  // prefixes, loaded now so that they arrive during the ranking
  constexpr int DPT = NB > kBlock ? NB / kBlock : 1;
  uint32_t pf_tot[DPT], pf_tab[DPT];
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const int d = t * DPT + k;
    pf_tot[k] = d < NB ? totals[d] : 0u;
    pf_tab[k] = (!LOOKBACK && d < NB) ? table[(size_t)part * NB + d] : 0u;
  }

  // warp-striped load: wave w owns keys [w*64*ITEMS, (w+1)*64*ITEMS); the
  // values are loaded with the keys so both round trips overlap
  KeyT k[ITEMS];
  uint32_t v[ITEMS], pos[ITEMS];
  const uint32_t wbase = base + wave * 64 * ITEMS + lane;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t idx = wbase + i * 64;
    k[i] = idx < n ? kin[idx] : ~KeyT(0);
  }
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t idx = wbase + i * 64;
    v[i] = idx < n ? (vin ? vin[idx] : idx) : 0u;
  }
  if (!LOOKBACK) __syncthreads();  // s_whist zeroed
  // rank within the wave: kept keys in index order, equal digits by lane;
  // keys are taken relative to *kbase (the pass writes them so)
  const KeyT kb = kbase ? (KeyT)*kbase : KeyT(0);
  const uint64_t lt = lanemask_lt();
  uint32_t kept = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const bool keep = key_kept(k[i], wbase + i * 64, n, drop);
    k[i] -= kb;
    kept |= (uint32_t)keep << i;
    const uint32_t d = digit_of<KeyT, BITS>(k[i], shift);
    const uint64_t peers = match_digit<BITS>(d, ballot(keep));
    const uint32_t c = s_whist[wave][d];
    pos[i] = c + (uint32_t)__builtin_popcountll(peers & lt);
    if (keep && (peers & lt) == 0) s_whist[wave][d] = c + (uint32_t)__builtin_popcountll(peers);
  }
  __syncthreads();

  // per digit: offsets of each wave, partition total, global digit start
  // (DPT consecutive digits per thread when there are more digits than
  // threads)
  static_assert(!LOOKBACK || NB <= kBlock, "look-back passes take at most 8-bit digits");
  uint32_t tot[DPT], gcount[DPT], tsum = 0, gsum = 0;
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const int d = t * DPT + k;
    tot[k] = 0;
    gcount[k] = 0;
    if (d < NB) {
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint32_t x = s_whist[w][d];
        s_whist[w][d] = run;
        run += x;
      }
      tot[k] = run;
      gcount[k] = pf_tot[k];
      if (LOOKBACK) st_agent(&lb[part * NB + d], (part == 0 ? kLbFlagInc : kLbFlagAgg) | run);
    }
    tsum += tot[k];
    gsum += gcount[k];
  }
  const uint32_t inc_tot = wave_incl_scan(tsum);
  const uint32_t inc_g = wave_incl_scan(gsum);
  if (lane == 63) {
    s_scan[0][wave] = inc_tot;
    s_scan[1][wave] = inc_g;
  }
  __syncthreads();
  {
    uint32_t off_tot = 0, off_g = 0;
    for (int w = 0; w < wave; ++w) {
      off_tot += s_scan[0][w];
      off_g += s_scan[1][w];
    }
    uint32_t local = off_tot + inc_tot - tsum;
    uint32_t gstart = off_g + inc_g - gsum;
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      const int d = t * DPT + k;
      if (d < NB) {
        uint32_t prefix = 0;
        if (!LOOKBACK) {
          prefix = pf_tab[k];
        } else if (part > 0) {
          int j = (int)part - 1;
          while (true) {
            uint32_t sw[kLbWindow];
#pragma unroll
            for (int w = 0; w < kLbWindow; ++w)
              sw[w] = (j - w >= 0) ? ld_agent(&lb[(j - w) * NB + d]) : kLbFlagInc;
            int used = 0;
            bool done = false;
#pragma unroll
            for (int w = 0; w < kLbWindow; ++w) {
              if (done || used < w) continue;  // stop at the first unpublished word
              if ((sw[w] & (kLbFlagAgg | kLbFlagInc)) == 0) continue;
              prefix += sw[w] & kLbValue;
              used = w + 1;
              if (sw[w] & kLbFlagInc) done = true;
            }
            if (done) break;
            j -= used;
          }
          st_agent(&lb[part * NB + d], kLbFlagInc | (prefix + tot[k]));
        }
        s_local[d] = local;
        s_gbase[d] = gstart + prefix - local;
      }
      local += tot[k];
      gstart += gcount[k];
    }
  }
  uint32_t nkept = 0;  // kept keys of the partition
#pragma unroll
  for (int w = 0; w < NW; ++w) nkept += s_scan[0][w];
  __syncthreads();

  // stage the pairs in digit order, then write them out so that
  // consecutive threads store consecutive addresses of one digit run
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (kept >> i & 1u) {
      const uint32_t d = digit_of<KeyT, BITS>(k[i], shift);
      const uint32_t p = pos[i] + s_local[d] + s_whist[wave][d];
      s_keys[p] = k[i];
      s_vals[p] = v[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t j = (uint32_t)(i * kBlock + t);
    if (j < nkept) {
      const KeyT key = s_keys[j];
      const uint32_t g = s_gbase[digit_of<KeyT, BITS>(key, shift)] + j;
      if (g < n) {  // always true for consistent counts; never stores outside
        if (WRITE_KEYS) kout[g] = key;
        vout[g] = s_vals[j];
      }
    }
  }
}

// ---------------------------------------------------------------- keygen

__device__ __forceinline__ uint32_t rect_tiles(uint32_t lo, uint32_t hi) {
  return ((hi & 0xFFFFu) - (lo & 0xFFFFu) + 1) * ((hi >> 16) - (lo >> 16) + 1);
}

// Tiles touched by each 1024-Gaussian slice of the depth-sorted visible
// list.  The kernel also gathers the slice's tile rects into depth order
// (rects[sorted_idx[p]] -> sorted_rects[p]) for k_kg_write: a light kernel
// with four independent gathers per thread keeps many random reads in
// flight.
__global__ __launch_bounds__(kBlock) void k_kg_count(uint32_t n, const uint32_t* __restrict__ vis_count,
                                                     const uint32_t* __restrict__ sorted_idx,
                                                     const uint2* __restrict__ rects,
                                                     uint2* __restrict__ sorted_rects,
                                                     uint32_t* __restrict__ kg_counts) {
  __shared__ uint32_t s_tmp[kBlock / 64];
  const uint32_t nvis = *vis_count;
  const uint32_t base = blockIdx.x * kKgPart;
  if (base >= nvis) {
    if (threadIdx.x == 0) kg_counts[blockIdx.x] = 0;
    return;
  }
  // branch-free loads (positions past the end read the last Gaussian and
  // are ignored), so that all four gathers are in flight together
  uint32_t g[kKgItems];
  uint2 r[kKgItems];
#pragma unroll
  for (int j = 0; j < kKgItems; ++j)
    g[j] = sorted_idx[min(base + j * kBlock + threadIdx.x, nvis - 1)];
#pragma unroll
  for (int j = 0; j < kKgItems; ++j) r[j] = rects[min(g[j], n - 1)];  // (indices are < n)
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kKgItems; ++j) {
    const uint32_t p = base + j * kBlock + threadIdx.x;
    if (p < nvis) {
      sorted_rects[p] = r[j];
      sum += rect_tiles(r[j].x, r[j].y);
    }
  }
  uint32_t tot;
  block_excl_scan(sum, s_tmp, &tot);
  if (threadIdx.x == 0) kg_counts[blockIdx.x] = tot;
}

// Block-wide exclusive max-scan of one u32 per thread (NT threads): the
// largest value held by any lower thread, 0 for thread 0.
template <int NT = kBlock>
__device__ __forceinline__ uint32_t block_excl_max(uint32_t v, uint32_t* s_tmp) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_max_dpp(v);
  uint32_t excl = wave_shr1(incl);
  if (lane == 63) s_tmp[wave] = incl;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < NT / 64; ++w)
    if (w < wave) excl = max(excl, s_tmp[w]);
  __syncthreads();
  return excl;
}

constexpr int kKgWin = 2048;              // instances expanded per window
constexpr int kKgWinItems = kKgWin / kBlock;
// The fused keygen scatter: threads per workgroup and instances per window.
// A slice's windows run one after another.  Up to kKgWideMaxN Gaussians
// the slices fit on the GPU at once, and the kernel takes as long as its
// heaviest slice (the nearest, largest Gaussians): 512 threads expand its
// windows faster (1M frame 35.7 -> 29.4 us).  Beyond that the slices come
// in several rounds, and 256-thread workgroups, more of which fit at once,
// are faster (6M frame 82.9 -> 79.1 us).
constexpr int kKgScatThreads = 256;
constexpr int kKgScatWideThreads = 512;
constexpr int kKgScatWin = 2048;
constexpr int64_t kKgWideMaxN = 2000000;
// The rect histogram walks each rect's tile rows in one thread; a wider
// workgroup spreads a slice's large rects over more threads (6M frame
// 72.4 -> 70.8 us, 500k 11.8 -> 10.5 us against 256 threads).
constexpr int kKgHistThreads = 1024;

// Instances in depth order: slice p of the depth-sorted visible list starts
// at kg_prefix[p] (scanned slice counts) and writes (tile id, Gaussian
// index) for each tile of each rect in row-major order.  The expansion is
// spread evenly over the workgroup: per window of 2048 instances, each
// Gaussian marks the position where its run starts (its local index + 1)
// and a block-wide max-scan hands every position its Gaussian, so large
// splats do not serialise a thread.
__global__ __launch_bounds__(kBlock) void k_kg_write(const uint32_t* __restrict__ sorted_idx,
                                                     const uint32_t* __restrict__ vis_count,
                                                     const uint2* __restrict__ sorted_rects,
                                                     int tiles_x,
                                                     const uint32_t* __restrict__ inst_count,
                                                     const uint32_t* __restrict__ kg_prefix,
                                                     uint32_t* __restrict__ tkeys,
                                                     uint32_t* __restrict__ tvals) {
  __shared__ uint32_t s_off[kKgPart];
  __shared__ uint32_t s_lo[kKgPart], s_hi[kKgPart], s_g[kKgPart];
  __shared__ uint32_t s_own[kKgWin];
  __shared__ uint32_t s_tmp[kBlock / 64];
  const int t = threadIdx.x;
  const uint32_t nvis = *vis_count, cap = *inst_count;
  const uint32_t base = blockIdx.x * kKgPart;
  if (base >= nvis) return;
  uint32_t cnt[kKgItems], off[kKgItems], sum = 0;
#pragma unroll
  for (int j = 0; j < kKgItems; ++j) {
    const int li = t * kKgItems + j;
    const uint32_t p = base + li;
    uint32_t g = 0, lo = 0, hi = 0, c = 0;
    if (p < nvis) {
      g = sorted_idx[p];
      const uint2 r = sorted_rects[p];
      lo = r.x;
      hi = r.y;
      c = rect_tiles(lo, hi);
    }
    s_g[li] = g;
    s_lo[li] = lo;
    s_hi[li] = hi;
    cnt[j] = c;
    sum += c;
  }
  uint32_t btot;
  uint32_t run = block_excl_scan(sum, s_tmp, &btot);
#pragma unroll
  for (int j = 0; j < kKgItems; ++j) {
    off[j] = run;
    s_off[t * kKgItems + j] = run;
    run += cnt[j];
  }
  const uint32_t prefix = kg_prefix[blockIdx.x];
  for (uint32_t w0 = 0; w0 < btot; w0 += kKgWin) {
#pragma unroll
    for (int k = 0; k < kKgWinItems; ++k) s_own[t * kKgWinItems + k] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kKgItems; ++j) {
      if (cnt[j] && off[j] < w0 + kKgWin && off[j] + cnt[j] > w0)
        s_own[(off[j] > w0 ? off[j] : w0) - w0] = (uint32_t)(t * kKgItems + j) + 1;
    }
    __syncthreads();
    uint32_t v[kKgWinItems], m = 0;
#pragma unroll
    for (int k = 0; k < kKgWinItems; ++k) {
      v[k] = s_own[t * kKgWinItems + k];
      m = max(m, v[k]);
    }
    uint32_t carry = block_excl_max(m, s_tmp);
#pragma unroll
    for (int k = 0; k < kKgWinItems; ++k) {
      carry = max(carry, v[k]);
      s_own[t * kKgWinItems + k] = carry;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kKgWinItems; ++k) {
      const uint32_t q = (uint32_t)(k * kBlock + t);
      const uint32_t kk = w0 + q;
      if (kk < btot) {
        const uint32_t li = s_own[q] - 1;
        const uint32_t local = kk - s_off[li];
        const uint32_t rl = s_lo[li], rh = s_hi[li];
        const uint32_t tx0 = rl & 0xFFFFu, ty0 = rl >> 16, tx1 = rh & 0xFFFFu;
        const uint32_t w = tx1 - tx0 + 1;
        const uint32_t ry = local / w;
        const uint32_t gp = prefix + kk;
        if (gp < cap) {
          tkeys[gp] = (ty0 + ry) * (uint32_t)tiles_x + tx0 + (local - ry * w);
          tvals[gp] = s_g[li];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- keygen + first tile pass

// First-tile-digit histogram of each 1024-Gaussian slice of the depth-sorted
// visible list, written partition-major (table[slice * NB + d]), with the
// rect gather of k_kg_count.  The tiles of one row of a rect have
// consecutive ids, so their digits are consecutive residues mod NB: each
// row adds one over a circular range of digits, which a difference array
// in LDS takes as two increments (four across the wrap), and each whole
// turn of NB tiles adds one to every digit.
template <int BITS, int NT>
__global__ __launch_bounds__(NT) void k_kg_hist(uint32_t n, const uint32_t* __restrict__ vis_count,
                                                    const uint32_t* __restrict__ sorted_idx,
                                                    const uint2* __restrict__ rects,
                                                    uint2* __restrict__ sorted_rects,
                                                    int tiles_x, uint32_t* __restrict__ table) {
  constexpr int NB = 1 << BITS;
  constexpr int KI = kKgPart / NT;  // slice Gaussians per thread
  __shared__ int s_diff[NB + 1];
  __shared__ uint32_t s_tmp[NT / 64];
  __shared__ uint32_t s_turns;
  const int t = threadIdx.x;
  const uint32_t nvis = *vis_count;
  const uint32_t base = blockIdx.x * kKgPart;
  if (base >= nvis) return;
  for (int d = t; d <= NB; d += NT) s_diff[d] = 0;
  if (t == 0) s_turns = 0;
  // branch-free loads (positions past the end read the last Gaussian and
  // are ignored), so that all four gathers are in flight together
  uint32_t g[KI];
  uint2 r[KI];
#pragma unroll
  for (int j = 0; j < KI; ++j) g[j] = sorted_idx[min(base + j * NT + t, nvis - 1)];
#pragma unroll
  for (int j = 0; j < KI; ++j) r[j] = rects[min(g[j], n - 1)];  // (indices are < n)
  __syncthreads();
  uint32_t turns = 0;
#pragma unroll
  for (int j = 0; j < KI; ++j) {
    const uint32_t p = base + j * NT + t;
    if (p < nvis) {
      sorted_rects[p] = r[j];
      const uint32_t tx0 = r[j].x & 0xFFFFu, ty0 = r[j].x >> 16;
      const uint32_t tx1 = r[j].y & 0xFFFFu, ty1 = r[j].y >> 16;
      const uint32_t w = tx1 - tx0 + 1;
      const uint32_t full = w >> BITS, rem = w & (NB - 1);
      turns += full * (ty1 - ty0 + 1);
      if (rem) {
        for (uint32_t ty = ty0; ty <= ty1; ++ty) {
          const uint32_t a = (ty * (uint32_t)tiles_x + tx0) & (NB - 1), e = a + rem;
          atomicAdd(&s_diff[a], 1);
          if (e <= NB) {
            atomicAdd(&s_diff[e], -1);
          } else {
            atomicAdd(&s_diff[0], 1);
            atomicAdd(&s_diff[e - NB], -1);
          }
        }
      }
    }
  }
  turns = wave_sum_u32(turns);
  if (lane_id() == 0 && turns) atomicAdd(&s_turns, turns);
  __syncthreads();
  const uint32_t v = t < NB ? (uint32_t)s_diff[t] : 0u;
  uint32_t tot;
  const uint32_t incl = block_excl_scan<NT>(v, s_tmp, &tot) + v;
  if (t < NB) table[(size_t)blockIdx.x * NB + t] = incl + s_turns;
}

// Key generation fused with the first radix pass over the tile keys.  Each
// slice's instances (depth order, then row-major within a rect) are
// expanded in windows of 2048 as in k_kg_write, ranked within the window by
// their first tile digit (ballot matching, stable), staged in digit order
// and written at the digit's running offset: its global start (scanned
// digit totals), plus its count in the earlier slices (scanned table),
// plus the earlier windows.  The result is the first pass's output, with
// no key list written and read back in between.  Positions at or past
// `cap` are skipped (capacity overflow); every position below it still
// receives exactly one pair.
template <int BITS, int NT, int WIN>
__global__ __launch_bounds__(NT) void k_kg_scatter(const uint32_t* __restrict__ sorted_idx,
                                                       const uint32_t* __restrict__ vis_count,
                                                       const uint2* __restrict__ sorted_rects,
                                                       int tiles_x,
                                                       const uint32_t* __restrict__ inst_count,
                                                       const uint32_t* __restrict__ table,
                                                       const uint32_t* __restrict__ totals,
                                                       uint32_t* __restrict__ tkeys,
                                                       uint32_t* __restrict__ tvals) {
  constexpr int NB = 1 << BITS;
  constexpr int NW = NT / 64;
  constexpr int IT = WIN / NT;       // window positions per thread
  constexpr int KI = kKgPart / NT;   // slice Gaussians per thread
  static_assert(NT >= (1 << BITS) && kKgPart % NT == 0 && WIN % NT == 0, "shape");
  __shared__ uint32_t s_off[kKgPart];
  __shared__ uint32_t s_lo[kKgPart], s_hi[kKgPart], s_g[kKgPart];
  __shared__ uint32_t s_own[WIN];  // window owners, then the staged keys
  __shared__ uint32_t s_val[WIN];
  __shared__ uint32_t s_whist[NW][NB];
  __shared__ uint32_t s_local[NB], s_scat[NB];
  __shared__ uint32_t s_tmp[NW], s_sc[NW];
  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  const uint32_t nvis = *vis_count, cap = *inst_count;
  const uint32_t nsl = (nvis + kKgPart - 1) / kKgPart;
  if (blockIdx.x >= nsl) return;
  const uint32_t slice = blockIdx.x;
  const uint32_t base = slice * kKgPart;
  // every load of the prologue is issued before the first is used
  // (branch-free: positions past the end read the last Gaussian)
  const uint32_t gcount = t < NB ? totals[t] : 0u;
  const uint32_t tprefix = t < NB ? table[(size_t)slice * NB + t] : 0u;
  uint32_t gi[KI];
  uint2 rr[KI];
#pragma unroll
  for (int j = 0; j < KI; ++j) {
    const uint32_t pc = min(base + t * KI + j, nvis - 1);
    gi[j] = sorted_idx[pc];
    rr[j] = sorted_rects[pc];
  }
  uint32_t cnt[KI], off[KI], sum = 0;
#pragma unroll
  for (int j = 0; j < KI; ++j) {
    const int li = t * KI + j;
    const bool ok = base + li < nvis;
    const uint32_t c = ok ? rect_tiles(rr[j].x, rr[j].y) : 0u;
    s_g[li] = gi[j];
    s_lo[li] = rr[j].x;
    s_hi[li] = rr[j].y;
    cnt[j] = c;
    sum += c;
  }
  uint32_t btot;
  uint32_t run = block_excl_scan<NT>(sum, s_tmp, &btot);
#pragma unroll
  for (int j = 0; j < KI; ++j) {
    off[j] = run;
    s_off[t * KI + j] = run;
    run += cnt[j];
  }
  // running write base of digit t: its global start plus its count in the
  // earlier slices
  uint32_t gb = 0;
  {
    uint32_t all;
    const uint32_t gstart = block_excl_scan<NT>(gcount, s_sc, &all);
    if (t < NB) gb = gstart + tprefix;
  }
  const uint64_t lt = lanemask_lt();
  for (uint32_t w0 = 0; w0 < btot; w0 += WIN) {
#pragma unroll
    for (int k = 0; k < IT; ++k) s_own[t * IT + k] = 0;
    for (int b = t; b < NW * NB; b += NT) (&s_whist[0][0])[b] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KI; ++j) {
      if (cnt[j] && off[j] < w0 + WIN && off[j] + cnt[j] > w0)
        s_own[(off[j] > w0 ? off[j] : w0) - w0] = (uint32_t)(t * KI + j) + 1;
    }
    __syncthreads();
    {
      uint32_t v[IT], m = 0;
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        v[k] = s_own[t * IT + k];
        m = max(m, v[k]);
      }
      uint32_t carry = block_excl_max<NT>(m, s_tmp);
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        carry = max(carry, v[k]);
        s_own[t * IT + k] = carry;
      }
    }
    __syncthreads();
    // this thread's instances, warp-striped: wave w holds window positions
    // [w*64*IT, (w+1)*64*IT), lane-minor, so ranking order = window order
    uint32_t key[IT], val[IT], pos[IT], kept = 0;
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const uint32_t q = (uint32_t)(wave * 64 * IT + i * 64 + lane);
      const uint32_t kk = w0 + q;
      key[i] = 0;
      val[i] = 0;
      if (kk < btot) {
        const uint32_t li = s_own[q] - 1;
        const uint32_t local = kk - s_off[li];
        const uint32_t rl = s_lo[li], rh = s_hi[li];
        const uint32_t tx0 = rl & 0xFFFFu, ty0 = rl >> 16, tx1 = rh & 0xFFFFu;
        const uint32_t w = tx1 - tx0 + 1;
        const uint32_t ry = local / w;
        key[i] = (ty0 + ry) * (uint32_t)tiles_x + tx0 + (local - ry * w);
        val[i] = s_g[li];
        kept |= 1u << i;
      }
    }
    __syncthreads();  // s_own is read; it stages the keys next
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const bool keep = (kept >> i) & 1u;
      const uint32_t d = key[i] & (NB - 1);
      const uint64_t peers = match_digit<BITS>(d, ballot(keep));
      const uint32_t c = s_whist[wave][d];
      pos[i] = c + (uint32_t)__builtin_popcountll(peers & lt);
      if (keep && (peers & lt) == 0) s_whist[wave][d] = c + (uint32_t)__builtin_popcountll(peers);
    }
    __syncthreads();
    uint32_t tot = 0;
    if (t < NB) {
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint32_t x = s_whist[w][t];
        s_whist[w][t] = tot;
        tot += x;
      }
    }
    uint32_t nwin;
    const uint32_t lstart = block_excl_scan<NT>(tot, s_sc, &nwin);
    if (t < NB) {
      s_local[t] = lstart;
      s_scat[t] = gb - lstart;
      gb += tot;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      if ((kept >> i) & 1u) {
        const uint32_t d = key[i] & (NB - 1);
        const uint32_t p = pos[i] + s_local[d] + s_whist[wave][d];
        s_own[p] = key[i];
        s_val[p] = val[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const uint32_t j = (uint32_t)(i * NT + t);
      if (j < nwin) {
        const uint32_t k = s_own[j];
        const uint32_t g = s_scat[k & (NB - 1)] + j;
        if (g < cap) {
          tkeys[g] = k;
          tvals[g] = s_val[j];
        }
      }
    }
    __syncthreads();
  }
}

// The heavy-first tile order of at most kFusedOrderTiles tiles, computed
// by one workgroup from the finished ranges: each tile's class (by the
// length of its list), the class sizes counted with one LDS atomic per
// class and wave, their exclusive scan, then each tile written at its
// class's next free rank.  Order within a class is unspecified.
constexpr int kFoBlock = 1024;                        // threads of the one workgroup
constexpr int kFoPer = kFusedOrderTiles / kFoBlock;  // tiles per thread
constexpr int kFoChunk = 4;                           // range loads in flight per thread
__device__ void order_tiles_block(const uint32_t* ranges, int tiles, uint32_t* order) {
  __shared__ uint32_t s_cnt[kTileClasses];
  __shared__ uint8_t s_cls[kFusedOrderTiles];
  const int t = threadIdx.x, lane = lane_id();
  if (tiles <= 0) return;
  if (t < kTileClasses) s_cnt[t] = 0;
  __syncthreads();
  // thread t takes tiles t, t + kFoBlock, ...: classes into LDS, counted
  for (int j0 = 0; j0 < kFoPer && j0 * kFoBlock < tiles; j0 += kFoChunk) {
    // branch-free loads (past the last tile: the last tile, not used)
    uint2 r[kFoChunk];
#pragma unroll
    for (int j = 0; j < kFoChunk; ++j)
      r[j] = *reinterpret_cast<const uint2*>(ranges + 2 * min((j0 + j) * kFoBlock + t, tiles - 1));
#pragma unroll
    for (int j = 0; j < kFoChunk; ++j) {
      const int tile = (j0 + j) * kFoBlock + t;
      const bool ok = tile < tiles;
      const int lg = 31 - __builtin_clz(r[j].y - r[j].x + 1u);  // floor(log2(len + 1))
      const uint32_t k = (uint32_t)(kTileClasses - 1 - min(lg, kTileClasses - 1));
      if (ok) s_cls[tile] = (uint8_t)k;
      const uint64_t same = match_digit<4>(k, ballot(ok));
      if (ok && lane == __builtin_ctzll(same))
        atomicAdd(&s_cnt[k], (uint32_t)__builtin_popcountll(same));
    }
  }
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    for (int k = 0; k < kTileClasses; ++k) {
      const uint32_t c = s_cnt[k];
      s_cnt[k] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int j = 0; j < kFoPer && j * kFoBlock < tiles; ++j) {
    const int tile = j * kFoBlock + t;
    const bool ok = tile < tiles;
    const uint32_t k = ok ? s_cls[tile] : 0u;
    const uint64_t same = match_digit<4>(k, ballot(ok));
    const int leader = same ? __builtin_ctzll(same) : 0;
    uint32_t base = 0;
    if (ok && lane == leader) base = atomicAdd(&s_cnt[k], (uint32_t)__builtin_popcountll(same));
    base = shfl_u32(base, leader);
    if (ok) order[base + (uint32_t)__builtin_popcountll(same & lanemask_lt())] = (uint32_t)tile;
  }
}

// Tile ranges of the sorted tile keys.  Each thread takes 4 consecutive
// keys with one 16-byte load plus the keys on either side.  The key buffer
// is padded to a multiple of 64 keys, so the vector load of the last group
// stays inside it (keys past n are never used).
__global__ __launch_bounds__(kBlock) void k_tile_ranges(const uint32_t* __restrict__ count,
                                                        const uint32_t* __restrict__ tkeys,
                                                        uint32_t* __restrict__ ranges) {
  const int64_t n = *count;
  const int64_t stride = (int64_t)gridDim.x * kBlock * 4;
  for (int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 4; i0 < n; i0 += stride) {
    const uint4 q = *reinterpret_cast<const uint4*>(tkeys + i0);
    const uint32_t kk[6] = {i0 > 0 ? tkeys[i0 - 1] : 0u, q.x, q.y, q.z, q.w,
                            i0 + 4 < n ? tkeys[i0 + 4] : 0u};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = i0 + j;
      if (i < n) {
        const uint32_t tile = kk[j + 1];
        if (i == 0 || kk[j] != tile) ranges[2 * tile] = (uint32_t)i;
        if (i == n - 1 || kk[j + 2] != tile) ranges[2 * tile + 1] = (uint32_t)(i + 1);
      }
    }
  }
}

// The heavy-first order of at most kFusedOrderTiles tiles in one
// workgroup (one launch instead of the class and order kernels).
__global__ __launch_bounds__(kFoBlock) void k_tile_order_one(const uint32_t* __restrict__ ranges,
                                                           int tiles,
                                                           uint32_t* __restrict__ order) {
  order_tiles_block(ranges, tiles, order);
}

// Heavy-first tile order, step 1: each tile joins its class (by the
// length of its list) at a position taken with one atomic per class and
// wave; class k's members go to seg[k * tiles ..].
__global__ __launch_bounds__(kBlock) void k_tile_classes(const uint32_t* __restrict__ ranges,
                                                         int tiles, uint32_t* cls_count,
                                                         uint32_t* __restrict__ seg) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const bool ok = t < tiles;
  uint32_t k = 0;
  if (ok) {
    const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
    const int lg = 31 - __builtin_clz(len + 1u);  // floor(log2(len + 1)), len + 1 >= 1
    k = (uint32_t)(kTileClasses - 1 - min(lg, kTileClasses - 1));
  }
  const uint64_t same = match_digit<4>(k, ballot(ok));
  const int lane = lane_id();
  const int leader = same ? __builtin_ctzll(same) : 0;
  uint32_t base = 0;
  if (ok && lane == leader) base = atomicAdd(cls_count + k, (uint32_t)__builtin_popcountll(same));
  base = shfl_u32(base, leader);
  if (ok) seg[(size_t)k * tiles + base + (uint32_t)__builtin_popcountll(same & lanemask_lt())] =
      (uint32_t)t;
}

// Step 2: rank r of the order is member r - (members of earlier classes)
// of the first class whose members reach past r.
__global__ __launch_bounds__(kBlock) void k_tile_order(const uint32_t* __restrict__ cls_count,
                                                       const uint32_t* __restrict__ seg,
                                                       int tiles, uint32_t* __restrict__ order) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= tiles) return;
  uint32_t before = 0;
  int k = 0;
  for (; k < kTileClasses - 1; ++k) {
    const uint32_t c = cls_count[k];
    if ((uint32_t)r < before + c) break;
    before += c;
  }
  order[r] = seg[(size_t)k * tiles + ((uint32_t)r - before)];
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

// Keys per thread of a reduce-then-scan pass: enough partitions to give
// every CU a few workgroups (small passes are latency-bound), else 16.
inline int rs_items(int64_t n, int min_parts) {
  const int64_t m = min_parts > 0 ? min_parts : kRsMinParts;
  if ((n + kBlock * 16 - 1) / (kBlock * 16) >= m) return 16;
  if ((n + kBlock * 8 - 1) / (kBlock * 8) >= m) return 8;
  return 4;
}

// Launch of one downsweep kernel with or without key stores.
template <typename KeyT, int BITS, int ITEMS, bool LOOKBACK>
void launch_pass(int grid, bool write_keys, const KeyT* ki, const uint32_t* vi, KeyT* kd,
                 uint32_t* vd, const uint32_t* cnt, int64_t n_grid, int drop,
                 const uint32_t* kbase, int shift, const uint32_t* table, const uint32_t* totals,
                 uint32_t* ticket, uint32_t* lb, uint32_t* lb_next, hipStream_t st) {
  if (write_keys)
    hipLaunchKernelGGL((k_radix_pass<KeyT, BITS, ITEMS, true, LOOKBACK>), dim3(grid),
                       dim3(kBlock), 0, st, ki, vi, kd, vd, cnt, n_grid, drop, kbase, shift,
                       table, totals, ticket, lb, lb_next);
  else
    hipLaunchKernelGGL((k_radix_pass<KeyT, BITS, ITEMS, false, LOOKBACK>), dim3(grid),
                       dim3(kBlock), 0, st, ki, vi, kd, vd, cnt, n_grid, drop, kbase, shift,
                       table, totals, ticket, lb, lb_next);
}

template <typename KeyT, int BITS, int ITEMS>
void rs_pass(const RadixArgs<KeyT>& a, int shift, const uint32_t* cnt, int drop,
             const uint32_t* kbase, const KeyT* ki, const uint32_t* vi, KeyT* kd, uint32_t* vd,
             bool write_keys, const SortInitK& init, hipStream_t st) {
  constexpr int PART = kBlock * ITEMS;
  constexpr int NB = 1 << BITS;
  const int parts = (int)((a.n_grid + PART - 1) / PART);
  hipLaunchKernelGGL((k_rs_upsweep<KeyT, BITS, ITEMS>), dim3(parts), dim3(kBlock), 0, st, ki, cnt,
                     a.n_grid, drop, kbase, shift, a.table, init);
  hipLaunchKernelGGL((k_col_scan<NB, PART>), dim3(NB / 4), dim3(kBlock), 0, st, a.table, cnt,
                     a.n_grid, a.totals);
  launch_pass<KeyT, BITS, ITEMS, false>(parts, write_keys, ki, vi, kd, vd, cnt, a.n_grid, drop,
                                        kbase, shift, a.table, a.totals, nullptr, nullptr, nullptr,
                                        st);
}

// Pass p of a sort whose first pass may drop all-ones keys and take the
// keys relative to *kbase (later passes see the relative keys it wrote).
template <typename KeyT, int BITS>
void rs_pass_items(const RadixArgs<KeyT>& a, int p, int shift, const KeyT* ki, const uint32_t* vi,
                   KeyT* kd, uint32_t* vd, bool write_keys, hipStream_t st) {
  const bool first = p == 0;
  const int drop = first && a.drop_first ? 1 : 0;
  const uint32_t* kbase = first ? a.kbase : nullptr;
  const uint32_t* cnt = (!first && a.drop_first) ? a.count_rest : a.count;
  SortInitK init = a.init;
  init.active = first && a.init.active;  // the set-up runs once, with the first pass
  switch (rs_items(a.n_grid, a.min_parts)) {
    case 16: rs_pass<KeyT, BITS, 16>(a, shift, cnt, drop, kbase, ki, vi, kd, vd, write_keys, init, st); break;
    case 8: rs_pass<KeyT, BITS, 8>(a, shift, cnt, drop, kbase, ki, vi, kd, vd, write_keys, init, st); break;
    default: rs_pass<KeyT, BITS, 4>(a, shift, cnt, drop, kbase, ki, vi, kd, vd, write_keys, init, st); break;
  }
}

template <typename KeyT, int BITS>
void pass_t(const RadixArgs<KeyT>& a, int p, int q, const KeyT* ki, const uint32_t* vi, KeyT* kd,
            uint32_t* vd, bool write_keys, hipStream_t st) {
  const int shift = p * BITS;
  if (a.mode == 1) {
    const bool first = p == 0;
    const int drop = first && a.drop_first ? 1 : 0;
    const uint32_t* kbase = first ? a.kbase : nullptr;
    const uint32_t* cnt = (!first && a.drop_first) ? a.count_rest : a.count;
    const int parts = (int)((a.n_grid + kSortPart - 1) / kSortPart);
    uint32_t* lb = a.lookback + (size_t)(q & 1) * a.lb_parts * 256;
    uint32_t* lb_next = a.lookback + (size_t)((q + 1) & 1) * a.lb_parts * 256;
    const uint32_t* h = a.hist + p * 256;
    launch_pass<KeyT, BITS, kSortItems, true>(parts, write_keys, ki, vi, kd, vd, cnt, a.n_grid,
                                              drop, kbase, shift, nullptr, h, a.tickets + q, lb,
                                              lb_next, st);
  } else {
    rs_pass_items<KeyT, BITS>(a, p, shift, ki, vi, kd, vd, write_keys, st);
  }
}

template <typename KeyT, int BITS>
void hist_t(const RadixArgs<KeyT>& a, int passes, hipStream_t st) {
  const int parts = (int)((a.n_grid + kSortPart - 1) / kSortPart);
  hipLaunchKernelGGL((k_histogram<KeyT, BITS>), dim3(parts < 512 ? parts : 512), dim3(kBlock), 0,
                     st, a.kin, a.count, a.n_grid, a.drop_first, a.kbase, passes, a.hist);
}

}  // namespace

SortLayout sort_layout(int64_t n, int64_t capacity, int tiles) {
  SortLayout L;
  const int64_t nn = n > 0 ? n : 1, cap = capacity > 0 ? capacity : 1;
  const int64_t big = nn > cap ? nn : cap;
  L.parts = (int)((big + kSortPart - 1) / kSortPart);
  L.rs_parts = (int)((big + kBlock * 4 - 1) / (kBlock * 4));
  L.kg_parts = (int)((nn + kKgPart - 1) / kKgPart);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.dk[0] = take((size_t)nn * 4); L.dv[0] = take((size_t)nn * 4);
  L.dk[1] = take((size_t)nn * 4); L.dv[1] = take((size_t)nn * 4);
  L.drect = take((size_t)nn * 8);
  L.tk[0] = take((size_t)cap * 4); L.tv[0] = take((size_t)cap * 4);
  L.tk[1] = take((size_t)cap * 4); L.tv[1] = take((size_t)cap * 4);
  L.tkf = take((size_t)cap * 4);
  L.hist = take((size_t)kMaxPassTotal * 256 * 4);
  L.tickets = take((size_t)kMaxPassTotal * 4);
  L.lookback = take((size_t)2 * L.parts * 256 * 4);
  L.table = take((size_t)L.rs_parts * kMaxDigits * 4);
  L.totals = take(kMaxDigits * 4);
  L.kg_counts = take((size_t)L.kg_parts * 4);
  L.count = take(4);
  L.tcls = take((size_t)kTileClasses * 4);
  L.tseg = take((size_t)kTileClasses * (tiles > 0 ? tiles : 1) * 4);
  L.bytes = o;
  return L;
}

SortLayout pairs_layout(int64_t n) {
  SortLayout L;
  const int64_t nn = n > 0 ? n : 1;
  L.parts = (int)((nn + kSortPart - 1) / kSortPart);
  L.rs_parts = (int)((nn + kBlock * 4 - 1) / (kBlock * 4));
  L.kg_parts = 0;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.dk[0] = take((size_t)nn * 8);  // alternate key buffer (u64)
  L.dv[0] = take((size_t)nn * 4);  // alternate value buffer
  L.dk[1] = L.dv[1] = L.drect = L.tk[0] = L.tv[0] = L.tk[1] = L.tv[1] = L.tkf = 0;
  L.hist = take((size_t)kMaxPassTotal * 256 * 4);
  L.tickets = take((size_t)kMaxPassTotal * 4);
  L.lookback = take((size_t)2 * L.parts * 256 * 4);
  L.table = take((size_t)L.rs_parts * kMaxDigits * 4);
  L.totals = take(kMaxDigits * 4);
  L.kg_counts = 0;
  L.count = take(4);
  L.bytes = o;
  return L;
}

SortInitK sort_init_args(const SortLayout& L, char* ws, uint32_t* tile_ranges, int tiles,
                         uint32_t* status_flag, const uint32_t* total_src, int64_t capacity,
                         uint32_t* cls_count, int depth_bits) {
  SortInitK I{};
  I.ranges = tile_ranges;
  I.ranges_len = tile_ranges ? 2 * tiles : 0;
  I.tickets = reinterpret_cast<uint32_t*>(ws + L.tickets);
  I.ntickets = kMaxPassTotal;
  I.cls_count = cls_count;
  I.count = reinterpret_cast<uint32_t*>(ws + L.count);
  I.total_src = total_src;
  I.host_total = (uint32_t)capacity;
  I.capacity = capacity;
  I.status_flag = status_flag;
  I.depth_bits = depth_bits;
  I.active = 1;
  return I;
}

hipError_t launch_sort_init(const SortLayout& L, char* ws, int mode, uint32_t* tile_ranges,
                            int tiles, uint32_t* status_flag, const uint32_t* total_src,
                            int64_t capacity, hipStream_t st, uint32_t* cls_count,
                            int depth_bits) {
  const int lb_len = mode == 1 ? 2 * L.parts * 256 : 0;
  const SortInitK I = sort_init_args(L, ws, tile_ranges, tiles, status_flag, total_src, capacity,
                                     cls_count, depth_bits);
  const int64_t most = lb_len > I.ranges_len ? lb_len : I.ranges_len;
  hipLaunchKernelGGL(k_sort_init, dim3(stream_grid(most, 1024)), dim3(kBlock), 0, st, I,
                     reinterpret_cast<uint32_t*>(ws + L.hist), mode == 1 ? kMaxPassTotal * 256 : 0,
                     reinterpret_cast<uint32_t*>(ws + L.lookback), lb_len);
  return hipGetLastError();
}

template <typename KeyT>
hipError_t launch_radix_sort(const RadixArgs<KeyT>& a, int bits, int passes, int pass_base,
                             bool last_keys, const char* label, hipStream_t st, int first_pass) {
  if (a.n_grid == 0 || passes <= first_pass) return hipSuccess;
  if (first_pass > 0 && a.mode == 1) return hipErrorInvalidValue;
  if (a.mode == 1) {
    trace_mark(st, "radix_hist");
    switch (bits) {
      case 6: hist_t<KeyT, 6>(a, passes, st); break;
      case 7: hist_t<KeyT, 7>(a, passes, st); break;
      default: hist_t<KeyT, 8>(a, passes, st); break;
    }
  }
  const KeyT* ki = a.kin;
  const uint32_t* vi = a.vin;
  for (int p = first_pass; p < passes; ++p) {
    const int q = pass_base + p;  // global pass index: ticket and look-back buffer parity
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    KeyT* kd = to_out ? a.k_out : a.k_alt;
    uint32_t* vd = to_out ? a.v_out : a.v_alt;
    const bool wk = (p + 1 < passes) || last_keys;
    trace_mark(st, label);
    switch (bits) {
      case 6: pass_t<KeyT, 6>(a, p, q, ki, vi, kd, vd, wk, st); break;
      case 7: pass_t<KeyT, 7>(a, p, q, ki, vi, kd, vd, wk, st); break;
      default: pass_t<KeyT, 8>(a, p, q, ki, vi, kd, vd, wk, st); break;
    }
    ki = kd;
    vi = vd;
  }
  return hipGetLastError();
}
hipError_t launch_radix_sort_widths(const RadixArgs<uint32_t>& a, const int* widths, int passes,
                                    bool last_keys, const char* label, hipStream_t st) {
  if (a.n_grid == 0 || passes == 0) return hipSuccess;
  if (a.mode != 0) return hipErrorInvalidValue;
  const uint32_t* ki = a.kin;
  const uint32_t* vi = a.vin;
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    uint32_t* kd = to_out ? a.k_out : a.k_alt;
    uint32_t* vd = to_out ? a.v_out : a.v_alt;
    const bool wk = (p + 1 < passes) || last_keys;
    trace_mark(st, label);
    switch (widths[p]) {
      case 6: rs_pass_items<uint32_t, 6>(a, p, shift, ki, vi, kd, vd, wk, st); break;
      case 7: rs_pass_items<uint32_t, 7>(a, p, shift, ki, vi, kd, vd, wk, st); break;
      case 8: rs_pass_items<uint32_t, 8>(a, p, shift, ki, vi, kd, vd, wk, st); break;
      case 9: rs_pass_items<uint32_t, 9>(a, p, shift, ki, vi, kd, vd, wk, st); break;
      default: return hipErrorInvalidValue;
    }
    shift += widths[p];
    ki = kd;
    vi = vd;
  }
  return hipGetLastError();
}

template hipError_t launch_radix_sort<uint32_t>(const RadixArgs<uint32_t>&, int, int, int, bool,
                                                const char*, hipStream_t, int);
template hipError_t launch_radix_sort<uint64_t>(const RadixArgs<uint64_t>&, int, int, int, bool,
                                                const char*, hipStream_t, int);

hipError_t launch_keygen(int64_t n, const uint32_t* sorted_idx, const uint32_t* vis_count,
                         const uint2* rects, uint2* sorted_rects, int tiles_x,
                         const uint32_t* inst_count, uint32_t* kg_counts, uint32_t* kg_total,
                         uint32_t* tkeys, uint32_t* tvals, hipStream_t st) {
  const int parts = (int)((n + kKgPart - 1) / kKgPart);
  if (parts == 0) return hipSuccess;
  trace_mark(st, "kg_count");
  hipLaunchKernelGGL(k_kg_count, dim3(parts), dim3(kBlock), 0, st, (uint32_t)n, vis_count,
                     sorted_idx, rects, sorted_rects, kg_counts);
  trace_mark(st, "kg_scan");
  hipLaunchKernelGGL(k_row_scan, dim3(1), dim3(kBlock), 0, st, kg_counts, parts, kg_total);
  trace_mark(st, "keygen");
  hipLaunchKernelGGL(k_kg_write, dim3(parts), dim3(kBlock), 0, st, sorted_idx, vis_count,
                     sorted_rects,
                     tiles_x, inst_count, kg_counts, tkeys, tvals);
  return hipGetLastError();
}

namespace {
template <int BITS>
void kg_fused_t(int64_t n, int parts, const uint32_t* sorted_idx, const uint32_t* vis_count,
                const uint2* rects, uint2* sorted_rects, int tiles_x, const uint32_t* inst_count,
                uint32_t* table, uint32_t* totals, uint32_t* tkeys, uint32_t* tvals,
                hipStream_t st) {
  constexpr int NB = 1 << BITS;
  trace_mark(st, "kg_hist");
  hipLaunchKernelGGL((k_kg_hist<BITS, kKgHistThreads>), dim3(parts), dim3(kKgHistThreads), 0, st,
                     (uint32_t)n, vis_count, sorted_idx, rects, sorted_rects, tiles_x, table);
  trace_mark(st, "kg_scan");
  hipLaunchKernelGGL((k_col_scan<NB, kKgPart>), dim3(NB / 4), dim3(kBlock), 0, st, table,
                     vis_count, (int64_t)0, totals);
  trace_mark(st, "keygen");
  if (n <= kKgWideMaxN)
    hipLaunchKernelGGL((k_kg_scatter<BITS, kKgScatWideThreads, kKgScatWin>), dim3(parts),
                       dim3(kKgScatWideThreads), 0, st, sorted_idx, vis_count, sorted_rects,
                       tiles_x, inst_count, table, totals, tkeys, tvals);
  else
    hipLaunchKernelGGL((k_kg_scatter<BITS, kKgScatThreads, kKgScatWin>), dim3(parts),
                       dim3(kKgScatThreads), 0, st, sorted_idx, vis_count, sorted_rects,
                       tiles_x, inst_count, table, totals, tkeys, tvals);
}
}  // namespace

hipError_t launch_keygen_fused(int64_t n, int bits, const uint32_t* sorted_idx,
                               const uint32_t* vis_count, const uint2* rects,
                               uint2* sorted_rects, int tiles_x, const uint32_t* inst_count,
                               uint32_t* table, uint32_t* totals, uint32_t* tkeys,
                               uint32_t* tvals, hipStream_t st) {
  const int parts = (int)((n + kKgPart - 1) / kKgPart);
  if (parts == 0) return hipSuccess;
  switch (bits) {
    case 6: kg_fused_t<6>(n, parts, sorted_idx, vis_count, rects, sorted_rects, tiles_x, inst_count,
                          table, totals, tkeys, tvals, st); break;
    case 7: kg_fused_t<7>(n, parts, sorted_idx, vis_count, rects, sorted_rects, tiles_x, inst_count,
                          table, totals, tkeys, tvals, st); break;
    default: kg_fused_t<8>(n, parts, sorted_idx, vis_count, rects, sorted_rects, tiles_x,
                           inst_count, table, totals, tkeys, tvals, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_tile_ranges(int64_t capacity, const uint32_t* count, const uint32_t* tkeys,
                              uint32_t* ranges, hipStream_t st) {
  if (capacity == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_ranges, dim3(stream_grid((capacity + 3) / 4, 4096)), dim3(kBlock), 0,
                     st, count, tkeys, ranges);
  return hipGetLastError();
}

hipError_t launch_tile_order(uint32_t* ranges, int tiles, uint32_t* cls_count, uint32_t* seg,
                             hipStream_t st) {
  if (tiles <= 0) return hipSuccess;
  if (tiles <= kFusedOrderTiles) {
    hipLaunchKernelGGL(k_tile_order_one, dim3(1), dim3(kFoBlock), 0, st, ranges, tiles,
                       ranges + 2 * (size_t)tiles);
    return hipGetLastError();
  }
  const int grid = (tiles + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_tile_classes, dim3(grid), dim3(kBlock), 0, st, ranges, tiles, cls_count,
                     seg);
  hipLaunchKernelGGL(k_tile_order, dim3(grid), dim3(kBlock), 0, st, cls_count, seg, tiles,
                     ranges + 2 * (size_t)tiles);
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
