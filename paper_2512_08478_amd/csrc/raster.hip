// Tile compositing (Section 3.2 Eqs. 2-3) forward and backward.
//
// The sort groups splats by tile (TW x TH pixels).  Both kernels run one
// 64-thread workgroup -- one wave -- per 8x8 quadrant of a tile, each lane
// owning one pixel; the quadrant walks its tile's whole list (in (depth,
// index) order) and works only on the splats that reach it.  Quadrants of
// one tile never wait on each other, and the grid has four to eight times
// as many workgroups as tiles, which balances uneven lists.  Splats are
// staged through LDS in batches of 64:
//   * only the splats whose opacity-aware footprint (where
//     o exp(-Q/2) >= alpha_min) reaches the quadrant -- by the pixel bbox
//     that preprocess rounded outwards from the ellipse's exact extents --
//     are staged, densely and in list order, so the compositing loops walk
//     them with a plain counter and no per-splat mask bookkeeping;
//   * each staged splat gets per-row terms of the log2 weight
//       e = log2(o) - (log2e/2) Q = rowterm[r] - qa' (ubase[r] + lx)^2,
//     with Q = qa (dx - qb dy)^2 + qc dy^2, qa' = qa log2e/2, and
//     ubase[r] the value of dx - qb dy at the quadrant's first column in
//     row r.  A pixel then costs an add, a multiply and an fma.  The terms
//     depend only on the pixel's row and 8-aligned column group, never on
//     the tile shape, so every tile shape gives bitwise-identical images;
//     the backward kernel stages them identically, so its skip decisions
//     match the forward pass exactly.
// Per pixel, front to back: skip when e < log2(alpha_min); otherwise
// alpha = min(alpha_max, 2^e), C += T alpha rgb, T *= 1 - alpha, and stop
// right after the blend that takes T below t_eps.  The workgroup leaves
// once all its pixels have stopped.
//
// Mesh depth composition (Algorithm 1, DrawSplatsWithMeshDepth; Section
// 3.4): given the camera-space depth D(p) of a mesh prepass, a splat whose
// depth exceeds D(p) is hidden at pixel p; the list is in depth order, so
// the pixel stops at the first such splat.  The mesh colour, if given,
// takes the place of the background behind the Gaussians.
//
// Order of the quadrants (pick_unit): by default the tiles with the
// longest lists start first (the sort writes that order), which keeps a few
// dense tiles from running alone at the end; or block-cyclic runs of
// neighbouring tiles over the XCDs, whose L2s then share those tiles'
// splats.  Either way dense regions are spread over all eight XCDs.
#include <utility>

#include "gs_device.h"
#include "gs_internal.h"

namespace gs {
namespace {

constexpr float kHalfLog2e = 0.72134752044448170f;  // log2(e) / 2
constexpr float kLn2 = 0.69314718055994531f;
constexpr int kXcds = 8;
constexpr int kRunTiles = 16;  // tiles per XCD run

// 2^e on the hardware exponential unit.  Only exponents at or above
// log2(alpha_min) reach it, far from the denormal range, so the library's
// range reduction is unnecessary; forward and backward share it, so both
// see the same alpha.
__device__ __forceinline__ float hw_exp2(float e) { return __builtin_amdgcn_exp2f(e); }

// Block-cyclic over the XCDs: runs of `run` consecutive units (whole
// tiles' quadrants, neighbouring tiles of one tile row) go to the XCDs in
// turn, so every XCD's L2 sees coherent runs while dense image regions are
// spread over all eight.  Units past the end return at once.
__host__ __device__ __forceinline__ int xcd_tile(int b, int run) {
  const int x = b % kXcds, i = b / kXcds;
  return ((i / run) * kXcds + x) * run + i % run;
}

// The tile, quadrant and row band of workgroup b.  raster_order bit 0 clear:
// block-cyclic runs (xcd_tile).  Bit 0 set: the tiles in the heavy-first
// order that the sort wrote after the ranges, one tile's units on one XCD,
// runs of kRunTiles consecutive ranks dealt to the XCDs in turn: the
// longest lists start first and spread over the chip, and since the order
// keeps each wave's tiles of a class in row-major order, a run is mostly
// neighbouring tiles, which share splats in that XCD's L2.
// raster_order >> 1 = ls (forward only, SPLIT): each quadrant is 2^ls
// units of 8 >> ls pixel rows (bands), each staging only the splats that
// reach its rows.  A dense tile's walk is then split over 2^ls waves,
// which shortens the tail of a frame whose time goes to a few long lists,
// at the price of idle lanes and of staging a splat once per band it
// reaches.  band is in [0, 2^ls).
// False for padding workgroups (and for an order entry out of range, which
// only a caller mixing raster_order values can produce).
// The same on the host (gs_raster_unit, for tests): nq quadrants per
// tile, ls = log2 bands per quadrant, `order` the heavy-first tile order.
__host__ __device__ __forceinline__ bool unit_of(int b, int tiles, int nq, int raster_order,
                                                 int ls, const uint32_t* order, int& tile,
                                                 int& q, int& band) {
  const int U = nq << ls;  // units per tile
  int u;
  if (raster_order & 1) {
    const int x = b % kXcds, i = b / kXcds, j = i / U;  // this XCD's j-th tile
    const int rank = ((j / kRunTiles) * kXcds + x) * kRunTiles + j % kRunTiles;
    if (rank >= tiles) return false;
    tile = (int)order[rank];
    u = i % U;
    if (tile >= tiles) return false;
  } else {
    const int unit = xcd_tile(b, kRunTiles * U);
    if (unit >= tiles * U) return false;
    tile = unit / U;
    u = unit % U;
  }
  q = u >> ls;
  band = u & ((1 << ls) - 1);
  return true;
}

template <int NQ, bool SPLIT>
__device__ __forceinline__ bool pick_unit(int b, const SetK& set,
                                          const uint32_t* __restrict__ ranges, int& tile,
                                          int& q, int& band) {
  const int tiles = set.tiles_x * set.tiles_y;
  const int ls = SPLIT ? (set.raster_order >> 1) : 0;  // log2 bands per quadrant
  return unit_of(b, tiles, NQ, set.raster_order, ls, ranges + 2 * tiles, tile, q, band);
}

inline int xcd_grid(int units, int run) {
  const int per = kXcds * run;
  return (units + per - 1) / per * per;
}

inline int raster_grid(const SetK& set, int tw, int th, bool split) {
  const int tiles = set.tiles_x * set.tiles_y;
  const int u = ((tw / 8) * (th / 8)) << (split ? set.raster_order >> 1 : 0);
  return xcd_grid(tiles * u, kRunTiles * u);
}


// LDS staging of one batch of splats for one 8x8 quadrant, shared by the
// forward and backward kernels.  Only the splats whose footprint reaches
// the quadrant are staged, densely in list order (their rank among the
// batch's hits), so the compositing loops walk them with a plain counter.
// Row terms are stored row-contiguous per splat, so the writes
// (consecutive threads on consecutive rows) and the wave's reads (its 8
// rows of one splat) both touch consecutive words.
constexpr int kBatch = 64;  // splats per batch: one per lane
// The forward stages no backward terms: its smaller LDS footprint lets more
// of its one-wave workgroups share a CU.
template <bool DEPTH, bool BWD>
struct StageT {
  float4 hdr[kBatch];      // qa', r, g, b
  float2 rows[kBatch][8];  // per quadrant row: log2(o) - qc' dy^2, and dx - qb dy at the
                           // quadrant's first column
  uint32_t pos[kBatch];    // the splat's position in the tile's list (as the kernel counts it)
  float dep[DEPTH ? kBatch : 1];  // camera-space depth (mesh depth test only)
  float4 aux[BWD ? kBatch : 1];   // qb, qc', dy at the quadrant's first row, 1 / opacity
  uint32_t gid[BWD ? kBatch : 1];  // Gaussian index
};

// The LDS operands of staged splats k and k + 1 at one pixel row: the row
// terms (log2 weight offset, dx - qb dy at the first column) and headers.
struct PairOps {
  float2 q0, q1;
  float4 h0, h1;
  float d0, d1;  // depths (mesh depth test only)
};
template <bool DEPTH, int K>
__device__ __forceinline__ void read_pair(const StageT<DEPTH, false>& S, std::integral_constant<int, K>,
                                          int row, PairOps& o) {
  o.q0 = S.rows[K][row];
  o.q1 = S.rows[K + 1][row];
  o.h0 = S.hdr[K];
  o.h1 = S.hdr[K + 1];
  if constexpr (DEPTH) {
    o.d0 = S.dep[K];
    o.d1 = S.dep[K + 1];
  }
}

// Calls f(0), f(2), f(4), ... with compile-time arguments until one returns
// false: a fully unrolled walk over the pairs of a batch.
template <typename F, int... K>
__device__ __forceinline__ void walk_pairs(F&& f, std::integer_sequence<int, K...>) {
  (void)(f(std::integral_constant<int, 2 * K>{}) && ...);
}

// A batch of views (set.n_views > 0): the view whose band of tile rows holds
// grid tile row `trow` (binary search over the bands' first rows); its
// tile row within the view, size and pixel offset.  Returns false for a
// tile right of the view's last tile column (the grid is as wide as the
// widest view; such tiles never hold splats).
__device__ __forceinline__ bool view_of_tile(const SetK& set, int trow, int tcol, int& vrow,
                                             int& W, int& H, size_t& pix) {
  int lo = 0, hi = set.n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (set.views[mid].row <= trow) lo = mid;
    else hi = mid - 1;
  }
  const ViewK& v = set.views[lo];
  vrow = trow - v.row;
  W = v.W;
  H = v.H;
  pix = v.pix;
  return tcol < v.tiles_x && vrow < v.tiles_y;
}

// The fields of a splat record the compositing kernels read.
struct SplatRec {
  float4 a;  // mx, my, qa, qb
  float4 b;  // qc, opacity, r, g
  float c;   // b
  float depth;
  uint32_t lo, hi;  // pixel bbox: px0 | py0 << 16, px1 | py1 << 16
};

__device__ __forceinline__ SplatRec load_splat(const gs_splat* __restrict__ splats, uint32_t g) {
  const float4* rec = reinterpret_cast<const float4*>(splats + g);
  SplatRec r;
  r.a = rec[0];
  r.b = rec[1];
  const float4 t = rec[2];
  r.c = t.x;
  r.depth = t.y;
  r.lo = __float_as_uint(t.z);
  r.hi = __float_as_uint(t.w);
  return r;
}

// Staging of one batch, called by every lane of the wave (lane j holds the
// batch's j-th splat when `valid`): whether the splat's footprint reaches
// pixel rows hy0..hy1 of the quadrant whose top-left pixel is (qx0, qy0)
// (all 8 rows, or the band the wave composites), and if so its
// parameters, list position `pos` and per-row weight terms (with BWD also
// the backward's terms and the Gaussian index g), written
// at its rank among the batch's hits.  The reach test uses the record's
// pixel bbox, which preprocess rounded outwards from the opacity-aware
// footprint.  DEPTH also stages the depth.  An odd count is padded with
// one splat that no pixel takes (its log2 weight is -inf and it hides
// nothing), so the forward walk can take the splats in pairs without a
// test.  Returns the number of hits.
template <bool DEPTH, bool BWD>
__device__ __forceinline__ int stage_batch(StageT<DEPTH, BWD>& S, bool valid, const SplatRec& r,
                                           uint32_t g, uint32_t pos, int qx0, int qy0,
                                           int lane, int hy0, int hy1) {
  const float4 a = r.a, b = r.b;
  const float c = r.c;
  const float mx = a.x, my = a.y, qb = a.w;  // mean relative to the bbox corner (px0, py0)
  const float qa_ = a.z * kHalfLog2e, qc_ = b.x * kHalfLog2e;
  const float lo = log2f(b.y);
  const int px0 = (int)(r.lo & 0xFFFFu), py0 = (int)(r.lo >> 16);
  const int px1 = (int)(r.hi & 0xFFFFu), py1 = (int)(r.hi >> 16);
  const bool hit = valid && px0 <= qx0 + 7 && px1 >= qx0 && py0 <= hy1 && py1 >= hy0;
  const uint64_t hits = ballot(hit);
  const int nh = __builtin_popcountll(hits);
  if (hit) {
    const int k = __builtin_popcountll(hits & ((1ull << lane) - 1ull));
    S.hdr[k] = make_float4(qa_, b.z, b.w, c);
    // pixel offsets from the mean: exact integer differences from the bbox
    // corner, minus the mean's (small) offset from it
    const float uy = (float)(qy0 - py0) + 0.5f - my;  // dy at the quadrant's first row
    if constexpr (BWD) {  // only the backward's gradient terms and atomics read these
      S.aux[k] = make_float4(qb, qc_, uy, 1.f / b.y);
      S.gid[k] = g;
    }
    S.pos[k] = pos;
    if constexpr (DEPTH) S.dep[k] = r.depth;
    // log2(o) - qc' dy^2 and dx - qb dy at the first column, per row
    const float ux = (float)(qx0 - px0) + 0.5f - mx;
    float4* dst = reinterpret_cast<float4*>(S.rows[k]);
    if (hy1 - hy0 == 7) {  // the whole quadrant
      float2 t[8];
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const float dy = uy + (float)rr;
        t[rr] = make_float2(fmaf(-qc_, dy * dy, lo), fmaf(-qb, dy, ux));
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        dst[rr] = make_float4(t[2 * rr].x, t[2 * rr].y, t[2 * rr + 1].x, t[2 * rr + 1].y);
    } else {  // a band of 2 or 4 rows starting at an even row: only its rows
      for (int rr = hy0 - qy0; rr <= hy1 - qy0; rr += 2) {
        const float dy0 = uy + (float)rr, dy1 = uy + (float)(rr + 1);
        dst[rr >> 1] = make_float4(fmaf(-qc_, dy0 * dy0, lo), fmaf(-qb, dy0, ux),
                                   fmaf(-qc_, dy1 * dy1, lo), fmaf(-qb, dy1, ux));
      }
    }
  }
  if ((nh & 1) && lane < 8) {  // nh is odd, so slot nh < kBatch is free
    S.rows[nh][lane] = make_float2(-__builtin_inff(), 0.f);
    if (lane == 0) {
      S.hdr[nh] = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (DEPTH) S.dep[nh] = -__builtin_inff();
    }
  }
  return nh;
}

// One 64-thread workgroup (one wave) per 8x8 quadrant of a TW x TH tile:
// it walks the tile's whole list and composites the splats that reach its
// quadrant.  Waves of one tile never wait on each other, and a quadrant
// whose pixels have all stopped leaves at once.
template <int TW, int TH, bool MESH, bool COUNT>
__global__ __launch_bounds__(64) void k_raster(const gs_splat* __restrict__ splats,
                                               const uint32_t* __restrict__ values,
                                               const uint32_t* __restrict__ ranges,
                                               SetK set, int W, int H,
                                               const float* __restrict__ mesh_depth,
                                               const float* __restrict__ mesh_rgb,
                                               float* __restrict__ image,
                                               float* __restrict__ T_final,
                                               uint32_t* __restrict__ last,
                                               uint32_t* __restrict__ n_blend) {
  constexpr int QX = TW / 8, NQ = (TW / 8) * (TH / 8);
  __shared__ StageT<MESH, false> S;
  int tile, q, band;
  if (!pick_unit<NQ, true>(blockIdx.x, set, ranges, tile, q, band)) return;
  int trow = tile / set.tiles_x;
  if (set.n_views > 0) {  // a batch: this tile's view, its pixels
    size_t pix;
    if (!view_of_tile(set, trow, tile % set.tiles_x, trow, W, H, pix)) return;
    image += 4 * pix;
    T_final += pix;
    last += pix;
    if (COUNT) n_blend += pix;
  }
  const int tx0 = (tile % set.tiles_x) * TW + 8 * (q % QX);
  const int ty0 = trow * TH + 8 * (q / QX);
  if (tx0 >= W || ty0 >= H) return;  // quadrant wholly outside the image
  const int lane = threadIdx.x;
  const int lx = lane & 7, row = lane >> 3;
  const int px = tx0 + lx, py = ty0 + row;
  // a band unit takes the pixels of its rows; the other lanes stay idle
  const int ls = set.raster_order >> 1, prow = 8 >> ls;  // pixel rows per unit
  const bool inside = px < W && py < H && (row >> (3 - ls)) == band;
  const int hy0 = ty0 + prow * band, hy1 = hy0 + prow - 1;
  const float lxf = (float)lx;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  const float log2_tau = set.log2_tau, t_eps = set.t_eps;
  const float amax = set.amax;

  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  uint32_t lastc = 0, nb = 0;
  bool done = !inside;
  // The pixel takes a splat when its log2 weight reaches `thr`:
  // log2(alpha_min) while the pixel composites, +inf once it stopped (T
  // fell below t_eps, a mesh hides the splats from here on, or the pixel
  // lies outside the image), so one compare decides and the loop needs no
  // lane-mask bookkeeping.  No log2 weight is +inf.
  const float kStopped = __builtin_inff();
  float thr = log2_tau;
  // mesh depth at this pixel (splats deeper than it are hidden)
  float D = __builtin_inff();
  if (MESH && inside) D = mesh_depth[py * W + px];
  // Software pipeline over batches: while a batch composites, the records
  // of the next batch and the indices of the one after are in flight.
  // Loads past the range are clamped to its last entry (their values are
  // never staged); branch-free loads let the compiler keep them in flight
  // across the compositing of the current batch.
  const uint32_t lastpos = end > start ? end - 1 : start;
  uint32_t g_cur = 0, g_next = 0;
  SplatRec r_cur = {};
  if (start < end) {
    g_cur = values[min(start + lane, lastpos)];
    g_next = values[min(start + kBatch + lane, lastpos)];
    r_cur = load_splat(splats, g_cur);
  }
  for (uint32_t bs = start; bs < end; bs += kBatch) {
    if (!ballot(!done)) break;
    const int cnt = (int)min((uint32_t)kBatch, end - bs);
    __syncthreads();  // the previous batch's reads of S are done
    int nh = stage_batch<MESH, false>(S, lane < cnt, r_cur, g_cur, bs - start + lane + 1, tx0,
                                      ty0, lane, hy0, hy1);
    // an opaque 32-bit scalar, so that the walk's end tests stay one
    // scalar compare (the compiler otherwise compares the 64-bit mask)
    asm volatile("" : "+s"(nh));
    const SplatRec r_next = load_splat(splats, g_next);
    const uint32_t g_after = values[min(bs + 2 * kBatch + lane, lastpos)];
    __syncthreads();
    // Lanes never branch apart here: a pair a lane must not blend (weight
    // below alpha_min, or the pixel already stopped) gets alpha = 0, which
    // leaves C and T bitwise unchanged; only wave-uniform branches remain
    // (no lane blends this splat; every pixel of the wave has stopped).
    // Testing a splat costs 4 vector instructions per pair (u, u^2, the
    // log2 weight, the compare).  Predicated blends beat exec-masked ones
    // here: the mask changes lengthen the walk of a wave that runs alone.
    thr = done ? kStopped : log2_tau;
    int lastk = -1;  // rank of this batch's last splat blended into the pixel
    // `tested`: the caller has already found a lane that may take the
    // splat (a superset: thresholds only rise), so the blend runs without
    // a test of its own; lanes that do not take it leave everything as is.
    auto blend = [&](int k, float e, float cr, float cg, float cb, float dep, bool tested) {
      if constexpr (MESH) thr = dep > D ? kStopped : thr;  // hidden from here on
      const bool take = e >= thr;
      if (!tested && !ballot(take)) return;
      // min(alpha_max, 2^e) as a median (2^e > 0): one instruction
      const float alpha = take ? __builtin_amdgcn_fmed3f(hw_exp2(e), 0.f, amax) : 0.f;
      const float w = alpha * T;
      C0 = fmaf(w, cr, C0);
      C1 = fmaf(w, cg, C1);
      C2 = fmaf(w, cb, C2);
      T = T - w;  // T (1 - alpha), one instruction fewer
      lastk = take ? k : lastk;
      if constexpr (COUNT) nb += take ? 1u : 0u;
      thr = T < t_eps ? kStopped : thr;
    };
    // Two staged splats per step (an odd count ends on the padding splat),
    // unrolled so that every LDS address and rank is a constant; the walk
    // stops after the staged splats or soon after every pixel has stopped.  Each
    // step first reads the next pair's operands into the other of two
    // register sets (slots past the staged splats hold stale values that
    // are never used), so a wave running alone does not wait for LDS on
    // every step.
    PairOps ops[2];
    read_pair(S, std::integral_constant<int, 0>{}, row, ops[0]);
    auto step = [&](auto kc) -> bool {
      constexpr int k = decltype(kc)::value;
      constexpr int cur = (k / 2) & 1;
      if (k >= nh) return false;
      if constexpr (k + 2 < kBatch)
        read_pair(S, std::integral_constant<int, k + 2>{}, row, ops[cur ^ 1]);
      const PairOps& o = ops[cur];
      // both headers whole in registers here: otherwise the colour reads
      // sink into the blend and wait for LDS a second time
      float r0 = o.h0.y, g0 = o.h0.z, b0 = o.h0.w;
      asm volatile("" ::"v"(r0), "v"(g0), "v"(b0));
      const float u0 = o.q0.y + lxf, u1 = o.q1.y + lxf;
      const float e0 = fmaf(-o.h0.x, u0 * u0, o.q0.x);
      const float e1 = fmaf(-o.h1.x, u1 * u1, o.q1.x);
      // whether a lane may take the second splat, decided before the first
      // blends, so that branch does not wait on the first blend's results
      const bool any1 = ballot(e1 >= thr) != 0;
      blend(k, e0, r0, g0, b0, o.d0, false);
      if (any1) blend(k + 1, e1, o.h1.y, o.h1.z, o.h1.w, o.d1, true);
      // whether every pixel has stopped, tested after every second pair (a
      // wave that has stopped walks at most one pair more, with no effect)
      if constexpr ((k / 2) % 2 == 1) return ballot(thr != kStopped) != 0;
      return true;
    };
    walk_pairs(step, std::make_integer_sequence<int, kBatch / 2>{});
    if (lastk >= 0) lastc = S.pos[lastk];
    done = thr == kStopped;
    g_cur = g_next;
    r_cur = r_next;
    g_next = g_after;
  }
  if (inside) {
    const int p = py * W + px;
    float b0 = set.bg[0], b1 = set.bg[1], b2 = set.bg[2];
    if (mesh_rgb) {
      b0 = mesh_rgb[3 * p];
      b1 = mesh_rgb[3 * p + 1];
      b2 = mesh_rgb[3 * p + 2];
    }
    reinterpret_cast<float4*>(image)[p] =
        make_float4(fmaf(T, b0, C0), fmaf(T, b1, C1), fmaf(T, b2, C2), 1.f - T);
    T_final[p] = T;
    last[p] = lastc;
    if (COUNT) n_blend[p] = nb;
  }
}

// Backward: walk each pixel's blended splats back to front from `last`,
// recovering T_i = T_{i+1} / (1 - alpha_i) from T_final.  With
//   S_i = colour composited behind i (normalised by T_{i+1}),
//   B_i = T_final / T_{i+1},
// dC/dalpha_i = T_i (c_i - S_i - B_i bg) and dA/dalpha_i = T_i B_i.
// Per splat the 9 partial derivatives are summed over each pixel row (8
// lanes) with DPP; the last lane of each row stores its 9 sums to LDS,
// lanes 0-8 each add up one value's 8 row sums and add it to the
// Gaussian's 2-D gradient record: one float-atomic instruction per splat
// and quadrant.
//
// Each 8x8 quadrant of a TW x TH tile is its own one-wave workgroup that
// walks the tile's whole list (skipping splats that miss the quadrant), so
// a frame has tiles * (TW/8) * (TH/8) small workgroups: the per-pair work
// here is heavy, and small workgroups balance it across the CUs far better
// than one workgroup per tile.  A quadrant stages exactly the row terms the
// forward kernel used for its pixels, so every skip decision matches.
template <int TW, int TH>
__global__ __launch_bounds__(64) void k_raster_bwd(const gs_splat* __restrict__ splats,
                                                   const uint32_t* __restrict__ values,
                                                   const uint32_t* __restrict__ ranges,
                                                   SetK set, int W, int H,
                                                   const float* __restrict__ bg_rgb,
                                                   const float* __restrict__ T_final,
                                                   const uint32_t* __restrict__ last,
                                                   const float* __restrict__ dL_dimage,
                                                   float* __restrict__ grad2d) {
  constexpr int QX = TW / 8, NQ = (TW / 8) * (TH / 8);
  __shared__ StageT<false, true> S;
  // per 8-lane group (pixel row): the 9 gradient sums of up to two splats
  __shared__ __attribute__((aligned(16))) float s_red[8][24];
  int tile, q, band;
  if (!pick_unit<NQ, false>(blockIdx.x, set, ranges, tile, q, band)) return;
  int trow = tile / set.tiles_x;
  if (set.n_views > 0) {  // a batch: this tile's view, its pixels
    size_t pix;
    if (!view_of_tile(set, trow, tile % set.tiles_x, trow, W, H, pix)) return;
    if (bg_rgb) bg_rgb += 3 * pix;
    T_final += pix;
    last += pix;
    dL_dimage += 4 * pix;
  }
  const int tx0 = (tile % set.tiles_x) * TW + 8 * (q % QX);
  const int ty0 = trow * TH + 8 * (q / QX);
  if (tx0 >= W || ty0 >= H) return;  // quadrant wholly outside the image
  const int lane = threadIdx.x;
  const int lx = lane & 7, row = lane >> 3;
  const int px = tx0 + lx, py = ty0 + row;
  const bool inside = px < W && py < H;
  const float lxf = (float)lx, rowf = (float)row;
  const uint32_t start = ranges[2 * tile];
  const float log2_tau = set.log2_tau;

  float T = 1.f, dC0 = 0.f, dC1 = 0.f, dC2 = 0.f, dA = 0.f;
  float b0 = set.bg[0], b1 = set.bg[1], b2 = set.bg[2];  // colour behind the Gaussians
  uint32_t mylast = 0;
  if (inside) {
    const int p = py * W + px;
    T = T_final[p];
    mylast = last[p];
    const float4 g = reinterpret_cast<const float4*>(dL_dimage)[p];
    dC0 = g.x; dC1 = g.y; dC2 = g.z; dA = g.w;
    if (bg_rgb) {
      b0 = bg_rgb[3 * p];
      b1 = bg_rgb[3 * p + 1];
      b2 = bg_rgb[3 * p + 2];
    }
  }
  // the quadrant's largest `last`: later splats blend into none of its pixels
  uint32_t nlast = mylast;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) nlast = max(nlast, shfl_u32(nlast, lane ^ d));
  nlast = __builtin_amdgcn_readfirstlane(nlast);
  const float bgdot = dC0 * b0 + dC1 * b1 + dC2 * b2;
  float S0 = 0.f, S1 = 0.f, S2 = 0.f, B = 1.f;

  // batches cover positions [0, nlast) of the tile's range, last batch first
  const int nb = (int)((nlast + kBatch - 1) / kBatch);
  for (int bi = nb - 1; bi >= 0; --bi) {
    const uint32_t bs = (uint32_t)bi * kBatch;
    __syncthreads();
    const int cnt = (int)min((uint32_t)kBatch, nlast - bs);
    uint32_t g = 0;
    SplatRec rec = {};
    if (lane < cnt) {
      g = values[start + bs + lane];
      rec = load_splat(splats, g);
    }
    const int nh = stage_batch<false, true>(S, lane < cnt, rec, g, bs + lane, tx0, ty0, lane,
                                            ty0, ty0 + 7);
    __syncthreads();
    // Lanes never branch apart: a pair a lane must not revisit (position at
    // or past its `last`, or weight below alpha_min) gets alpha = 0, which
    // leaves T, S and B bitwise unchanged and yields zero gradients.
    // One splat's visit: the back-to-front state update and this lane's
    // gradient terms (zero where the lane does not take the splat).  False
    // when no lane takes it (nothing changes).
    struct Terms {
      float q, a, uu, r, g, b;  // dQ, dQ qa' u, dQ u^2, dL/d(r, g, b) of the pixel
    };
    auto visit = [&](int k, float u, float e, const float4& h, Terms& t) -> bool {
      const bool take = S.pos[k] < mylast && e >= log2_tau;
      if (!ballot(take)) return false;
      const float gw = take ? hw_exp2(e) : 0.f;
      const float alpha = __builtin_amdgcn_fmed3f(gw, 0.f, set.amax);  // as the forward
      const float om = 1.f - alpha;
      // T before this splat; 1 - alpha >= 1 - alpha_max, far from 0
      const float Ti = take ? T * __builtin_amdgcn_rcpf(om) : T;
      const float cr = h.y, cg = h.z, cb = h.w;
      const float w = alpha * Ti;
      const float dalpha = Ti * (dC0 * (cr - S0) + dC1 * (cg - S1) + dC2 * (cb - S2) -
                                 B * bgdot + dA * B);
      S0 = fmaf(alpha, cr - S0, S0);
      S1 = fmaf(alpha, cg - S1, S1);
      S2 = fmaf(alpha, cb - S2, S2);
      B *= om;
      T = Ti;
      // weight 2^e, e = log2(o) - Q', Q' = qa' u^2 + qc' dy^2,
      // u = dx - qb dy, dx = px + 1/2 - mean_x, dy = py + 1/2 - mean_y;
      // no gradient flows through alpha where the alpha_max clamp binds
      const float dal = take && gw < set.amax ? dalpha : 0.f;
      t.q = -kLn2 * gw * dal;  // dL/dQ'
      t.a = t.q * (h.x * u);
      t.uu = t.q * (u * u);
      t.r = dC0 * w;
      t.g = dC1 * w;
      t.b = dC2 * w;
      return true;
    };
    // The 9 gradient sums of splat k over this lane's pixel row, written
    // by the row's last lane to dst[0..8].  Per pixel, with dQ = dL/dQ':
    //   mean x: -2 dQ qa' u      mean y: 2 dQ (qa' u qb - qc' dy)
    //   qa': c dQ u^2            qb: -2 dQ qa' u dy
    //   qc': c dQ dy^2           opacity: dal 2^e / o = -dQ / (ln2 o)
    // (c = log2(e) / 2).  dy is the same for the 8 pixels of a row, so the
    // row's 9 sums follow from the row sums of dQ, dQ qa' u and dQ u^2 and
    // the 3 colour terms.
    auto row_sums = [&](int k, const Terms& t, float* dst) {
      const float sQ = oct_sum_dpp(t.q), sA = oct_sum_dpp(t.a), sU = oct_sum_dpp(t.uu);
      const float sr = oct_sum_dpp(t.r), sg = oct_sum_dpp(t.g), sb = oct_sum_dpp(t.b);
      if ((lane & 7) == 7) {
        const float4 x = S.aux[k];  // qb, qc', dy at the quadrant's first row, 1 / opacity
        const float dy = x.z + rowf;
        *reinterpret_cast<float4*>(dst) =
            make_float4(-2.f * sA, 2.f * (sA * x.x - (x.y * dy) * sQ), kHalfLog2e * sU,
                        -2.f * dy * sA);
        *reinterpret_cast<float4*>(dst + 4) =
            make_float4(kHalfLog2e * (dy * dy) * sQ, -sQ * x.w * (1.f / kLn2), sr, sg);
        dst[8] = sb;
      }
    };
    // The 8 rows' sums added up and sent with one float-atomic instruction:
    // lane j < 9 adds value j of splat k0, lane 12 + j value j of splat k1
    // (when `both`).
    auto send = [&](int k0, int k1, bool both) {
      const int j = lane % 12;
      if (lane < (both ? 24 : 12) && j < 9) {
        const float v = ((s_red[0][lane] + s_red[1][lane]) + (s_red[2][lane] + s_red[3][lane])) +
                        ((s_red[4][lane] + s_red[5][lane]) + (s_red[6][lane] + s_red[7][lane]));
        const uint32_t gid = S.gid[lane < 12 ? k0 : k1];
        atomicAdd(grad2d + (size_t)gid * kGrad2dStride + j, v);
      }
    };
    // two staged splats per step, back to front: both LDS reads are in
    // flight before the first one is visited; the two visits' gradients go
    // through one LDS exchange and one atomic instruction
    for (int k0 = nh - 1; k0 >= 0; k0 -= 2) {
      const bool two = k0 > 0;
      const int k1 = two ? k0 - 1 : k0;
      const float2 q0 = S.rows[k0][row], q1 = S.rows[k1][row];
      const float4 h0 = S.hdr[k0], h1 = S.hdr[k1];
      const float u0 = q0.y + lxf, u1 = q1.y + lxf;
      const float e0 = fmaf(-h0.x, u0 * u0, q0.x);
      const float e1 = fmaf(-h1.x, u1 * u1, q1.x);
      Terms t0, t1;
      const bool v0 = visit(k0, u0, e0, h0, t0);
      const bool v1 = two && visit(k1, u1, e1, h1, t1);
      if (v0 && v1) {
        row_sums(k0, t0, s_red[row]);
        row_sums(k1, t1, s_red[row] + 12);
        send(k0, k1, true);
      } else if (v0 || v1) {
        const int k = v0 ? k0 : k1;
        row_sums(k, v0 ? t0 : t1, s_red[row]);
        send(k, k, false);
      }
    }
  }
}

template <int TW, int TH>
void raster_fwd(const gs_splat* splats, const uint32_t* values, const uint32_t* ranges,
                const SetK& set, int W, int H, const float* mesh_depth, const float* mesh_rgb,
                float* image, float* T_final, uint32_t* last, uint32_t* n_blend, hipStream_t st) {
#define GS_K(M, C) hipLaunchKernelGGL((k_raster<TW, TH, M, C>), dim3(raster_grid(set, TW, TH, true)), dim3(64), 0, st, splats, values, ranges, set, W, H, mesh_depth, mesh_rgb, image, T_final, last, n_blend)
  if (mesh_depth) {
    if (n_blend) GS_K(true, true); else GS_K(true, false);
  } else {
    if (n_blend) GS_K(false, true); else GS_K(false, false);
  }
#undef GS_K
}

template <int TW, int TH>
void raster_bwd(const gs_splat* splats, const uint32_t* values, const uint32_t* ranges,
                const SetK& set, int W, int H, const float* bg_rgb, const float* T_final,
                const uint32_t* last, const float* dL_dimage, float* grad2d, hipStream_t st) {
  hipLaunchKernelGGL((k_raster_bwd<TW, TH>), dim3(raster_grid(set, TW, TH, false)), dim3(64), 0, st,
                     splats, values, ranges, set, W, H, bg_rgb, T_final, last, dL_dimage, grad2d);
}

// The L1 loss gradient of every view of a batch (blockIdx.y = view):
// dL/dRGBA of L_v = mean over (H, W, 3) of |RGB - target| is
// sign(RGB - target) / (3 H W) for the colour channels and 0 for alpha.
// image and grad hold 4 floats per pixel, target 3, views concatenated.
__global__ __launch_bounds__(kBlock) void k_l1_grad(const ViewK* __restrict__ views,
                                                    const float4* __restrict__ image,
                                                    const float* __restrict__ target,
                                                    float4* __restrict__ grad) {
  const ViewK v = views[blockIdx.y];
  const size_t n = (size_t)v.W * v.H;
  const size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const float d = (float)(3 * n);
  const size_t q = v.pix + p;
  const float4 c = image[q];
  const float* t = target + 3 * q;
  auto sgn = [](float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); };
  grad[q] = make_float4(__fdiv_rn(sgn(c.x - t[0]), d), __fdiv_rn(sgn(c.y - t[1]), d),
                        __fdiv_rn(sgn(c.z - t[2]), d), 0.f);
}

}  // namespace

hipError_t launch_l1_grad(const ViewK* views, int n_views, int max_pixels, const float* image,
                          const float* target, float* grad, hipStream_t st) {
  if (n_views <= 0 || max_pixels <= 0) return hipSuccess;
  trace_mark(st, "l1_grad");
  hipLaunchKernelGGL(k_l1_grad, dim3((max_pixels + kBlock - 1) / kBlock, n_views), dim3(kBlock), 0,
                     st, views, reinterpret_cast<const float4*>(image), target,
                     reinterpret_cast<float4*>(grad));
  return hipGetLastError();
}

int64_t raster_units_grid(const SetK& set, bool forward) {
  return raster_grid(set, set.tile_w, set.tile_h, forward);
}

bool raster_unit_host(const SetK& set, bool forward, const uint32_t* order, int b, int* tile,
                      int* quadrant, int* band) {
  const int tiles = set.tiles_x * set.tiles_y;
  const int nq = (set.tile_w / 8) * (set.tile_h / 8);
  const int ls = forward ? (set.raster_order >> 1) : 0;
  return unit_of(b, tiles, nq, set.raster_order, ls, order, *tile, *quadrant, *band);
}

bool tile_shape_supported(int tw, int th) {
  return (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 16 && th == 16) ||
         (tw == 32 && th == 8) || (tw == 32 && th == 16) || (tw == 32 && th == 32) ||
         (tw == 64 && th == 16) || (tw == 64 && th == 32);
}

hipError_t launch_rasterize(const gs_splat* splats, const uint32_t* values,
                            const uint32_t* ranges, const SetK& set, int W, int H,
                            const float* mesh_depth, const float* mesh_rgb, float* image,
                            float* T_final, uint32_t* last, uint32_t* n_blend, hipStream_t st) {
  const int tw = set.tile_w, th = set.tile_h;
#define GS_RF(A, B) raster_fwd<A, B>(splats, values, ranges, set, W, H, mesh_depth, mesh_rgb, image, T_final, last, n_blend, st)
  if (tw == 8 && th == 8) GS_RF(8, 8);
  else if (tw == 16 && th == 8) GS_RF(16, 8);
  else if (tw == 16 && th == 16) GS_RF(16, 16);
  else if (tw == 32 && th == 8) GS_RF(32, 8);
  else if (tw == 32 && th == 16) GS_RF(32, 16);
  else if (tw == 32 && th == 32) GS_RF(32, 32);
  else if (tw == 64 && th == 16) GS_RF(64, 16);
  else GS_RF(64, 32);
#undef GS_RF
  return hipGetLastError();
}

hipError_t launch_rasterize_backward(const gs_splat* splats, const uint32_t* values,
                                     const uint32_t* ranges, const SetK& set, int W, int H,
                                     const float* bg_rgb, const float* T_final,
                                     const uint32_t* last, const float* dL_dimage, float* grad2d,
                                     hipStream_t st) {
  const int tw = set.tile_w, th = set.tile_h;
#define GS_RB(A, B) raster_bwd<A, B>(splats, values, ranges, set, W, H, bg_rgb, T_final, last, dL_dimage, grad2d, st)
  if (tw == 8 && th == 8) GS_RB(8, 8);
  else if (tw == 16 && th == 8) GS_RB(16, 8);
  else if (tw == 16 && th == 16) GS_RB(16, 16);
  else if (tw == 32 && th == 8) GS_RB(32, 8);
  else if (tw == 32 && th == 16) GS_RB(32, 16);
  else if (tw == 32 && th == 32) GS_RB(32, 32);
  else if (tw == 64 && th == 16) GS_RB(64, 16);
  else GS_RB(64, 32);
#undef GS_RB
  return hipGetLastError();
}

}  // namespace gs
