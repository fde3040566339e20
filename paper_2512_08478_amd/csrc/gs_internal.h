// Internal declarations shared by the libgs translation units (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gs.h"

namespace gs {

constexpr int kBlock = 256;          // threads per block for streaming kernels
constexpr int kViewsPerBlock = 16;   // views a batch preprocess workgroup projects in turn
constexpr int kSortItems = 16;       // keys per thread in a radix pass
constexpr int kSortPart = kBlock * kSortItems;  // keys per partition (4096)
constexpr int kMaxPassTotal = 32;    // radix passes per call (depth + tile, or 64-bit)

constexpr uint32_t kLbFlagAgg = 1u << 30;   // look-back: partition count published
constexpr uint32_t kLbFlagInc = 2u << 30;   // look-back: inclusive prefix published
constexpr uint32_t kLbValue = (1u << 30) - 1;

// Camera and settings as kernels see them (by value, in kernarg memory).
struct CamK {
  float V[12];        // world->camera rows 0..2 (3x4)
  float T3[9];        // (view rotation) x (model linear part): maps an
                      // asset-local direction into camera space
  float Rk[9];        // model rotation (model linear part / its scale)
  float A[12];        // model transform [s R | t]
  float campos[3];    // camera centre in world coordinates
  float fx, fy, cx, cy;
  float limx, limy;   // clip * half-FoV tangents
  float znear;
  int W, H;
  int has_model;
  int tile_row;       // first tile row of this view in a batch's tile grid (0: one view)
};

// Cameras (as seen by one asset) and 2-D gradient records of up to
// kBwdViews views, for the multi-view preprocess backward.
constexpr int kBwdViews = 8;
struct ViewsK {
  CamK cam[kBwdViews];
  const float* g2d[kBwdViews];
  int nv;
};

// The asset table of a batched preprocess (kernel argument): asset a's
// Gaussians are [offset[a], offset[a] + count[a]) of each view's n, and its
// workgroups are blocks [block0[a], block0[a + 1]).
constexpr int kMaxAssetsK = 64;
struct BatchPreK {
  int64_t n;
  int n_assets;
  int block0[kMaxAssetsK + 1];
  int64_t offset[kMaxAssetsK];
  int count[kMaxAssetsK];
};

// One view of a batch: its band of tile rows [row, row + tiles_y) in the
// batch's tile grid (columns 0 .. tiles_x-1 of the grid's width), its size
// and the offset of its pixels in the batch's per-pixel arrays.
struct ViewK {
  int row, tiles_x, tiles_y, W, H, pad;
  size_t pix;
};

struct SetK {
  int tile_w, tile_h, tiles_x, tiles_y;
  int tile_w_shift, tile_h_shift;  // log2 of the tile shape (every supported one is a power of 2)
  int raster_order;   // 0: spatial runs over the XCDs; 1: heavy tiles first
  float eps2d, tau, log2_tau, amax, t_eps;
  float bg[3];
  // a batch of views (n_views > 0): tiles_x/tiles_y are the batch grid's,
  // views[] (device) maps each band of tile rows to its view
  const ViewK* views;
  int n_views;
};

// Workspace carve-up helpers.
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// gs_sort workspace: depth ping-pong (u32 keys/values, n each), tile
// ping-pong and final tile keys (u32, capacity each), onesweep histograms,
// tickets and look-back words (two buffers), the reduce-then-scan count
// table and digit totals, keygen slice counts, the kept instance count.
struct SortLayout {
  size_t dk[2], dv[2], drect, tk[2], tv[2], tkf, hist, tickets, lookback, table, totals, kg_counts,
      count, tcls, tseg;
  size_t bytes;
  int parts;     // 4096-key partitions of the largest sort
  int rs_parts;  // 1024-key partitions of the largest sort (reduce-then-scan table rows)
  int kg_parts;  // keygen slices
};
SortLayout sort_layout(int64_t n, int64_t capacity, int tiles);
// Tile classes for the heavy-first compositing order: class k holds the
// tiles with floor(log2(list length + 1)) = kTileClasses - 1 - k (the last
// class also every shorter list).
constexpr int kTileClasses = 16;
// Up to this many tiles, one workgroup writes the heavy-first order (one
// launch instead of the class and order kernels).
constexpr int kFusedOrderTiles = 8192;
SortLayout pairs_layout(int64_t n);  // gs_sort_pairs: dk[0]/dv[0] are the u64/u32 alternates

// One stable LSD radix sort of (key, value) pairs.
// The sort's set-up: tile ranges, tickets and class counts cleared, and
// the instance count (counts[0] capped at the capacity) and status flag
// written.  Done by k_sort_init, or in sort mode 0 by the first depth
// pass's count kernel (`active`), which saves a launch.
struct SortInitK {
  uint32_t* ranges;
  int ranges_len;
  uint32_t* tickets;
  int ntickets;
  uint32_t* cls_count;
  uint32_t* count;
  const uint32_t* total_src;
  uint32_t host_total;
  int64_t capacity;
  uint32_t* status_flag;
  int depth_bits;
  int active;
};

template <typename KeyT>
struct RadixArgs {
  int mode;                 // 0 reduce-then-scan, 1 onesweep (decoupled look-back)
  int64_t n_grid;           // upper bound of n: sizes the grids
  const uint32_t* count;    // device n (NULL: n = n_grid)
  int drop_first;           // the first pass drops all-ones keys ...
  const uint32_t* count_rest;  // ... and the later passes sort *count_rest pairs
  const uint32_t* kbase;    // the first pass orders and writes key - *kbase (NULL: key)
  const KeyT* kin;          // input keys (not modified)
  const uint32_t* vin;      // input values (NULL: value = position)
  KeyT* k_alt;              // ping-pong buffers
  uint32_t* v_alt;
  KeyT* k_out;              // the result
  uint32_t* v_out;
  uint32_t* table;          // mode 0: partitions x 2^bits counts (partition-major)
  uint32_t* totals;         // mode 0: 256 digit totals
  uint32_t* hist;           // mode 1: 256 bins per pass
  uint32_t* tickets;        // mode 1: one per pass
  uint32_t* lookback;       // mode 1: two buffers of lb_parts x 256 words
  int lb_parts;
  SortInitK init;           // mode 0: the set-up, done by the first pass's count kernel
  int min_parts;            // mode 0: partitions each pass aims for (0: the default)
};
// The tile passes (after key generation) aim for more partitions than the
// depth passes: on the 1M frame 8 keys per thread instead of 16 (1,685
// partitions) made the tile pass 4 us faster, while 4 instead of 8 made
// the depth passes 5 us slower.
constexpr int kTilePassMinParts = 1024;

// Launchers (enqueue only; return the first launch error).
constexpr int kMaxAssets = 64;       // assets per preprocess / backward call
size_t preprocess_ws_bytes(int64_t n);
int preprocess_blocks(int64_t n);
// Projection of n Gaussians; per-block (instances, visible, smallest and
// largest visible depth key) partials go to partial[0 .. preprocess_blocks(n)).
// Every view x asset of a batch in one launch (k_preprocess_views); cams
// (device) holds n_views * n_assets cameras, view-major.  Partials: n_views *
// B.block0[n_assets] slots.
hipError_t launch_preprocess_views(const BatchPreK& B, int n_views, const float* means,
                                   const float* log_scales, const float* quats,
                                   const float* logits, const float* sh, int degree,
                                   const CamK* cams, const SetK& set, gs_splat* splats,
                                   uint32_t* depth_keys, uint32_t* tile_rects, uint4* partial,
                                   hipStream_t st);
hipError_t launch_preprocess(int n, const float* means, const float* log_scales,
                             const float* quats, const float* logits, const float* sh,
                             int degree, const CamK& cam, const SetK& set,
                             gs_splat* splats, uint32_t* depth_keys, uint32_t* tile_rects,
                             uint4* partial, hipStream_t st);
// FP16 pre-pack (binary16 posop n*4, cov n*6, sh16 n*packed_sh_stride) and
// the projection that reads it; same outputs as launch_preprocess.
int packed_sh_stride(int degree);
hipError_t launch_prepack(int n, const float* means, const float* log_scales, const float* quats,
                          const float* logits, const float* sh, int degree, uint16_t* posop,
                          uint16_t* cov, uint16_t* sh16, hipStream_t st);
// Linear blend skinning: packed canonical (posop, cov) -> deformed, with
// 4 joint influences per Gaussian (u8 indices, f32 weights) and up to 256
// 3x4 joint transforms.
hipError_t launch_lbs(int n, const uint16_t* canon_posop, const uint16_t* canon_cov,
                      const uint8_t* joint_idx, const float* joint_w, int n_joints,
                      const float* joints, uint16_t* posop, uint16_t* cov, hipStream_t st);
hipError_t launch_preprocess_packed(int n, const uint16_t* posop, const uint16_t* cov,
                                    const uint16_t* sh16, int degree, const CamK& cam,
                                    const SetK& set, gs_splat* splats, uint32_t* depth_keys,
                                    uint32_t* tile_rects, uint4* partial, hipStream_t st);
// counts[0] = sum of partial[].x (instances), counts[1] = sum of partial[].y
// (visible), counts[2] = min of partial[].z, counts[3] = max of partial[].w
// (the visible depth key range)
hipError_t launch_count_finalize(const uint4* partial, int blocks, uint32_t* counts,
                                 hipStream_t st);
// total_src (device counts of gs_preprocess, or NULL: host_total) gives the
// instance count; with depth_bits in 1..31 bit 1 of status_flag reports a
// visible depth key range that does not fit in depth_bits.
hipError_t launch_sort_init(const SortLayout& L, char* ws, int mode, uint32_t* tile_ranges,
                            int tiles, uint32_t* status_flag, const uint32_t* total_src,
                            int64_t capacity, hipStream_t st, uint32_t* cls_count = nullptr,
                            int depth_bits = 0);
// The same set-up (sort mode 0) as arguments for the first depth pass.
SortInitK sort_init_args(const SortLayout& L, char* ws, uint32_t* tile_ranges, int tiles,
                         uint32_t* status_flag, const uint32_t* total_src, int64_t capacity,
                         uint32_t* cls_count, int depth_bits);
// Passes first_pass .. passes-1 (digit p at shift p * bits); the pass that
// would have come before first_pass has left its output in kin/vin.
template <typename KeyT>
hipError_t launch_radix_sort(const RadixArgs<KeyT>& a, int bits, int passes, int pass_base,
                             bool last_keys, const char* label, hipStream_t st,
                             int first_pass = 0);
// Instances of the depth-sorted visible Gaussians: gathers their tile rects
// (rects -> sorted_rects, depth order), counts tiles per slice, scans the
// slices and writes (tile, Gaussian) pairs in depth order.
hipError_t launch_keygen(int64_t n, const uint32_t* sorted_idx, const uint32_t* vis_count,
                         const uint2* rects, uint2* sorted_rects, int tiles_x,
                         const uint32_t* inst_count, uint32_t* kg_counts, uint32_t* kg_total,
                         uint32_t* tkeys, uint32_t* tvals, hipStream_t st);
// A reduce-then-scan sort (mode 0) of u32 keys whose pass p takes widths[p]
// (6..9) bits, the shifts adding up from bit 0.
hipError_t launch_radix_sort_widths(const RadixArgs<uint32_t>& a, const int* widths, int passes,
                                    bool last_keys, const char* label, hipStream_t st);
// Key generation fused with the first tile-digit pass (reduce-then-scan
// mode): the first-digit histogram of each slice (with the rect gather),
// its column scan into table/totals, and the instances written in the
// order of that pass to tkeys/tvals.
hipError_t launch_keygen_fused(int64_t n, int bits, const uint32_t* sorted_idx,
                               const uint32_t* vis_count, const uint2* rects,
                               uint2* sorted_rects, int tiles_x, const uint32_t* inst_count,
                               uint32_t* table, uint32_t* totals, uint32_t* tkeys,
                               uint32_t* tvals, hipStream_t st);
// Host mirror of the compositing kernels' work split (the same function
// the kernels run): their grid, and the (tile, quadrant, band) workgroup b
// takes (false for a padding workgroup); `order` is the heavy-first tile
// order when raster_order bit 0 is set.
int64_t raster_units_grid(const SetK& set, bool forward);
bool raster_unit_host(const SetK& set, bool forward, const uint32_t* order, int b, int* tile,
                      int* quadrant, int* band);
hipError_t launch_tile_ranges(int64_t capacity, const uint32_t* count, const uint32_t* tkeys,
                              uint32_t* ranges, hipStream_t st);
// ranges[2*tiles .. 3*tiles) = the tiles, longest lists first (class
// counters zeroed by launch_sort_init).
hipError_t launch_tile_order(uint32_t* ranges, int tiles, uint32_t* cls_count, uint32_t* seg,
                             hipStream_t st);
hipError_t launch_compose_keys(int64_t capacity, const uint32_t* count, const uint32_t* tkeys,
                               const uint32_t* values, const gs_splat* splats, uint64_t* keys,
                               hipStream_t st);
// mesh_depth (H*W, camera-space z; NULL: no mesh) hides deeper splats;
// mesh_rgb / bg_rgb (H*W*3; NULL: the settings' background) is the colour
// behind the Gaussians.
hipError_t launch_rasterize(const gs_splat* splats, const uint32_t* values,
                            const uint32_t* ranges, const SetK& set, int W, int H,
                            const float* mesh_depth, const float* mesh_rgb, float* image,
                            float* T_final, uint32_t* last, uint32_t* n_blend, hipStream_t st);
hipError_t launch_rasterize_backward(const gs_splat* splats, const uint32_t* values,
                                     const uint32_t* ranges, const SetK& set, int W, int H,
                                     const float* bg_rgb, const float* T_final,
                                     const uint32_t* last, const float* dL_dimage, float* grad2d,
                                     hipStream_t st);
hipError_t launch_preprocess_backward(int n, const float* means, const float* log_scales,
                                      const float* quats, const float* logits, const float* sh,
                                      int degree, const CamK& cam, const SetK& set,
                                      const gs_splat* splats, const float* grad2d,
                                      float* d_means, float* d_log_scales, float* d_quats,
                                      float* d_logits, float* d_sh, int accumulate,
                                      hipStream_t st);
hipError_t launch_preprocess_backward_views(int n, const float* means, const float* log_scales,
                                            const float* quats, const float* logits,
                                            const float* sh, int degree, const ViewsK& views,
                                            const SetK& set, float* d_means, float* d_log_scales,
                                            float* d_quats, float* d_logits, float* d_sh,
                                            int accumulate, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t st);
// L1 loss gradient of every view of a batch (views: device table; image and
// grad 4 floats per pixel, target 3, views concatenated).
hipError_t launch_l1_grad(const ViewK* views, int n_views, int max_pixels, const float* image,
                          const float* target, float* grad, hipStream_t st);

// Opt-in kernel tracer: when enabled, trace_mark records a HIP event on the
// stream; the interval from one mark to the next is attributed to the
// first mark's label (an empty label closes the interval).
void trace_mark(hipStream_t st, const char* label);

// Per-Gaussian 2-D gradient record written by the raster backward:
// d(mean_x, mean_y, qa, qb, qc, opacity, r, g, b), padded to 12 floats.
constexpr int kGrad2dStride = 12;

}  // namespace gs
