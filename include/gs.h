/*
 * gs.h -- C ABI of libgs, a gfx950 (MI355X) implementation of the per-frame
 * 3D Gaussian Splatting render path.
 *
 * The method follows "Visionary" (arXiv 2512.08478): the 3DGS definition of
 * Section 3.2 (Eq. 1 projection, Eq. 2 pixel weight, Eq. 3 front-to-back
 * compositing over depth-sorted Gaussians) and the per-frame GPU pipeline of
 * Algorithm 1 / Section 3.4 (per-model preprocess with frustum and opacity
 * culls, a GPU radix sort, then the splat draw).  This library sorts
 * (tile, depth) keys and composites front to back per pixel in a compute
 * kernel instead of drawing depth-sorted quads; the sum is the same Eq. 3.
 *
 * Conventions for every entry point
 *   - All array arguments are DEVICE pointers owned by the caller, row-major
 *     and contiguous, float32 unless noted, with base addresses aligned to
 *     16 bytes.  The library never allocates device memory and never
 *     synchronises the stream, except where a function says so.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  All
 *     work is enqueued on it, in order.
 *   - Structs (gs_camera, gs_settings, model transforms) are HOST pointers,
 *     read during the call.
 *   - Every function returns a gs_status.  Argument checks run before any
 *     HIP call, so a rejected call has no effect on the device.  On
 *     GS_ERR_HIP the HIP error code is kept per thread (gs_last_hip_error).
 *   - n == 0 (no Gaussians) is valid and renders the background.
 *   - Calls that share a workspace must not overlap in time.
 */
#ifndef GS_H_
#define GS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gs_status {
  GS_OK = 0,
  GS_ERR_INVALID_ARGUMENT = 1, /* null pointer, negative size, bad struct field */
  GS_ERR_UNSUPPORTED = 2,      /* SH degree > 3, tile shape, digit width */
  GS_ERR_CAPACITY = 3,         /* more (Gaussian, tile) instances than capacity */
  GS_ERR_HIP = 4,              /* a HIP runtime call failed; see gs_last_hip_error */
  GS_ERR_MISALIGNED = 5,       /* a device pointer is not 16-byte aligned */
  GS_ERR_WORKSPACE = 6         /* workspace smaller than gs_workspace_size() */
} gs_status;

/*
 * Pinhole camera (Eq. 1's projection operator; Algorithm 1's (V, P)).
 * viewmat: row-major 4x4 world->camera matrix, OpenCV axes (+x right,
 * +y down, +z forward); its upper 3x3 must be a rotation.  A camera-space
 * point t maps to pixel coordinates (fx*t.x/t.z + cx, fy*t.y/t.z + cy);
 * pixel (i, j) samples the point (i + 1/2, j + 1/2).  Gaussians with
 * camera-space depth <= znear are culled.
 */
typedef struct gs_camera {
  float viewmat[16];
  float fx, fy, cx, cy;
  int32_t width, height;
  float znear;
  float reserved;
} gs_camera;

/*
 * Constants the paper leaves open, with the defaults gs_default_settings()
 * fills in:
 *   tile_w x tile_h   8x8, 16x8, 16x16 (default), 32x8, 32x16, 32x32, 64x16
 *                    or 64x32 pixels
 *   eps2d      0.3   px^2 added to the diagonal of the 2-D covariance S
 *   alpha_min  1/255 opacity cull (Algorithm 1) and per-pixel skip
 *   alpha_max  0.99  clamp of the pixel weight of Eq. 2
 *   t_eps      1e-4  compositing blends a Gaussian, then stops once the
 *                    transmittance is below t_eps
 *   clip       1.3   x/z, y/z inside the Jacobian J are clamped to clip
 *                    times the half-FoV tangent
 *   bg         (0,0,0) background colour; output alpha is 1 - T_final
 *   radix_bits 8     digit width of the radix sort (6, 7 or 8)
 *   sort_mode  0     0: reduce-then-scan radix passes (count, scan, scatter
 *                    kernels; no workgroup waits on another); 1: onesweep
 *                    passes with decoupled look-back between workgroups.
 *                    Both give the same (unique) stable result.
 *   raster_order 1   how the compositing kernels take the tiles (0..5).
 *                    Bit 0 clear: runs of neighbouring tiles dealt to the
 *                    GPU's XCDs in turn; set: tiles with the longest splat
 *                    lists first (gs_sort then also writes that order).
 *                    raster_order >> 1 = s (0, 1 or 2; forward compositing
 *                    only): each 8x8 pixel quadrant is taken as 2^s bands
 *                    of 8 / 2^s rows, each by its own wave, which shortens
 *                    the frame's tail when a few tiles hold very long
 *                    lists.  gs_sort and the compositing calls of a frame
 *                    must use the same value.  Images do not depend on it.
 *   depth_bits 0     how many bits of the depth keys gs_sort orders.  0:
 *                    all 32 bits, in radix_bits-wide passes.  1..32: the
 *                    keys relative to the smallest visible key (counts[2]
 *                    of gs_preprocess), in ceil(depth_bits / 9) passes of
 *                    at most 9 bits in sort mode 0 (radix_bits-wide passes
 *                    in mode 1).  The caller takes it from the bit length
 *                    of counts[3] - counts[2] (the same frame, or a
 *                    previous one with headroom); if the frame's range does
 *                    not fit, gs_sort sets bit 1 of status_flag, the order
 *                    is not valid, and the caller sorts again with more
 *                    bits.  The order, when valid, does not depend on it.
 */
typedef struct gs_settings {
  int32_t tile_w, tile_h;
  float eps2d;
  float alpha_min;
  float alpha_max;
  float t_eps;
  float clip;
  float bg[3];
  int32_t radix_bits;
  int32_t sort_mode;
  int32_t raster_order;
  int32_t depth_bits;
} gs_settings;

/*
 * Projected splat: the per-Gaussian record written by gs_preprocess
 * (Algorithm 1's `points2d` entry), 48 bytes.  The 2-D quadratic form of
 * Eq. 2 is stored in a whitened form:
 *     Q(dx, dy) = (dx, dy) S^-1 (dx, dy)^T = qa * (dx - qb*dy)^2 + qc * dy^2
 * with S = [[a, b], [b, c]], qa = c/det S, qb = b/c, qc = 1/c.  Both terms
 * are non-negative, so Q is evaluated without cancellation.
 * Pixel bbox [px0..px1] x [py0..py1] is inclusive: the pixels whose
 * centres the opacity-aware footprint (o exp(-Q/2) >= alpha_min) can reach,
 * rounded outwards; a culled Gaussian has px1 < px0 and reaches no pixel.
 * Its tiles are the tiles this bbox overlaps (gs_preprocess's tile_rects).
 * The 2-D mean (Eq. 1's projected mean, in pixels) is stored relative to
 * the bbox corner: the mean is (px0 + mean_x, py0 + mean_y).  It is formed
 * in float64, so a pixel's offset from it is accurate to ~1e-7 px anywhere
 * in the image.  `depth` is the float32 rounding of the camera-space depth
 * (formed in float64).
 */
typedef struct gs_splat {
  float mean_x, mean_y;
  float qa, qb;
  float qc, opacity;
  float r, g, b;
  float depth;
  uint16_t px0, py0, px1, py1;
} gs_splat;

/* Workspace stages for gs_workspace_size. */
typedef enum gs_stage {
  GS_STAGE_PREPROCESS = 0,
  GS_STAGE_SORT = 1,
  GS_STAGE_SORT_PAIRS = 2,
  GS_STAGE_BACKWARD = 3
} gs_stage;

const char* gs_version(void);
const char* gs_status_string(int32_t status);
/* hipError_t of the last GS_ERR_HIP on this thread (0 if none). */
int32_t gs_last_hip_error(void);
/* Fill *s with the defaults listed above. */
void gs_default_settings(gs_settings* s);

/*
 * Opt-in kernel tracer (for profiling; not thread-safe).  gs_trace_enable(1)
 * creates a pool of HIP events on first use and starts recording one event
 * before each kernel the library launches and one after the last; 0 stops.
 * gs_trace_read waits for the last recorded event, then writes up to
 * max_entries (label, milliseconds) pairs -- labels are 32-byte
 * NUL-terminated strings in `labels` -- sets *count and clears the record.
 * Each interval runs from a kernel's launch point in the stream to the
 * next, so it covers that kernel and any gap before the next one.
 */
int32_t gs_trace_enable(int32_t on);
int32_t gs_trace_read(int32_t max_entries, char* labels, float* ms, int32_t* count);

/*
 * Bytes of workspace a stage needs.  `n` is the number of Gaussians,
 * `capacity` the instance capacity (for the sort stages; for
 * GS_STAGE_SORT_PAIRS the number of pairs).  Returns 0 on invalid input.
 */
size_t gs_workspace_size(int32_t stage, int64_t n, int64_t capacity,
                         const gs_camera* cam, const gs_settings* set);

/*
 * Significant key bits of gs_sort for this camera and settings: 32 depth
 * bits plus ceil(log2(tiles)) tile bits.  The sort makes
 * ceil(32 / radix_bits) depth passes and ceil(tile bits / radix_bits)
 * tile passes.
 */
int32_t gs_sort_key_bits(const gs_camera* cam, const gs_settings* set);

/*
 * gs_preprocess -- per-Gaussian projection (Section 3.2, Eq. 1) and colour,
 * with the culls of Algorithm 1's Preprocess procedure.
 *
 * Inputs (raw parameters, device, float32):
 *   means[n*3], log_scales[n*3] (scale = exp), quats[n*4] as (w, x, y, z)
 *   (normalised here; a zero quaternion is culled), opacity_logits[n]
 *   (opacity = sigmoid), sh[n*K*3] with K = (sh_degree+1)^2, coefficient-
 *   major with RGB innermost; sh_degree in 0..3.
 *   model: host pointer to a 3x4 row-major similarity transform [s*R | t]
 *   placing this asset in the world (Algorithm 1's per-model M_k), or NULL
 *   for the identity.  Covariances become (sR) Sigma (sR)^T and the SH
 *   view direction is taken in the asset's own frame (R^T d).
 * Outputs (device):
 *   splats[n]       one gs_splat per Gaussian (culled ones have an empty rect).
 *   depth_keys[n]   u32 depth sort key per Gaussian: the float32 bits of its
 *                   camera-space depth (Algorithm 1's `depths`), or
 *                   0xFFFFFFFF when culled, so culled Gaussians sort last.
 *   tile_rects[2n]  u32 pair per Gaussian: the tile rect of its record,
 *                   (tx0 | ty0 << 16, tx1 | ty1 << 16), packed densely so
 *                   that key generation gathers 8 bytes per Gaussian.
 *   counts[4]       u32: counts[0] = (Gaussian, tile) instances in total,
 *                   counts[1] = visible Gaussians, counts[2] and counts[3]
 *                   = the smallest and the largest depth key of a visible
 *                   Gaussian (0xFFFFFFFF and 0 when none is visible); the
 *                   host may read the range back to plan depth_bits.
 * Culled (record with an empty rect, zero tiles): camera depth <= znear,
 * opacity < alpha_min, non-finite values, zero quaternion, or a footprint
 * whose opacity-aware bounding box (where o*exp(-Q/2) >= alpha_min)
 * contains no pixel centre.
 * Workspace: gs_workspace_size(GS_STAGE_PREPROCESS, n, 0, ...) bytes
 * (per-workgroup partial counts).
 */
int32_t gs_preprocess(int64_t n, const float* means, const float* log_scales,
                      const float* quats, const float* opacity_logits,
                      const float* sh, int32_t sh_degree, const float* model,
                      const gs_camera* cam, const gs_settings* set,
                      gs_splat* splats, uint32_t* depth_keys, uint32_t* tile_rects,
                      uint32_t* counts, void* workspace, size_t workspace_bytes,
                      void* stream);

/*
 * gs_preprocess_noalloc -- gs_preprocess without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same inputs,
 * outputs and results as gs_preprocess (bit for bit).  Its per-workgroup
 * partial counts live in a 1 MiB array inside the library, one copy per GPU,
 * kept until the process ends; each call writes every slot it reads, so no
 * clearing is needed.  The call allocates nothing (no hipMalloc, no library
 * allocation).  n may be at most gs_preprocess_noalloc_max_n() (16,760,832);
 * larger n returns GS_ERR_WORKSPACE before any HIP call.  Calls that overlap
 * in time on one GPU (other streams, other host threads) share that array
 * and race: serialise them.  The first call on a device looks up its copy's
 * address once (hipGetSymbolAddress with that device current).
 */
int32_t gs_preprocess_noalloc(int64_t n, const float* means, const float* log_scales,
                              const float* quats, const float* opacity_logits, const float* sh,
                              int32_t sh_degree, const float* model, const gs_camera* cam,
                              const gs_settings* set, gs_splat* splats, uint32_t* depth_keys,
                              uint32_t* tile_rects, uint32_t* counts, void* stream);
/* Largest n gs_preprocess_noalloc accepts. */
int64_t gs_preprocess_noalloc_max_n(void);

/*
 * One asset of a multi-asset scene (Algorithm 1 loops over models, each with
 * its own model matrix M_k, and feeds all of them to one global sort).  The
 * assets' Gaussians are concatenated in the parameter arrays: asset a owns
 * indices [offset, offset + count).  model: HOST pointer to the asset's 3x4
 * row-major similarity transform, or NULL for the identity.
 */
typedef struct gs_asset {
  int64_t offset;
  int64_t count;
  const float* model;
} gs_asset;

/*
 * gs_preprocess_assets -- gs_preprocess over n_assets assets (1 to 64) whose
 * Gaussians are concatenated (assets[0].offset = 0, each asset starts where
 * the previous one ends, the counts sum to n; otherwise
 * GS_ERR_INVALID_ARGUMENT).  Record i, depth_keys[i] and the sort values
 * refer to the global index i, so one gs_sort / gs_rasterize call renders
 * every asset with a single global depth order.  counts[] sums over all
 * assets.  Same workspace as gs_preprocess for n Gaussians.  Each asset is
 * one kernel launch; assets with count 0 launch nothing.
 */
int32_t gs_preprocess_assets(int32_t n_assets, const gs_asset* assets, int64_t n,
                             const float* means, const float* log_scales,
                             const float* quats, const float* opacity_logits,
                             const float* sh, int32_t sh_degree, const gs_camera* cam,
                             const gs_settings* set, gs_splat* splats,
                             uint32_t* depth_keys, uint32_t* tile_rects, uint32_t* counts,
                             void* workspace, size_t workspace_bytes, void* stream);

/*
 * FP16 pre-pack (Algorithm 1's Pre-pack step; Section 3.4): scale and
 * rotation become the covariance Sigma = R diag(s^2) R^T, and the mean,
 * activated opacity, upper triangle of Sigma and SH coefficients are stored
 * as IEEE binary16, two to a 32-bit word.  Layout (device, little-endian
 * halves, n Gaussians):
 *   posop[n*4]  (mu_x, mu_y, mu_z, alpha), alpha = sigmoid(logit)
 *   cov[n*6]    (xx, xy, xz, yy, yz, zz) of Sigma
 *   sh16[n*S]   the K*3 SH coefficients in the raw order (coefficient-major,
 *               RGB innermost), zero-padded to S = gs_packed_sh_stride()
 * gs_packed_sh_stride returns S for sh_degree 0..3 (4, 12, 28, 48), -1
 * otherwise.
 */
int32_t gs_packed_sh_stride(int32_t sh_degree);

/*
 * gs_prepack -- converts n raw Gaussians (the inputs of gs_preprocess) to
 * the layout above; run once per asset.  Opacity and covariance are
 * computed in float64 and rounded once to the nearest binary16 (ties to
 * even); means and SH are rounded from float32 directly.  Values beyond
 * the binary16 range become infinities, and gs_preprocess_packed culls
 * such Gaussians.  The outputs must not overlap the inputs.
 */
int32_t gs_prepack(int64_t n, const float* means, const float* log_scales, const float* quats,
                   const float* opacity_logits, const float* sh, int32_t sh_degree,
                   uint16_t* posop, uint16_t* cov, uint16_t* sh16, void* stream);

/*
 * gs_lbs_deform -- the avatar pre-decoder (Section 3.3, Eqs. 5-6): linear
 * blend skinning of n pre-packed canonical Gaussians.  Per Gaussian i,
 *   T_i = sum_k w_ik M_{j_ik} = [R_i | t_i]   (k = 0..3),
 *   mu_i = R_i mu^_i + t_i,   Sigma_i = R_i Sigma^_i R_i^T.
 * canon_posop[n*4], canon_cov[n*6]: the canonical Gaussians in the
 * gs_prepack layout (binary16).  joint_idx[n*4] (u8) and joint_w[n*4]
 * (float32): four joint influences per Gaussian (weight 0 for unused
 * slots).  joints[n_joints*12]: device float32 3x4 row-major joint
 * transforms M_k, n_joints in 1..256; an index >= n_joints contributes
 * nothing.  Writes posop[n*4] (deformed mean, opacity copied) and
 * cov[n*6], computed in float64 from the decoded canonical values and
 * rounded once to binary16 (the identity pose reproduces the input bits);
 * outputs must not alias the canonical inputs.  SH pass through unchanged:
 * render the result with gs_preprocess_packed and the canonical sh16.
 */
int32_t gs_lbs_deform(int64_t n, const uint16_t* canon_posop, const uint16_t* canon_cov,
                      const uint8_t* joint_idx, const float* joint_w, int32_t n_joints,
                      const float* joints, uint16_t* posop, uint16_t* cov, void* stream);

/*
 * gs_preprocess_packed -- gs_preprocess_assets from the pre-packed layout:
 * the same culls, records, depth keys, tile rects and counts, computed from
 * the binary16 mean, opacity, covariance and SH (exactly as decoded).  The
 * 2-D covariance J W Sigma W^T J^T and its determinant are formed in
 * float64.  Asset offsets index Gaussians (posop + 4*offset, cov +
 * 6*offset, sh16 + S*offset).  Forward only: the packed form has no
 * backward.  Same workspace as gs_preprocess for n Gaussians.
 */
int32_t gs_preprocess_packed(int32_t n_assets, const gs_asset* assets, int64_t n,
                             const uint16_t* posop, const uint16_t* cov, const uint16_t* sh16,
                             int32_t sh_degree, const gs_camera* cam, const gs_settings* set,
                             gs_splat* splats, uint32_t* depth_keys, uint32_t* tile_rects,
                             uint32_t* counts, void* workspace, size_t workspace_bytes,
                             void* stream);

/*
 * gs_sort -- key generation and the per-frame GPU radix sort (Algorithm 1,
 * Radix Sort; Section 3.4).  The sort order is that of the 64-bit keys
 *     key = tile_id << 32 | bits(float32 depth)
 * taken for each visible Gaussian in index order and each tile of its rect
 * in row-major order, sorted by a stable LSD radix sort: equal keys stay in
 * Gaussian-index order, so the permutation is unique.  Depth is camera-space
 * z, which orders like the paper's NDC z for z > 0.  The LSD passes over the
 * 32 depth bits run on the Gaussians before they are expanded into
 * (Gaussian, tile) instances (every instance of a Gaussian has the same
 * depth, so the order is the same); the passes over the tile bits run on
 * the instances.  Sorting all n depth keys keeps equal depths in index
 * order, which replaces Algorithm 1's nondeterministic atomic append.
 *
 * Reads splats[n], depth_keys[n], tile_rects[2n] and counts (device, from
 * gs_preprocess).  Writes values[capacity] (u32 Gaussian index per sorted
 * instance), tile_ranges[3*tiles] (u32: first the [start, end) of each
 * tile in the sorted list, tiles = ceil(W/tile_w) * ceil(H/tile_h),
 * row-major; then, with raster_order 1 or 3, the tiles in the order the
 * compositing kernels take them: by decreasing floor(log2(list length + 1)),
 * in an unspecified order within a class) and, if
 * `keys` is not NULL, keys[capacity] (the sorted u64 keys above).  Only the
 * first counts[0] entries are meaningful.
 *
 * Counts are read on the device; there is no host sync.  When counts[0] >
 * capacity, `status_flag[0]` (device u32, may be NULL) gets bit 0 set and
 * the output is not a valid instance list: some `capacity` instances are
 * kept (sort_mode 1: the first ones in depth order; sort_mode 0: those the
 * first tile-digit pass places below `capacity`, i.e. whole groups of
 * tiles), and the caller retries with a larger capacity after checking the
 * flag (or uses gs_sort_checked).  Bit 1 reports a depth key range wider
 * than settings.depth_bits (see gs_settings).
 * Workspace: gs_workspace_size(GS_STAGE_SORT, n, capacity, cam, set).
 */
int32_t gs_sort(int64_t n, const gs_splat* splats, const uint32_t* depth_keys,
                const uint32_t* tile_rects, const uint32_t* counts, const gs_camera* cam,
                const gs_settings* set, int64_t capacity,
                uint64_t* keys, uint32_t* values, uint32_t* tile_ranges,
                uint32_t* status_flag, void* workspace, size_t workspace_bytes,
                void* stream);

/*
 * gs_sort_checked -- gs_sort for callers that size the instance buffers per
 * frame (Algorithm 1 reads the instance count before sorting): waits for
 * `stream`, reads counts[0] back, stores it in *required (host, may be
 * NULL), and returns GS_ERR_CAPACITY without sorting when it exceeds
 * `capacity`; otherwise runs gs_sort with the same arguments (same
 * validation and errors).  One host sync per call.
 */
int32_t gs_sort_checked(int64_t n, const gs_splat* splats, const uint32_t* depth_keys,
                        const uint32_t* tile_rects, const uint32_t* counts,
                        const gs_camera* cam, const gs_settings* set, int64_t capacity,
                        uint64_t* keys, uint32_t* values, uint32_t* tile_ranges,
                        uint32_t* status_flag, void* workspace, size_t workspace_bytes,
                        int64_t* required, void* stream);

/*
 * gs_sort_plan -- host-only description of the radix passes gs_sort makes
 * for n Gaussians, `capacity` instances, this camera and these settings
 * (no HIP call; for tests and tools).  passes[0 .. *n_passes) in launch
 * order: the depth passes, then the tile passes (in sort mode 0 key
 * generation performs the first tile pass itself).  Each pass: its index
 * (also the parity of the look-back words it reads in mode 1: half
 * pass % 2), digit width, which count bounds its keys (GS_PASS_KEYS_ALL:
 * n; _VISIBLE: counts[1]; _INSTANCES: counts[0], at most capacity), and in
 * mode 1 the keys per partition and the partitions its grid launches (its
 * workgroups take partitions 0 .. grid_partitions-1 by ticket; a partition
 * holds keys when its first key index is below the pass's key count).
 * *lookback_words is the mode-1 look-back buffer (two halves), 0 in mode 0.
 * A mode-1 pass reads words [0, partitions holding keys * 2^digit_bits) of
 * its half, publishes the same words, and clears words
 * [0, grid_partitions * 2^digit_bits) of the other half; gs_sort clears both
 * halves before the first pass.  GS_ERR_INVALID_ARGUMENT when more than
 * max_passes passes.
 */
typedef enum gs_pass_keys {
  GS_PASS_KEYS_ALL = 0,
  GS_PASS_KEYS_VISIBLE = 1,
  GS_PASS_KEYS_INSTANCES = 2
} gs_pass_keys;
typedef struct gs_sort_pass {
  int32_t pass;
  int32_t digit_bits;
  int32_t keys;            /* gs_pass_keys */
  int32_t partition_keys;  /* mode 1; 0 in mode 0 */
  int32_t grid_partitions; /* mode 1; 0 in mode 0 */
} gs_sort_pass;
int32_t gs_sort_plan(int64_t n, int64_t capacity, const gs_camera* cam, const gs_settings* set,
                     int32_t max_passes, gs_sort_pass* passes, int32_t* n_passes,
                     int64_t* lookback_words);

/*
 * gs_raster_grid / gs_raster_unit -- host-only view of how the compositing
 * kernels split a frame into workgroups (no HIP call; for tests and tools;
 * the same function the kernels run).  gs_raster_grid: the workgroups of
 * the forward (forward != 0) or backward compositing launch for this
 * camera and these settings, or -1 for invalid arguments.
 * gs_raster_unit: the work of workgroup `workgroup` of that launch, written
 * to unit[3] = (tile, quadrant, band): tile row-major in the grid, quadrant
 * row-major among the tile's 8x8 pixel quadrants, band the row band of the
 * quadrant (0 unless raster_order >> 1 splits the forward's quadrants;
 * band j covers rows j * 8 / 2^s .. of the quadrant).  Returns 1, or 0 for
 * a padding workgroup that takes nothing (unit untouched).  With
 * raster_order bit 0 set, tile_order (host, tiles entries) is the
 * heavy-first order gs_sort wrote after the tile ranges.  Negative status
 * codes for invalid arguments, a workgroup outside the grid, or a missing
 * tile_order.
 */
int64_t gs_raster_grid(const gs_camera* cam, const gs_settings* set, int32_t forward);
int32_t gs_raster_unit(const gs_camera* cam, const gs_settings* set, int32_t forward,
                       const uint32_t* tile_order, int64_t workgroup, int32_t* unit);

/*
 * gs_sort_pairs -- the stable LSD radix sort on its own: sorts n
 * (key u64, value u32) pairs by the low `key_bits` bits of the key
 * (1..64; higher bits must be zero).  keys_in/values_in are not modified;
 * the result goes to keys_out/values_out (distinct buffers).
 * Workspace: gs_workspace_size(GS_STAGE_SORT_PAIRS, 0, n, NULL, set).
 */
int32_t gs_sort_pairs(int64_t n, const uint64_t* keys_in,
                      const uint32_t* values_in, int32_t key_bits,
                      uint64_t* keys_out, uint32_t* values_out,
                      const gs_settings* set, void* workspace,
                      size_t workspace_bytes, void* stream);

/*
 * gs_sort_pairs32 -- the same sort for 32-bit keys, e.g. the depth-only
 * global sort of Algorithm 1 (Section 3.4 sorts splats by depth alone):
 * sorts n (key u32, value u32) pairs by the low `key_bits` bits of the key
 * (1..32; higher bits must be zero), stably.  values_in may be NULL, which
 * stands for values 0..n-1 (the result is then the sorting permutation);
 * keys_out may be NULL when only the values are wanted.  keys_in and
 * values_in are not modified; outputs are distinct buffers.
 * Workspace: gs_workspace_size(GS_STAGE_SORT_PAIRS, 0, n, NULL, set).
 */
int32_t gs_sort_pairs32(int64_t n, const uint32_t* keys_in, const uint32_t* values_in,
                        int32_t key_bits, uint32_t* keys_out, uint32_t* values_out,
                        const gs_settings* set, void* workspace, size_t workspace_bytes,
                        void* stream);

/*
 * gs_rasterize -- Eqs. 2-3 per pixel.  For each tile, its splats are
 * visited in sorted (depth, index) order; per pixel
 *   alpha = min(alpha_max, opacity * exp(-Q/2)); skip if alpha < alpha_min;
 *   C += T * alpha * rgb; T *= (1 - alpha); stop once T < t_eps.
 * Writes image[H*W*4] (RGB = C + T*bg, A = 1 - T), T_final[H*W] and
 * last[H*W] (u32: one past the position, within the tile's sorted range,
 * of the last splat blended into the pixel; used by the backward pass).
 * n_blend[H*W] (u32, optional: NULL skips it) receives the number of
 * splats blended into each pixel, i.e. the count of (pixel, Gaussian)
 * pairs Eq. 3 actually composites.
 */
int32_t gs_rasterize(const gs_splat* splats, const uint32_t* values,
                     const uint32_t* tile_ranges, const gs_camera* cam,
                     const gs_settings* set, float* image, float* T_final,
                     uint32_t* last, uint32_t* n_blend, void* stream);

/*
 * gs_rasterize_mesh -- gs_rasterize composited with a mesh prepass
 * (Algorithm 1, RenderMeshDepthPrepass / DrawSplatsWithMeshDepth; Section
 * 3.4: depth test on, depth write off).  mesh_depth[H*W] (device float32,
 * may be NULL) is the camera-space z of the mesh surface at each pixel
 * centre (+inf where there is none); a splat whose depth is greater than
 * it is hidden at that pixel, and since the list is in depth order the
 * pixel stops there.  A splat exactly at the mesh depth is drawn.
 * mesh_rgb[H*W*3] (device float32, may be NULL) is the mesh colour, used
 * in place of the background behind the Gaussians:
 *   RGB = C + T_final * mesh_rgb,  A = 1 - T_final (the Gaussians' cover).
 * With both NULL this is gs_rasterize.  `last` counts only splats in
 * front of the mesh, so the backward pass needs no depth buffer, only the
 * colour: gs_rasterize_backward_2d_mesh.
 */
int32_t gs_rasterize_mesh(const gs_splat* splats, const uint32_t* values,
                          const uint32_t* tile_ranges, const gs_camera* cam,
                          const gs_settings* set, const float* mesh_depth,
                          const float* mesh_rgb, float* image, float* T_final, uint32_t* last,
                          uint32_t* n_blend, void* stream);

/*
 * gs_rasterize_backward -- gradients of a loss L through Eqs. 1-3
 * (Section 3.2: the formulation is differentiable) for the same inputs and
 * forward outputs, given dL_dimage[H*W*4] (RGBA).
 *
 * The blend order is re-walked from the saved sort (values, tile_ranges)
 * back to front, recovering each transmittance from T_final by division;
 * no per-pixel lists are stored.  Writes d_means[n*3], d_log_scales[n*3],
 * d_quats[n*4], d_opacity_logits[n], d_sh[n*K*3] (overwritten, or added
 * to when `accumulate` is non-zero).  Gradients are zero where a clamp
 * binds (alpha_max, the J clamp, colour at 0) and for culled Gaussians;
 * depth (the sort key) is not differentiated.  Accumulation across pixels
 * uses float atomics, so the last bits can vary from run to run.
 * Workspace: gs_workspace_size(GS_STAGE_BACKWARD, n, 0, cam, set).
 */
int32_t gs_rasterize_backward(
    int64_t n, const float* means, const float* log_scales, const float* quats,
    const float* opacity_logits, const float* sh, int32_t sh_degree,
    const float* model, const gs_camera* cam, const gs_settings* set,
    const gs_splat* splats, const uint32_t* values,
    const uint32_t* tile_ranges, const float* T_final, const uint32_t* last,
    const float* dL_dimage, float* d_means, float* d_log_scales,
    float* d_quats, float* d_opacity_logits, float* d_sh, int32_t accumulate,
    void* workspace, size_t workspace_bytes, void* stream);

/*
 * gs_rasterize_backward_assets -- gs_rasterize_backward for a frame made by
 * gs_preprocess_assets with the same asset table: the compositing backward
 * runs once over the global records, then each asset's chain rule uses its
 * own model transform.  Gradient arrays are indexed like the inputs
 * (concatenated assets).
 */
int32_t gs_rasterize_backward_assets(
    int32_t n_assets, const gs_asset* assets, int64_t n, const float* means,
    const float* log_scales, const float* quats, const float* opacity_logits,
    const float* sh, int32_t sh_degree, const gs_camera* cam, const gs_settings* set,
    const gs_splat* splats, const uint32_t* values, const uint32_t* tile_ranges,
    const float* T_final, const uint32_t* last, const float* dL_dimage,
    float* d_means, float* d_log_scales, float* d_quats, float* d_opacity_logits,
    float* d_sh, int32_t accumulate, void* workspace, size_t workspace_bytes,
    void* stream);

/*
 * gs_rasterize_backward_2d -- the compositing half of gs_rasterize_backward:
 * for one frame made by gs_rasterize, writes grad2d[n * 12] (floats; per
 * Gaussian the gradient of the loss with respect to its 2-D record --
 * mean2d x, y, the whitened form qa, qb, qc, opacity, r, g, b -- then three
 * unused words).  The array is cleared first; Gaussians that reach no
 * pixel keep an all-zero row.  Feed the rows of several views to
 * gs_preprocess_backward_views.
 */
int32_t gs_rasterize_backward_2d(const gs_splat* splats, const uint32_t* values,
                                 const uint32_t* tile_ranges, const gs_camera* cam,
                                 const gs_settings* set, const float* T_final,
                                 const uint32_t* last, const float* dL_dimage, int64_t n,
                                 float* grad2d, void* stream);

/*
 * gs_rasterize_backward_2d_mesh -- gs_rasterize_backward_2d for a frame made
 * by gs_rasterize_mesh: mesh_rgb (the same buffer, or NULL) is the colour
 * behind the Gaussians at each pixel.  Hidden splats lie past each pixel's
 * `last` and receive no gradient; the mesh itself is not differentiated.
 */
int32_t gs_rasterize_backward_2d_mesh(const gs_splat* splats, const uint32_t* values,
                                      const uint32_t* tile_ranges, const gs_camera* cam,
                                      const gs_settings* set, const float* mesh_rgb,
                                      const float* T_final, const uint32_t* last,
                                      const float* dL_dimage, int64_t n, float* grad2d,
                                      void* stream);

/*
 * gs_preprocess_backward_views -- the chain rule of gs_rasterize_backward
 * (Section 3.2) for n_views views at once: cams[v] (host array) and
 * grad2d[v] (host array of device pointers, each an n * 12 float array
 * from gs_rasterize_backward_2d) for the same Gaussians and asset table.
 * Per Gaussian the inputs are read once, the chain runs for every view
 * whose row is non-zero, and the summed input gradients are written to
 * d_means[n*3], d_log_scales[n*3], d_quats[n*4], d_opacity_logits[n],
 * d_sh[n*K*3] (overwritten, or added to when `accumulate` is non-zero).
 * Views are processed 8 per kernel launch.
 */
int32_t gs_preprocess_backward_views(
    int32_t n_views, const gs_camera* cams, const float* const* grad2d, int32_t n_assets,
    const gs_asset* assets, int64_t n, const float* means, const float* log_scales,
    const float* quats, const float* opacity_logits, const float* sh, int32_t sh_degree,
    const gs_settings* set, float* d_means, float* d_log_scales, float* d_quats,
    float* d_opacity_logits, float* d_sh, int32_t accumulate, void* stream);

/*
 * Batches of views (Algorithm 1 renders every model with one global sort;
 * Section 4.5 argues for a single global order).  A batch renders
 * n_views cameras of one scene (an asset table over n Gaussians, as in
 * gs_preprocess_assets) and, with targets, differentiates the mean L1 loss
 * of every view:
 *   L = sum over views v of mean over (H_v, W_v, 3) of |RGB_v - target_v|,
 * accumulating every view's gradient into one set of parameter gradients.
 *
 * The whole batch is a fixed sequence of launches on one stream, whatever
 * the number of views: one preprocess launch over every (view, asset,
 * Gaussian), one global sort whose tile keys cover every view (the views'
 * tile grids are stacked as bands of tile rows of one grid, as wide as the
 * widest view, so a key is band row * width + column), one compositing
 * launch over every view's tiles (longest lists first, over all views),
 * and with targets one loss-gradient launch, one compositing-backward
 * launch and the chain rule (one launch per asset and 8 views).  Counts are
 * read on the device; only gs_batch_plan syncs.  Images equal those of
 * single-view calls with the same settings, bit for bit.
 *
 * Sequence: gs_batch_create (host only; copies the tables) ->
 * gs_batch_plan (one counting pass and one sync: the instance capacity and
 * the depth key bits, each with headroom) -> gs_batch_workspace_size(b,
 * capacity) bytes of workspace -> gs_batch_run (eager) or
 * gs_batch_capture (the same launches recorded into a HIP graph by stream
 * capture on `stream`, instantiated and kept in the batch) and
 * gs_batch_launch (one graph launch).  status_flag (device u32, or NULL)
 * gets bit 0 when a frame needs more instances than planned and bit 1
 * when its depth key range outgrows the planned bits (then plan again; the
 * images are not valid).  The workspace, outputs and status flag bound at
 * capture are the ones every launch uses; they must stay allocated, and
 * the parameters and targets keep their addresses (their values may
 * change between launches; plan again if they change much).
 *
 * Layout of the per-pixel arrays: view v's H_v x W_v pixels start at pixel
 * gs_batch_pixel_offset(b, v); images hold 4 floats per pixel (RGBA),
 * targets 3 (RGB); gs_batch_pixels(b) pixels in all.
 */
typedef struct gs_batch gs_batch;
typedef struct gs_batch_desc {
  int32_t n_views;
  const gs_camera* cams;    /* host, n_views */
  int32_t n_assets;
  const gs_asset* assets;   /* host; model transforms copied */
  int64_t n;                /* Gaussians of all assets */
  const float* means;       /* device: the gs_preprocess inputs */
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* sh;
  int32_t sh_degree;
  const float* targets;     /* device RGB targets, or NULL: forward only */
} gs_batch_desc;

/* Validates the description (the gs_preprocess_assets checks for every
 * camera; at most 256 views) and makes the batch in host memory (no HIP
 * call).  The first gs_batch_plan / gs_batch_run / gs_batch_capture also
 * allocates one small pinned host block (hipHostMalloc) for the camera and
 * view tables that every run copies into the workspace, so that the copy
 * is ordered on the stream (GS_ERR_HIP if that fails).
 * GS_ERR_UNSUPPORTED when the stacked tile grid exceeds 65535 tile rows or
 * 2^26 tiles. */
int32_t gs_batch_create(const gs_batch_desc* desc, const gs_settings* set, gs_batch** batch);
/* Frees the batch and its graph; call it once no work of the batch is
 * pending on any stream. */
void gs_batch_destroy(gs_batch* batch);
int64_t gs_batch_pixels(const gs_batch* batch);
int64_t gs_batch_pixel_offset(const gs_batch* batch, int32_t view);
/* The planned instance capacity (-1 before gs_batch_plan). */
int64_t gs_batch_capacity(const gs_batch* batch);
/* Workspace bytes for an instance capacity (capacity 0: enough for
 * gs_batch_plan). */
size_t gs_batch_workspace_size(const gs_batch* batch, int64_t capacity);
/* Counting pass: preprocesses every view into the workspace, waits for the
 * stream, and sets the capacity to ceil(instances * headroom) (at least
 * 256; headroom in [1, 4]) and the depth key bits to the visible range's
 * bit length plus one.  *capacity receives the capacity.  A graph captured
 * before is dropped (capture again).  GS_ERR_CAPACITY when it would exceed
 * 2^30 - 1 instances. */
int32_t gs_batch_plan(gs_batch* batch, float headroom, void* workspace, size_t workspace_bytes,
                      int64_t* capacity, void* stream);
/* The batch, eagerly: images[pixels * 4] and, with targets, the parameter
 * gradients (overwritten; laid out like the inputs). */
int32_t gs_batch_run(gs_batch* batch, void* workspace, size_t workspace_bytes, float* images,
                     float* d_means, float* d_log_scales, float* d_quats,
                     float* d_opacity_logits, float* d_sh, uint32_t* status_flag, void* stream);
/* gs_batch_run recorded into a HIP graph (stream capture on `stream`, which
 * must not be NULL) and instantiated; nothing runs until gs_batch_launch. */
int32_t gs_batch_capture(gs_batch* batch, void* workspace, size_t workspace_bytes, float* images,
                         float* d_means, float* d_log_scales, float* d_quats,
                         float* d_opacity_logits, float* d_sh, uint32_t* status_flag,
                         void* stream);
/* One launch of the captured graph on `stream` (GS_ERR_INVALID_ARGUMENT
 * when there is none: not captured, or planned since). */
int32_t gs_batch_launch(gs_batch* batch, void* stream);

/*
 * gs_autotune -- picks tile shape, digit width, sort mode and compositing
 * order for a batch by timing whole batches (HIP events; `reps` timed
 * batches after a warm one): a coordinate search from `base`, one
 * dimension at a time in that order, each over its listed values.  Results
 * never depend on these settings, so tuning cannot change an image.
 * Candidates whose workspace exceeds workspace_bytes are skipped.  Syncs
 * the stream once per candidate.  *best, *best_ms and *evaluated
 * (candidates timed; may be NULL) receive the result; GS_ERR_WORKSPACE when
 * no candidate fits.  GS_ERR_INVALID_ARGUMENT for reps outside 1..100 or
 * a space with more than 16 tile shapes, 8 digit widths, 2 sort modes or
 * 6 compositing orders (or a negative count); listed values that
 * gs_settings does not support are skipped.
 */
typedef struct gs_autotune_space {
  int32_t n_tiles;
  int32_t tiles[32];        /* (tile_w, tile_h) pairs */
  int32_t n_bits;
  int32_t bits[8];          /* radix digit widths */
  int32_t n_modes;
  int32_t modes[2];         /* sort modes */
  int32_t n_orders;
  int32_t orders[6];        /* compositing orders */
} gs_autotune_space;
int32_t gs_autotune(const gs_batch_desc* desc, const gs_settings* base,
                    const gs_autotune_space* space, int32_t reps, float headroom, void* workspace,
                    size_t workspace_bytes, float* images, float* d_means, float* d_log_scales,
                    float* d_quats, float* d_opacity_logits, float* d_sh, uint32_t* status_flag,
                    gs_settings* best, float* best_ms, int32_t* evaluated, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H_ */
