// C ABI of libgs: argument validation, workspace layout and launch order.
// Every check runs before the first HIP call.
#include <array>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "gs_internal.h"

namespace gs {
bool tile_shape_supported(int tw, int th);

namespace {
constexpr int kTraceMax = 4096;
struct Tracer {
  bool on = false;
  bool created = false;
  int count = 0;
  hipEvent_t ev[kTraceMax];
  char label[kTraceMax][32];
};
Tracer g_trace;
}  // namespace

void trace_mark(hipStream_t st, const char* label) {
  Tracer& t = g_trace;
  if (!t.on || t.count >= kTraceMax) return;
  if (hipEventRecord(t.ev[t.count], st) != hipSuccess) return;
  std::strncpy(t.label[t.count], label ? label : "", 31);
  t.label[t.count][31] = 0;
  ++t.count;
}
}  // namespace gs

namespace {

thread_local int32_t g_last_hip_error = 0;

constexpr int64_t kMaxN = (int64_t)1 << 31;           // Gaussians per call
constexpr int64_t kMaxInstances = ((int64_t)1 << 30) - 1;  // look-back counters are 30 bits
constexpr int kMaxBatchViews = 256;                           // views per batch

int32_t hip_fail(hipError_t e) {
  g_last_hip_error = (int32_t)e;
  return GS_ERR_HIP;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// 0 = fine, else a gs_status
int32_t check_dev(const void* p, bool required = true) {
  if (!p) return required ? GS_ERR_INVALID_ARGUMENT : GS_OK;
  return aligned16(p) ? GS_OK : GS_ERR_MISALIGNED;
}

int32_t check_settings(const gs_settings* s) {
  if (!s) return GS_ERR_INVALID_ARGUMENT;
  if (!gs::tile_shape_supported(s->tile_w, s->tile_h)) return GS_ERR_UNSUPPORTED;
  if (s->radix_bits < 6 || s->radix_bits > 8) return GS_ERR_UNSUPPORTED;
  if (s->sort_mode != 0 && s->sort_mode != 1) return GS_ERR_UNSUPPORTED;
  if (s->raster_order < 0 || s->raster_order > 5) return GS_ERR_UNSUPPORTED;  // bands 1, 2, 4
  if (s->depth_bits < 0 || s->depth_bits > 32) return GS_ERR_INVALID_ARGUMENT;
  if (!(s->eps2d >= 0.f) || !std::isfinite(s->eps2d)) return GS_ERR_INVALID_ARGUMENT;
  if (!(s->alpha_min > 0.f) || !(s->alpha_max > s->alpha_min) || !(s->alpha_max < 1.f))
    return GS_ERR_INVALID_ARGUMENT;
  if (!(s->t_eps >= 0.f) || !(s->t_eps < 1.f)) return GS_ERR_INVALID_ARGUMENT;
  if (!(s->clip > 0.f)) return GS_ERR_INVALID_ARGUMENT;
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(s->bg[c])) return GS_ERR_INVALID_ARGUMENT;
  return GS_OK;
}

int32_t check_camera(const gs_camera* c, const gs_settings* s) {
  if (!c) return GS_ERR_INVALID_ARGUMENT;
  if (c->width <= 0 || c->height <= 0 || c->width > 32768 || c->height > 32768)
    return GS_ERR_INVALID_ARGUMENT;
  if (!(c->fx > 0.f) || !(c->fy > 0.f) || !std::isfinite(c->fx) || !std::isfinite(c->fy) ||
      !std::isfinite(c->cx) || !std::isfinite(c->cy) || !(c->znear > 0.f))
    return GS_ERR_INVALID_ARGUMENT;
  for (int k = 0; k < 16; ++k)
    if (!std::isfinite(c->viewmat[k])) return GS_ERR_INVALID_ARGUMENT;
  // upper 3x3 must be a rotation
  double R[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) R[3 * r + k] = c->viewmat[4 * r + k];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double d = 0;
      for (int k = 0; k < 3; ++k) d += R[3 * i + k] * R[3 * j + k];
      if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-4) return GS_ERR_INVALID_ARGUMENT;
    }
  (void)s;
  return GS_OK;
}

int tiles_x_of(const gs_camera* c, const gs_settings* s) { return (c->width + s->tile_w - 1) / s->tile_w; }
int tiles_y_of(const gs_camera* c, const gs_settings* s) { return (c->height + s->tile_h - 1) / s->tile_h; }

int key_bits_of(const gs_camera* c, const gs_settings* s) {
  const int64_t tiles = (int64_t)tiles_x_of(c, s) * tiles_y_of(c, s);
  int b = 0;
  while (((int64_t)1 << b) < tiles) ++b;
  return 32 + b;
}

gs::SetK make_setk(const gs_camera* c, const gs_settings* s) {
  gs::SetK k;
  k.tile_w = s->tile_w;
  k.tile_h = s->tile_h;
  k.tile_w_shift = 0;
  while ((1 << k.tile_w_shift) < s->tile_w) ++k.tile_w_shift;
  k.tile_h_shift = 0;
  while ((1 << k.tile_h_shift) < s->tile_h) ++k.tile_h_shift;
  k.tiles_x = tiles_x_of(c, s);
  k.tiles_y = tiles_y_of(c, s);
  k.raster_order = s->raster_order;
  k.eps2d = s->eps2d;
  k.tau = s->alpha_min;
  k.log2_tau = (float)std::log2((double)s->alpha_min);
  k.amax = s->alpha_max;
  k.t_eps = s->t_eps;
  for (int i = 0; i < 3; ++i) k.bg[i] = s->bg[i];
  k.views = nullptr;
  k.n_views = 0;
  return k;
}

// Camera (and optional similarity model transform) in the kernels' form.
int32_t make_camk(const gs_camera* c, const gs_settings* s, const float* model, gs::CamK* k) {
  std::memset(k, 0, sizeof(*k));
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 4; ++q) k->V[4 * r + q] = c->viewmat[4 * r + q];
  double Vr[9], A[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, tvec[3] = {0, 0, 0};
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) Vr[3 * r + q] = c->viewmat[4 * r + q];
  k->has_model = model ? 1 : 0;
  double sk = 1.0;
  if (model) {
    for (int r = 0; r < 3; ++r) {
      for (int q = 0; q < 3; ++q) A[3 * r + q] = model[4 * r + q];
      tvec[r] = model[4 * r + 3];
    }
    for (int q = 0; q < 12; ++q)
      if (!std::isfinite(model[q])) return GS_ERR_INVALID_ARGUMENT;
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(det > 0.0)) return GS_ERR_INVALID_ARGUMENT;
    sk = std::cbrt(det);
    // must be a similarity: A A^T = s^2 I
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double d = 0;
        for (int q = 0; q < 3; ++q) d += A[3 * i + q] * A[3 * j + q];
        if (std::fabs(d / (sk * sk) - (i == j ? 1.0 : 0.0)) > 1e-4) return GS_ERR_INVALID_ARGUMENT;
      }
  }
  for (int r = 0; r < 3; ++r) {
    for (int q = 0; q < 3; ++q) {
      k->A[4 * r + q] = (float)A[3 * r + q];
      k->Rk[3 * r + q] = (float)(A[3 * r + q] / sk);
      double t3 = 0;
      for (int m = 0; m < 3; ++m) t3 += Vr[3 * r + m] * A[3 * m + q];
      k->T3[3 * r + q] = (float)t3;
    }
    k->A[4 * r + 3] = (float)tvec[r];
  }
  for (int q = 0; q < 3; ++q)
    k->campos[q] = (float)(-(Vr[q] * c->viewmat[3] + Vr[3 + q] * c->viewmat[7] + Vr[6 + q] * c->viewmat[11]));
  k->fx = c->fx; k->fy = c->fy; k->cx = c->cx; k->cy = c->cy;
  k->limx = (float)(s->clip * 0.5 * c->width / c->fx);
  k->limy = (float)(s->clip * 0.5 * c->height / c->fy);
  k->znear = c->znear;
  k->W = c->width;
  k->H = c->height;
  return GS_OK;
}

int32_t check_inputs(int64_t n, const float* means, const float* log_scales, const float* quats,
                     const float* logits, const float* sh, int32_t deg) {
  if (n < 0 || n >= kMaxN) return GS_ERR_INVALID_ARGUMENT;
  if (deg < 0 || deg > 3) return GS_ERR_UNSUPPORTED;
  if (n == 0) return GS_OK;
  int32_t r;
  if ((r = check_dev(means)) || (r = check_dev(log_scales)) || (r = check_dev(quats)) ||
      (r = check_dev(logits)) || (r = check_dev(sh)))
    return r;
  return GS_OK;
}

// assets must tile [0, n) in order: offset_0 = 0, offset_{a+1} = offset_a + count_a
int32_t check_assets(int32_t n_assets, const gs_asset* assets, int64_t n) {
  if (n_assets < 1 || n_assets > gs::kMaxAssets || !assets) return GS_ERR_INVALID_ARGUMENT;
  int64_t next = 0;
  for (int a = 0; a < n_assets; ++a) {
    if (assets[a].offset != next || assets[a].count < 0) return GS_ERR_INVALID_ARGUMENT;
    next += assets[a].count;
  }
  return next == n ? GS_OK : GS_ERR_INVALID_ARGUMENT;
}

}  // namespace

extern "C" {

const char* gs_version(void) { return "libgs 0.1.0 (gfx950)"; }

const char* gs_status_string(int32_t status) {
  switch (status) {
    case GS_OK: return "ok";
    case GS_ERR_INVALID_ARGUMENT: return "invalid argument";
    case GS_ERR_UNSUPPORTED: return "unsupported (SH degree, tile shape or digit width)";
    case GS_ERR_CAPACITY: return "instance capacity exceeded";
    case GS_ERR_HIP: return "HIP runtime error";
    case GS_ERR_MISALIGNED: return "device pointer not 16-byte aligned";
    case GS_ERR_WORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

int32_t gs_last_hip_error(void) { return g_last_hip_error; }

int32_t gs_trace_enable(int32_t on) {
  gs::Tracer& t = gs::g_trace;
  if (on && !t.created) {
    for (int i = 0; i < gs::kTraceMax; ++i) {
      hipError_t e = hipEventCreate(&t.ev[i]);
      if (e != hipSuccess) return hip_fail(e);
    }
    t.created = true;
  }
  t.on = on != 0;
  t.count = 0;
  return GS_OK;
}

int32_t gs_trace_read(int32_t max_entries, char* labels, float* ms, int32_t* count) {
  gs::Tracer& t = gs::g_trace;
  if (!count || (max_entries > 0 && (!labels || !ms))) return GS_ERR_INVALID_ARGUMENT;
  *count = 0;
  if (!t.created || t.count == 0) return GS_OK;
  hipError_t e = hipEventSynchronize(t.ev[t.count - 1]);
  if (e != hipSuccess) return hip_fail(e);
  int k = 0;
  for (int i = 0; i + 1 < t.count && k < max_entries; ++i) {
    if (t.label[i][0] == 0) continue;
    float v = 0.f;
    e = hipEventElapsedTime(&v, t.ev[i], t.ev[i + 1]);
    if (e != hipSuccess) return hip_fail(e);
    std::memcpy(labels + 32 * k, t.label[i], 32);
    ms[k] = v;
    ++k;
  }
  *count = k;
  t.count = 0;
  return GS_OK;
}

void gs_default_settings(gs_settings* s) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->tile_w = 16;
  s->tile_h = 16;
  s->eps2d = 0.3f;
  s->alpha_min = 1.0f / 255.0f;
  s->alpha_max = 0.99f;
  s->t_eps = 1e-4f;
  s->clip = 1.3f;
  s->radix_bits = 8;
  s->sort_mode = 0;
  s->raster_order = 1;
  s->depth_bits = 0;
}

int32_t gs_sort_key_bits(const gs_camera* cam, const gs_settings* set) {
  if (check_settings(set) || check_camera(cam, set)) return -1;
  return key_bits_of(cam, set);
}

size_t gs_workspace_size(int32_t stage, int64_t n, int64_t capacity, const gs_camera* cam,
                         const gs_settings* set) {
  if (n < 0 || capacity < 0) return 0;
  switch (stage) {
    case GS_STAGE_PREPROCESS:
      if (n >= kMaxN) return 0;
      return gs::preprocess_ws_bytes(n);
    case GS_STAGE_SORT:
      if (check_settings(set) || check_camera(cam, set) || capacity > kMaxInstances || n >= kMaxN)
        return 0;
      return gs::sort_layout(n, capacity, tiles_x_of(cam, set) * tiles_y_of(cam, set)).bytes;
    case GS_STAGE_SORT_PAIRS:
      if (check_settings(set) || capacity > kMaxInstances) return 0;
      return gs::pairs_layout(capacity).bytes;
    case GS_STAGE_BACKWARD:
      return gs::align_up((size_t)(n > 0 ? n : 1) * gs::kGrad2dStride * 4, 256);
    default:
      return 0;
  }
}

int32_t gs_preprocess_assets(int32_t n_assets, const gs_asset* assets, int64_t n,
                             const float* means, const float* log_scales, const float* quats,
                             const float* opacity_logits, const float* sh, int32_t sh_degree,
                             const gs_camera* cam, const gs_settings* set, gs_splat* splats,
                             uint32_t* depth_keys, uint32_t* tile_rects, uint32_t* counts,
                             void* workspace, size_t workspace_bytes, void* stream) {
  int32_t r;
  if ((r = check_settings(set)) || (r = check_camera(cam, set))) return r;
  if ((r = check_inputs(n, means, log_scales, quats, opacity_logits, sh, sh_degree))) return r;
  if ((r = check_assets(n_assets, assets, n))) return r;
  if ((r = check_dev(counts))) return r;
  if (n > 0 && ((r = check_dev(splats)) || (r = check_dev(depth_keys)) ||
                (r = check_dev(tile_rects))))
    return r;
  if (workspace_bytes < gs::preprocess_ws_bytes(n)) return GS_ERR_WORKSPACE;
  if ((r = check_dev(workspace))) return r;
  gs::CamK ck[gs::kMaxAssets];
  for (int a = 0; a < n_assets; ++a)
    if ((r = make_camk(cam, set, assets[a].model, &ck[a]))) return r;
  const gs::SetK sk = make_setk(cam, set);
  const int K3 = (sh_degree + 1) * (sh_degree + 1) * 3;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint4* partial = static_cast<uint4*>(workspace);
  int blocks = 0;
  hipError_t e = hipSuccess;
  for (int a = 0; a < n_assets && e == hipSuccess; ++a) {
    const int64_t o = assets[a].offset, c = assets[a].count;
    if (c == 0) continue;
    e = gs::launch_preprocess((int)c, means + 3 * o, log_scales + 3 * o, quats + 4 * o,
                              opacity_logits + o, sh + K3 * o, sh_degree, ck[a], sk, splats + o,
                              depth_keys + o, tile_rects + 2 * o, partial + blocks, st);
    blocks += gs::preprocess_blocks(c);
  }
  if (e == hipSuccess) e = gs::launch_count_finalize(partial, blocks, counts, st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}

int32_t gs_preprocess(int64_t n, const float* means, const float* log_scales, const float* quats,
                      const float* opacity_logits, const float* sh, int32_t sh_degree,
                      const float* model, const gs_camera* cam, const gs_settings* set,
                      gs_splat* splats, uint32_t* depth_keys, uint32_t* tile_rects,
                      uint32_t* counts, void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 0 || n >= kMaxN) return GS_ERR_INVALID_ARGUMENT;
  const gs_asset one = {0, n, model};
  return gs_preprocess_assets(1, &one, n, means, log_scales, quats, opacity_logits, sh,
                              sh_degree, cam, set, splats, depth_keys, tile_rects, counts,
                              workspace, workspace_bytes, stream);
}

// Scratch of gs_preprocess_noalloc: the per-workgroup partial counts of up
// to kNoAllocMaxBytes.  Each GPU the library runs on holds its own copy until
// the process ends; host code reaches a device's copy only through the
// address hipGetSymbolAddress returns on that device.
namespace {
constexpr size_t kNoAllocMaxBytes = (size_t)1 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocMaxBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's scratch address, looked up once per device.
int32_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= kMaxDevices) return GS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (!p) return GS_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}
}  // namespace

int32_t gs_preprocess_noalloc(int64_t n, const float* means, const float* log_scales,
                              const float* quats, const float* opacity_logits, const float* sh,
                              int32_t sh_degree, const float* model, const gs_camera* cam,
                              const gs_settings* set, gs_splat* splats, uint32_t* depth_keys,
                              uint32_t* tile_rects, uint32_t* counts, void* stream) {
  if (n < 0 || n >= kMaxN) return GS_ERR_INVALID_ARGUMENT;
  if (gs::preprocess_ws_bytes(n) > kNoAllocMaxBytes) return GS_ERR_WORKSPACE;
  void* ws = nullptr;
  int32_t r;
  if ((r = scratch_address(&ws))) return r;
  return gs_preprocess(n, means, log_scales, quats, opacity_logits, sh, sh_degree, model, cam, set,
                       splats, depth_keys, tile_rects, counts, ws, kNoAllocMaxBytes, stream);
}

int64_t gs_preprocess_noalloc_max_n(void) {
  return (int64_t)(kNoAllocMaxBytes / 16 - gs::kMaxAssets) * gs::kBlock;
}

int32_t gs_packed_sh_stride(int32_t sh_degree) { return gs::packed_sh_stride(sh_degree); }

int32_t gs_prepack(int64_t n, const float* means, const float* log_scales, const float* quats,
                   const float* opacity_logits, const float* sh, int32_t sh_degree,
                   uint16_t* posop, uint16_t* cov, uint16_t* sh16, void* stream) {
  int32_t r;
  if ((r = check_inputs(n, means, log_scales, quats, opacity_logits, sh, sh_degree))) return r;
  if (n > 0 && ((r = check_dev(posop)) || (r = check_dev(cov)) || (r = check_dev(sh16))))
    return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e = gs::launch_prepack((int)n, means, log_scales, quats, opacity_logits, sh,
                                          sh_degree, posop, cov, sh16, st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}

int32_t gs_lbs_deform(int64_t n, const uint16_t* canon_posop, const uint16_t* canon_cov,
                      const uint8_t* joint_idx, const float* joint_w, int32_t n_joints,
                      const float* joints, uint16_t* posop, uint16_t* cov, void* stream) {
  if (n < 0 || n >= kMaxN || n_joints < 1 || n_joints > 256) return GS_ERR_INVALID_ARGUMENT;
  int32_t r;
  if ((r = check_dev(joints))) return r;
  if (n > 0 && ((r = check_dev(canon_posop)) || (r = check_dev(canon_cov)) ||
                (r = check_dev(joint_idx)) || (r = check_dev(joint_w)) ||
                (r = check_dev(posop)) || (r = check_dev(cov))))
    return r;
  if (n > 0 && (posop == canon_posop || cov == canon_cov)) return GS_ERR_INVALID_ARGUMENT;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e = gs::launch_lbs((int)n, canon_posop, canon_cov, joint_idx, joint_w,
                                      n_joints, joints, posop, cov, st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}

int32_t gs_preprocess_packed(int32_t n_assets, const gs_asset* assets, int64_t n,
                             const uint16_t* posop, const uint16_t* cov, const uint16_t* sh16,
                             int32_t sh_degree, const gs_camera* cam, const gs_settings* set,
                             gs_splat* splats, uint32_t* depth_keys, uint32_t* tile_rects,
                             uint32_t* counts, void* workspace, size_t workspace_bytes,
                             void* stream) {
  int32_t r;
  if ((r = check_settings(set)) || (r = check_camera(cam, set))) return r;
  if (n < 0 || n >= kMaxN) return GS_ERR_INVALID_ARGUMENT;
  if (sh_degree < 0 || sh_degree > 3) return GS_ERR_UNSUPPORTED;
  if ((r = check_assets(n_assets, assets, n))) return r;
  if ((r = check_dev(counts))) return r;
  if (n > 0 && ((r = check_dev(posop)) || (r = check_dev(cov)) || (r = check_dev(sh16)) ||
                (r = check_dev(splats)) || (r = check_dev(depth_keys)) ||
                (r = check_dev(tile_rects))))
    return r;
  if (workspace_bytes < gs::preprocess_ws_bytes(n)) return GS_ERR_WORKSPACE;
  if ((r = check_dev(workspace))) return r;
  gs::CamK ck[gs::kMaxAssets];
  for (int a = 0; a < n_assets; ++a)
    if ((r = make_camk(cam, set, assets[a].model, &ck[a]))) return r;
  const gs::SetK sk = make_setk(cam, set);
  const int S = gs::packed_sh_stride(sh_degree);
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint4* partial = static_cast<uint4*>(workspace);
  int blocks = 0;
  hipError_t e = hipSuccess;
  for (int a = 0; a < n_assets && e == hipSuccess; ++a) {
    const int64_t o = assets[a].offset, c = assets[a].count;
    if (c == 0) continue;
    e = gs::launch_preprocess_packed((int)c, posop + 4 * o, cov + 6 * o, sh16 + S * o, sh_degree,
                                     ck[a], sk, splats + o, depth_keys + o, tile_rects + 2 * o,
                                     partial + blocks, st);
    blocks += gs::preprocess_blocks(c);
  }
  if (e == hipSuccess) e = gs::launch_count_finalize(partial, blocks, counts, st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}

namespace {
// The radix passes of one gs_sort call (shared by gs_sort and gs_sort_plan):
// depth passes first (all 32 bits in radix_bits-wide passes, or depth_bits
// bits of the keys relative to the smallest visible key in balanced passes
// of at most 9 bits in mode 0 / radix_bits in mode 1), then the tile passes.
struct SortPlan {
  int pd = 0, pt = 0;
  int widths[gs::kMaxPassTotal] = {};  // depth pass digit widths
};

int tile_bits_of(int64_t tiles) {
  int b = 0;
  while (((int64_t)1 << b) < tiles) ++b;
  return b;
}

SortPlan plan_sort(int64_t tiles, const gs_settings* set) {
  SortPlan P;
  const int bits = set->radix_bits, mode = set->sort_mode, db = set->depth_bits;
  if (db > 0 && mode == 0) {
    P.pd = (db + 8) / 9;
    for (int p = 0; p < P.pd; ++p) {
      const int w = db / P.pd + (p < db % P.pd ? 1 : 0);
      P.widths[p] = w < 6 ? 6 : w;
    }
  } else {
    P.pd = ((db > 0 ? db : 32) + bits - 1) / bits;
    for (int p = 0; p < P.pd; ++p) P.widths[p] = bits;
  }
  const int tile_bits = tile_bits_of(tiles);
  P.pt = tile_bits > 0 ? (tile_bits + bits - 1) / bits : 1;
  return P;
}
}  // namespace

int32_t gs_sort_plan(int64_t n, int64_t capacity, const gs_camera* cam, const gs_settings* set,
                     int32_t max_passes, gs_sort_pass* passes, int32_t* n_passes,
                     int64_t* lookback_words) {
  int32_t r;
  if ((r = check_settings(set)) || (r = check_camera(cam, set))) return r;
  if (n < 0 || n >= kMaxN || capacity < 0 || capacity > kMaxInstances) return GS_ERR_INVALID_ARGUMENT;
  if (!passes || !n_passes || !lookback_words || max_passes < 0) return GS_ERR_INVALID_ARGUMENT;
  const int tiles = tiles_x_of(cam, set) * tiles_y_of(cam, set);
  const SortPlan P = plan_sort(tiles, set);
  if (P.pd + P.pt > max_passes) return GS_ERR_INVALID_ARGUMENT;
  const gs::SortLayout L = gs::sort_layout(n, capacity, tiles);
  const int64_t part = set->sort_mode == 1 ? gs::kSortPart : 0;
  for (int p = 0; p < P.pd + P.pt; ++p) {
    gs_sort_pass& o = passes[p];
    const bool depth = p < P.pd;
    o.pass = p;
    o.digit_bits = depth ? P.widths[p] : set->radix_bits;
    o.keys = depth ? (p == 0 ? GS_PASS_KEYS_ALL : GS_PASS_KEYS_VISIBLE) : GS_PASS_KEYS_INSTANCES;
    o.partition_keys = (int32_t)part;
    const int64_t grid_n = depth ? n : capacity;
    o.grid_partitions = part > 0 ? (int32_t)((grid_n + part - 1) / part) : 0;
  }
  // in mode 0 the key generation writes the first tile pass's output itself
  *n_passes = P.pd + P.pt;
  *lookback_words = set->sort_mode == 1 ? (int64_t)2 * L.parts * 256 : 0;
  return GS_OK;
}

int64_t gs_raster_grid(const gs_camera* cam, const gs_settings* set, int32_t forward) {
  if (check_settings(set) || check_camera(cam, set)) return -1;
  return gs::raster_units_grid(make_setk(cam, set), forward != 0);
}

int32_t gs_raster_unit(const gs_camera* cam, const gs_settings* set, int32_t forward,
                       const uint32_t* tile_order, int64_t workgroup, int32_t* unit) {
  int32_t r;
  if ((r = check_settings(set)) || (r = check_camera(cam, set))) return r;
  if (!unit || workgroup < 0) return GS_ERR_INVALID_ARGUMENT;
  if ((set->raster_order & 1) && !tile_order) return GS_ERR_INVALID_ARGUMENT;
  const gs::SetK sk = make_setk(cam, set);
  if (workgroup >= gs::raster_units_grid(sk, forward != 0)) return GS_ERR_INVALID_ARGUMENT;
  int tile = 0, q = 0, band = 0;
  if (!gs::raster_unit_host(sk, forward != 0, tile_order, (int)workgroup, &tile, &q, &band))
    return 0;
  unit[0] = tile;
  unit[1] = q;
  unit[2] = band;
  return 1;
}

namespace {
// gs_sort over a tile grid of tiles_x x tiles_y tiles (one view's, or a
// batch's stacked grid); arguments already checked.
int32_t sort_impl(int64_t n, const gs_splat* splats, const uint32_t* depth_keys,
                  const uint32_t* tile_rects, const uint32_t* counts, int tiles_x, int tiles_y,
                  const gs_settings* set, int64_t capacity, uint64_t* keys, uint32_t* values,
                  uint32_t* tile_ranges, uint32_t* status_flag, void* workspace, void* stream) {
  const int tiles = tiles_x * tiles_y;
  const gs::SortLayout L = gs::sort_layout(n, capacity, tiles);
  const int bits = set->radix_bits, mode = set->sort_mode;
  const bool heavy_first = (set->raster_order & 1) != 0;
  const int db = set->depth_bits;
  const SortPlan plan = plan_sort(tiles, set);
  const int* widths = plan.widths;
  const int pd = plan.pd, pt = plan.pt;
  char* ws = static_cast<char*>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto U = [&](size_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  uint32_t* count = U(L.count);
  // sort mode 0 with work to do: the first depth pass's count kernel does
  // the set-up; otherwise a launch of its own
  const bool fold_init = mode == 0 && n > 0 && capacity > 0;
  hipError_t e = hipSuccess;
  if (!fold_init) {
    gs::trace_mark(st, "sort_init");
    e = gs::launch_sort_init(L, ws, mode, tile_ranges, tiles, status_flag, counts, capacity, st,
                             heavy_first ? U(L.tcls) : nullptr, db);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (n == 0 || capacity == 0) {
    if (heavy_first) {
      gs::trace_mark(st, "tile_order");
      e = gs::launch_tile_order(tile_ranges, tiles, U(L.tcls), U(L.tseg), st);
      if (e != hipSuccess) return hip_fail(e);
    }
    gs::trace_mark(st, "");
    return GS_OK;
  }
  // depth digits: the first pass reads all n Gaussians and drops the culled
  // ones (their key is all ones), the later passes sort the visible ones
  gs::RadixArgs<uint32_t> d{};
  d.mode = mode;
  d.n_grid = n;
  d.count = nullptr;
  d.drop_first = 1;
  d.count_rest = counts + 1;
  d.kin = depth_keys;
  d.vin = nullptr;
  d.k_alt = U(L.dk[1]); d.v_alt = U(L.dv[1]);
  d.k_out = U(L.dk[0]); d.v_out = U(L.dv[0]);
  d.table = U(L.table); d.totals = U(L.totals);
  d.hist = U(L.hist); d.tickets = U(L.tickets); d.lookback = U(L.lookback); d.lb_parts = L.parts;
  d.kbase = db > 0 ? counts + 2 : nullptr;
  if (fold_init)
    d.init = gs::sort_init_args(L, ws, tile_ranges, tiles, status_flag, counts, capacity,
                                heavy_first ? U(L.tcls) : nullptr, db);
  if (mode == 0)
    e = gs::launch_radix_sort_widths(d, widths, pd, false, "depth_pass", st);
  else
    e = gs::launch_radix_sort<uint32_t>(d, bits, pd, 0, false, "depth_pass", st);
  if (e != hipSuccess) return hip_fail(e);
  // instances of the visible Gaussians in depth order (their tile rects are
  // gathered into depth order first), then the tile digits
  uint2* drect = reinterpret_cast<uint2*>(ws + L.drect);
  const uint2* rects = reinterpret_cast<const uint2*>(tile_rects);
  gs::RadixArgs<uint32_t> t = d;
  t.init.active = 0;
  t.min_parts = gs::kTilePassMinParts;
  t.n_grid = capacity;
  t.count = count;
  t.drop_first = 0;
  t.count_rest = nullptr;
  t.kbase = nullptr;
  t.k_alt = U(L.tk[1]); t.v_alt = U(L.tv[1]);
  t.k_out = U(L.tkf); t.v_out = values;
  t.hist = U(L.hist) + pd * 256;
  if (mode == 0) {
    // key generation writes the output of the first tile pass directly
    uint32_t* fk = pt > 1 ? U(L.tk[0]) : U(L.tkf);
    uint32_t* fv = pt > 1 ? U(L.tv[0]) : values;
    e = gs::launch_keygen_fused(n, bits, U(L.dv[0]), counts + 1, rects, drect, tiles_x, count,
                                U(L.table), U(L.totals), fk, fv, st);
    if (e != hipSuccess) return hip_fail(e);
    t.kin = fk;
    t.vin = fv;
    e = gs::launch_radix_sort<uint32_t>(t, bits, pt, pd, true, "tile_pass", st, 1);
  } else {
    e = gs::launch_keygen(n, U(L.dv[0]), counts + 1, rects, drect, tiles_x, count,
                          U(L.kg_counts), U(L.totals), U(L.tk[0]), U(L.tv[0]), st);
    if (e != hipSuccess) return hip_fail(e);
    t.kin = U(L.tk[0]);
    t.vin = U(L.tv[0]);
    e = gs::launch_radix_sort<uint32_t>(t, bits, pt, pd, true, "tile_pass", st);
  }
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "tile_ranges");
  e = gs::launch_tile_ranges(capacity, count, U(L.tkf), tile_ranges, st);
  if (e != hipSuccess) return hip_fail(e);
  if (heavy_first) {
    gs::trace_mark(st, "tile_order");
    e = gs::launch_tile_order(tile_ranges, tiles, U(L.tcls), U(L.tseg), st);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (keys) {
    gs::trace_mark(st, "compose_keys");
    e = gs::launch_compose_keys(capacity, count, U(L.tkf), values, splats, keys, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  gs::trace_mark(st, "");
  return GS_OK;
}
}  // namespace

namespace {
// gs_sort's argument checks (no HIP call)
int32_t sort_validate(int64_t n, const gs_splat* splats, const uint32_t* depth_keys,
                      const uint32_t* tile_rects, const uint32_t* counts, const gs_camera* cam,
                      const gs_settings* set, int64_t capacity, uint64_t* keys,
                      uint32_t* values, uint32_t* tile_ranges, uint32_t* status_flag,
                      void* workspace, size_t workspace_bytes) {
  int32_t r;
  if ((r = check_settings(set)) || (r = check_camera(cam, set))) return r;
  if (n < 0 || n >= kMaxN || capacity < 0 || capacity > kMaxInstances) return GS_ERR_INVALID_ARGUMENT;
  if ((r = check_dev(counts)) || (r = check_dev(tile_ranges))) return r;
  if (n > 0 && ((r = check_dev(splats)) || (r = check_dev(depth_keys)) ||
                (r = check_dev(tile_rects))))
    return r;
  if (capacity > 0 && (r = check_dev(values))) return r;
  if ((r = check_dev(keys, false)) || (r = check_dev(status_flag, false))) return r;
  const int tx = tiles_x_of(cam, set), ty = tiles_y_of(cam, set);
  if (workspace_bytes < gs::sort_layout(n, capacity, tx * ty).bytes) return GS_ERR_WORKSPACE;
  return check_dev(workspace);
}
}  // namespace

int32_t gs_sort(int64_t n, const gs_splat* splats, const uint32_t* depth_keys,
                const uint32_t* tile_rects, const uint32_t* counts, const gs_camera* cam,
                const gs_settings* set,
                int64_t capacity, uint64_t* keys, uint32_t* values, uint32_t* tile_ranges,
                uint32_t* status_flag, void* workspace, size_t workspace_bytes, void* stream) {
  int32_t r;
  if ((r = sort_validate(n, splats, depth_keys, tile_rects, counts, cam, set, capacity, keys,
                         values, tile_ranges, status_flag, workspace, workspace_bytes)))
    return r;
  return sort_impl(n, splats, depth_keys, tile_rects, counts, tiles_x_of(cam, set),
                   tiles_y_of(cam, set), set, capacity, keys, values, tile_ranges, status_flag,
                   workspace, stream);
}

int32_t gs_sort_checked(int64_t n, const gs_splat* splats, const uint32_t* depth_keys,
                        const uint32_t* tile_rects, const uint32_t* counts, const gs_camera* cam,
                        const gs_settings* set, int64_t capacity, uint64_t* keys,
                        uint32_t* values, uint32_t* tile_ranges, uint32_t* status_flag,
                        void* workspace, size_t workspace_bytes, int64_t* required,
                        void* stream) {
  int32_t r;
  if ((r = sort_validate(n, splats, depth_keys, tile_rects, counts, cam, set, capacity, keys,
                         values, tile_ranges, status_flag, workspace, workspace_bytes)))
    return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the count the preprocess wrote on this stream, once it is there
  uint32_t c0 = 0;
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipMemcpyAsync(&c0, counts, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  if (required) *required = (int64_t)c0;
  if ((int64_t)c0 > capacity) return GS_ERR_CAPACITY;
  return sort_impl(n, splats, depth_keys, tile_rects, counts, tiles_x_of(cam, set),
                   tiles_y_of(cam, set), set, capacity, keys, values, tile_ranges, status_flag,
                   workspace, stream);
}

int32_t gs_sort_pairs(int64_t n, const uint64_t* keys_in, const uint32_t* values_in,
                      int32_t key_bits, uint64_t* keys_out, uint32_t* values_out,
                      const gs_settings* set, void* workspace, size_t workspace_bytes,
                      void* stream) {
  int32_t r;
  if ((r = check_settings(set))) return r;
  if (n < 0 || n > kMaxInstances || key_bits < 1 || key_bits > 64) return GS_ERR_INVALID_ARGUMENT;
  if (n > 0) {
    if ((r = check_dev(keys_in)) || (r = check_dev(values_in)) || (r = check_dev(keys_out)) ||
        (r = check_dev(values_out)))
      return r;
    if ((const void*)keys_in == (const void*)keys_out || (const void*)values_in == (const void*)values_out)
      return GS_ERR_INVALID_ARGUMENT;
  }
  const gs::SortLayout L = gs::pairs_layout(n);
  if (workspace_bytes < L.bytes) return GS_ERR_WORKSPACE;
  if ((r = check_dev(workspace))) return r;
  if (n == 0) return GS_OK;
  const int bits = set->radix_bits;
  const int passes = (key_bits + bits - 1) / bits;
  char* ws = static_cast<char*>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto U = [&](size_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  gs::trace_mark(st, "sort_init");
  hipError_t e = gs::launch_sort_init(L, ws, set->sort_mode, nullptr, 0, nullptr, nullptr, n, st);
  if (e != hipSuccess) return hip_fail(e);
  gs::RadixArgs<uint64_t> a{};
  a.mode = set->sort_mode;
  a.n_grid = n;
  a.count = nullptr;
  a.kin = keys_in;
  a.vin = values_in;
  a.k_alt = reinterpret_cast<uint64_t*>(ws + L.dk[0]);
  a.v_alt = U(L.dv[0]);
  a.k_out = keys_out;
  a.v_out = values_out;
  a.table = U(L.table); a.totals = U(L.totals);
  a.hist = U(L.hist); a.tickets = U(L.tickets); a.lookback = U(L.lookback); a.lb_parts = L.parts;
  e = gs::launch_radix_sort<uint64_t>(a, bits, passes, 0, true, "radix_pass", st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}

int32_t gs_sort_pairs32(int64_t n, const uint32_t* keys_in, const uint32_t* values_in,
                        int32_t key_bits, uint32_t* keys_out, uint32_t* values_out,
                        const gs_settings* set, void* workspace, size_t workspace_bytes,
                        void* stream) {
  int32_t r;
  if ((r = check_settings(set))) return r;
  if (n < 0 || n > kMaxInstances || key_bits < 1 || key_bits > 32) return GS_ERR_INVALID_ARGUMENT;
  if (n > 0) {
    if ((r = check_dev(keys_in)) || (r = check_dev(values_in, false)) ||
        (r = check_dev(keys_out, false)) || (r = check_dev(values_out)))
      return r;
    if ((const void*)keys_in == (const void*)keys_out ||
        (values_in && (const void*)values_in == (const void*)values_out))
      return GS_ERR_INVALID_ARGUMENT;
  }
  const gs::SortLayout L = gs::pairs_layout(n);
  if (workspace_bytes < L.bytes) return GS_ERR_WORKSPACE;
  if ((r = check_dev(workspace))) return r;
  if (n == 0) return GS_OK;
  const int bits = set->radix_bits;
  const int passes = (key_bits + bits - 1) / bits;
  char* ws = static_cast<char*>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto U = [&](size_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  gs::trace_mark(st, "sort_init");
  hipError_t e = gs::launch_sort_init(L, ws, set->sort_mode, nullptr, 0, nullptr, nullptr, n, st);
  if (e != hipSuccess) return hip_fail(e);
  // a last pass without keys_out writes no keys: the other buffer of the
  // ping-pong pair stands in for keys_out
  uint32_t* kalt = U(L.dk[0]);
  uint32_t* kout = keys_out ? keys_out : U(L.dk[0]) + (size_t)n;
  gs::RadixArgs<uint32_t> a{};
  a.mode = set->sort_mode;
  a.n_grid = n;
  a.count = nullptr;
  a.kin = keys_in;
  a.vin = values_in;
  a.k_alt = kalt;
  a.v_alt = U(L.dv[0]);
  a.k_out = kout;
  a.v_out = values_out;
  a.table = U(L.table); a.totals = U(L.totals);
  a.hist = U(L.hist); a.tickets = U(L.tickets); a.lookback = U(L.lookback); a.lb_parts = L.parts;
  e = gs::launch_radix_sort<uint32_t>(a, bits, passes, 0, keys_out != nullptr, "sort32_pass", st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}

int32_t gs_rasterize_mesh(const gs_splat* splats, const uint32_t* values,
                          const uint32_t* tile_ranges, const gs_camera* cam,
                          const gs_settings* set, const float* mesh_depth,
                          const float* mesh_rgb, float* image, float* T_final, uint32_t* last,
                          uint32_t* n_blend, void* stream) {
  int32_t r;
  if ((r = check_settings(set)) || (r = check_camera(cam, set))) return r;
  if ((r = check_dev(splats, false)) || (r = check_dev(values, false)) ||
      (r = check_dev(tile_ranges)) || (r = check_dev(image)) || (r = check_dev(T_final)) ||
      (r = check_dev(last)) || (n_blend && (r = check_dev(n_blend))) ||
      (r = check_dev(mesh_depth, false)) || (r = check_dev(mesh_rgb, false)))
    return r;
  const gs::SetK sk = make_setk(cam, set);
  hipStream_t st = static_cast<hipStream_t>(stream);
  gs::trace_mark(st, mesh_depth ? "raster_mesh" : "raster");
  hipError_t e = gs::launch_rasterize(splats, values, tile_ranges, sk, cam->width, cam->height,
                                      mesh_depth, mesh_rgb, image, T_final, last, n_blend, st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}

int32_t gs_rasterize(const gs_splat* splats, const uint32_t* values, const uint32_t* tile_ranges,
                     const gs_camera* cam, const gs_settings* set, float* image, float* T_final,
                     uint32_t* last, uint32_t* n_blend, void* stream) {
  return gs_rasterize_mesh(splats, values, tile_ranges, cam, set, nullptr, nullptr, image,
                           T_final, last, n_blend, stream);
}

int32_t gs_rasterize_backward_assets(
    int32_t n_assets, const gs_asset* assets, int64_t n, const float* means,
    const float* log_scales, const float* quats, const float* opacity_logits, const float* sh,
    int32_t sh_degree, const gs_camera* cam, const gs_settings* set, const gs_splat* splats,
    const uint32_t* values, const uint32_t* tile_ranges, const float* T_final,
    const uint32_t* last, const float* dL_dimage, float* d_means, float* d_log_scales,
    float* d_quats, float* d_opacity_logits, float* d_sh, int32_t accumulate, void* workspace,
    size_t workspace_bytes, void* stream) {
  int32_t r;
  if ((r = check_settings(set)) || (r = check_camera(cam, set))) return r;
  if ((r = check_inputs(n, means, log_scales, quats, opacity_logits, sh, sh_degree))) return r;
  if ((r = check_assets(n_assets, assets, n))) return r;
  if ((r = check_dev(tile_ranges)) || (r = check_dev(T_final)) || (r = check_dev(last)) ||
      (r = check_dev(dL_dimage)) || (r = check_dev(values, false)))
    return r;
  if (n > 0 && ((r = check_dev(splats)) || (r = check_dev(d_means)) ||
                (r = check_dev(d_log_scales)) || (r = check_dev(d_quats)) ||
                (r = check_dev(d_opacity_logits)) || (r = check_dev(d_sh))))
    return r;
  const size_t need = gs_workspace_size(GS_STAGE_BACKWARD, n, 0, cam, set);
  if (workspace_bytes < need) return GS_ERR_WORKSPACE;
  if ((r = check_dev(workspace))) return r;
  gs::CamK ck[gs::kMaxAssets];
  for (int a = 0; a < n_assets; ++a)
    if ((r = make_camk(cam, set, assets[a].model, &ck[a]))) return r;
  const gs::SetK sk = make_setk(cam, set);
  if (n == 0) return GS_OK;
  const int K3 = (sh_degree + 1) * (sh_degree + 1) * 3;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* grad2d = static_cast<float*>(workspace);
  gs::trace_mark(st, "bwd_clear");
  hipError_t e = gs::launch_fill_u32(reinterpret_cast<uint32_t*>(grad2d), 0u,
                                     n * gs::kGrad2dStride, st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "raster_bwd");
  e = gs::launch_rasterize_backward(splats, values, tile_ranges, sk, cam->width, cam->height,
                                    nullptr, T_final, last, dL_dimage, grad2d, st);
  if (e != hipSuccess) return hip_fail(e);
  for (int a = 0; a < n_assets && e == hipSuccess; ++a) {
    const int64_t o = assets[a].offset, c = assets[a].count;
    if (c == 0) continue;
    gs::trace_mark(st, "preprocess_bwd");
    e = gs::launch_preprocess_backward(
        (int)c, means + 3 * o, log_scales + 3 * o, quats + 4 * o, opacity_logits + o, sh + K3 * o,
        sh_degree, ck[a], sk, splats + o, grad2d + gs::kGrad2dStride * o, d_means + 3 * o,
        d_log_scales + 3 * o, d_quats + 4 * o, d_opacity_logits + o, d_sh + K3 * o, accumulate,
        st);
  }
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}

int32_t gs_rasterize_backward(int64_t n, const float* means, const float* log_scales,
                              const float* quats, const float* opacity_logits, const float* sh,
                              int32_t sh_degree, const float* model, const gs_camera* cam,
                              const gs_settings* set, const gs_splat* splats,
                              const uint32_t* values, const uint32_t* tile_ranges,
                              const float* T_final, const uint32_t* last, const float* dL_dimage,
                              float* d_means, float* d_log_scales, float* d_quats,
                              float* d_opacity_logits, float* d_sh, int32_t accumulate,
                              void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 0 || n >= kMaxN) return GS_ERR_INVALID_ARGUMENT;
  const gs_asset one = {0, n, model};
  return gs_rasterize_backward_assets(1, &one, n, means, log_scales, quats, opacity_logits, sh,
                                      sh_degree, cam, set, splats, values, tile_ranges, T_final,
                                      last, dL_dimage, d_means, d_log_scales, d_quats,
                                      d_opacity_logits, d_sh, accumulate, workspace,
                                      workspace_bytes, stream);
}

int32_t gs_rasterize_backward_2d(const gs_splat* splats, const uint32_t* values,
                                 const uint32_t* tile_ranges, const gs_camera* cam,
                                 const gs_settings* set, const float* T_final,
                                 const uint32_t* last, const float* dL_dimage, int64_t n,
                                 float* grad2d, void* stream) {
  return gs_rasterize_backward_2d_mesh(splats, values, tile_ranges, cam, set, nullptr, T_final,
                                       last, dL_dimage, n, grad2d, stream);
}

int32_t gs_rasterize_backward_2d_mesh(const gs_splat* splats, const uint32_t* values,
                                      const uint32_t* tile_ranges, const gs_camera* cam,
                                      const gs_settings* set, const float* mesh_rgb,
                                      const float* T_final, const uint32_t* last,
                                      const float* dL_dimage, int64_t n, float* grad2d,
                                      void* stream) {
  int32_t r;
  if ((r = check_settings(set)) || (r = check_camera(cam, set))) return r;
  if (n < 0 || n >= kMaxN) return GS_ERR_INVALID_ARGUMENT;
  if ((r = check_dev(tile_ranges)) || (r = check_dev(T_final)) || (r = check_dev(last)) ||
      (r = check_dev(dL_dimage)) || (r = check_dev(values, false)) ||
      (r = check_dev(mesh_rgb, false)))
    return r;
  if (n > 0 && ((r = check_dev(splats)) || (r = check_dev(grad2d)))) return r;
  if (n == 0) return GS_OK;
  const gs::SetK sk = make_setk(cam, set);
  hipStream_t st = static_cast<hipStream_t>(stream);
  gs::trace_mark(st, "bwd_clear");
  hipError_t e = gs::launch_fill_u32(reinterpret_cast<uint32_t*>(grad2d), 0u,
                                     n * gs::kGrad2dStride, st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "raster_bwd");
  e = gs::launch_rasterize_backward(splats, values, tile_ranges, sk, cam->width, cam->height,
                                    mesh_rgb, T_final, last, dL_dimage, grad2d, st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}

int32_t gs_preprocess_backward_views(
    int32_t n_views, const gs_camera* cams, const float* const* grad2d, int32_t n_assets,
    const gs_asset* assets, int64_t n, const float* means, const float* log_scales,
    const float* quats, const float* opacity_logits, const float* sh, int32_t sh_degree,
    const gs_settings* set, float* d_means, float* d_log_scales, float* d_quats,
    float* d_opacity_logits, float* d_sh, int32_t accumulate, void* stream) {
  int32_t r;
  if ((r = check_settings(set))) return r;
  if (n_views < 1 || !cams || !grad2d) return GS_ERR_INVALID_ARGUMENT;
  if ((r = check_inputs(n, means, log_scales, quats, opacity_logits, sh, sh_degree))) return r;
  if ((r = check_assets(n_assets, assets, n))) return r;
  for (int v = 0; v < n_views; ++v) {
    if ((r = check_camera(&cams[v], set))) return r;
    if (n > 0 && (r = check_dev(grad2d[v]))) return r;
  }
  if (n > 0 && ((r = check_dev(d_means)) || (r = check_dev(d_log_scales)) ||
                (r = check_dev(d_quats)) || (r = check_dev(d_opacity_logits)) ||
                (r = check_dev(d_sh))))
    return r;
  // every camera must be valid for every asset before anything is launched
  for (int v = 0; v < n_views; ++v)
    for (int a = 0; a < n_assets; ++a) {
      gs::CamK ck;
      if ((r = make_camk(&cams[v], set, assets[a].model, &ck))) return r;
    }
  if (n == 0) return GS_OK;
  const gs::SetK sk = make_setk(&cams[0], set);
  const int K3 = (sh_degree + 1) * (sh_degree + 1) * 3;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  gs::trace_mark(st, "preprocess_bwd");
  for (int a = 0; a < n_assets && e == hipSuccess; ++a) {
    const int64_t o = assets[a].offset, c = assets[a].count;
    if (c == 0) continue;
    for (int v0 = 0; v0 < n_views && e == hipSuccess; v0 += gs::kBwdViews) {
      gs::ViewsK vk;
      vk.nv = n_views - v0 < gs::kBwdViews ? n_views - v0 : gs::kBwdViews;
      for (int k = 0; k < gs::kBwdViews; ++k) {
        if (k < vk.nv) {
          make_camk(&cams[v0 + k], set, assets[a].model, &vk.cam[k]);
          vk.g2d[k] = grad2d[v0 + k] + gs::kGrad2dStride * o;
        } else {
          vk.cam[k] = vk.cam[0];
          vk.g2d[k] = nullptr;
        }
      }
      e = gs::launch_preprocess_backward_views(
          (int)c, means + 3 * o, log_scales + 3 * o, quats + 4 * o, opacity_logits + o,
          sh + K3 * o, sh_degree, vk, sk, d_means + 3 * o, d_log_scales + 3 * o, d_quats + 4 * o,
          d_opacity_logits + o, d_sh + K3 * o, (v0 > 0 || accumulate) ? 1 : 0, st);
    }
  }
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}


// ---------------------------------------------------------------- batches of views

struct gs_batch {
  int V = 0, A = 0, deg = 0;
  int64_t n = 0;
  const float *means = nullptr, *log_scales = nullptr, *quats = nullptr, *logits = nullptr,
              *sh = nullptr, *targets = nullptr;
  std::vector<gs_camera> cams;
  std::vector<gs_asset> assets;
  std::vector<std::array<float, 12>> models;
  std::vector<gs::CamK> camk;   // V x A, view-major
  std::vector<gs::ViewK> viewk;
  gs::BatchPreK pre{};
  gs_settings set{};            // with the planned depth_bits
  int TX = 0, TY = 0, max_pix = 0;
  int64_t pixels = 0, capacity = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // pinned host copies of the camera and view tables and the count
  // read-back of gs_batch_plan: copies from pageable memory are not ordered
  // behind the stream's waits on other streams, so a table copied from
  // there could be overwritten by earlier work that still owns the memory
  unsigned char* host = nullptr;
  size_t host_camk = 0, host_viewk = 0, host_counts = 0;
  ~gs_batch() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (host) hipHostFree(host);
  }
};

namespace {
struct BatchLayout {
  size_t camk, viewk, recs, dkeys, rects, partial, counts, T, last, dL, g2d, values, ranges, sort,
      bytes;
};

BatchLayout batch_layout(const gs_batch* b, int64_t capacity) {
  BatchLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = gs::align_up(o + (bytes ? bytes : 1), 256);
    return at;
  };
  const int64_t vn = (int64_t)b->V * b->n, cap = capacity > 0 ? capacity : 0;
  const bool bwd = b->targets != nullptr;
  L.camk = take(b->camk.size() * sizeof(gs::CamK));
  L.viewk = take(b->viewk.size() * sizeof(gs::ViewK));
  L.recs = take((size_t)vn * sizeof(gs_splat));
  L.dkeys = take((size_t)vn * 4);
  L.rects = take((size_t)vn * 8);
  L.partial = take((size_t)b->V * b->pre.block0[b->A] * 16);
  L.counts = take(16);
  L.T = take((size_t)b->pixels * 4);
  L.last = take((size_t)b->pixels * 4);
  L.dL = take(bwd ? (size_t)b->pixels * 16 : 0);
  L.g2d = take(bwd ? (size_t)vn * gs::kGrad2dStride * 4 : 0);
  L.values = take((size_t)cap * 4);
  L.ranges = take((size_t)3 * b->TX * b->TY * 4);
  L.sort = take(gs::sort_layout(vn, cap, b->TX * b->TY).bytes);
  L.bytes = o;
  return L;
}

// The pinned host copy of the camera and view tables and the count
// read-back slot, made on the first call that uses the device.
int32_t batch_host(gs_batch* b) {
  if (b->host) return GS_OK;
  const size_t cb = b->camk.size() * sizeof(gs::CamK), vb = b->viewk.size() * sizeof(gs::ViewK);
  b->host_camk = 0;
  b->host_viewk = gs::align_up(cb, 64);
  b->host_counts = gs::align_up(b->host_viewk + vb, 64);
  void* hp = nullptr;
  const hipError_t e = hipHostMalloc(&hp, b->host_counts + 16, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(e);
  b->host = static_cast<unsigned char*>(hp);
  std::memcpy(b->host + b->host_camk, b->camk.data(), cb);
  std::memcpy(b->host + b->host_viewk, b->viewk.data(), vb);
  return GS_OK;
}

// A captured graph holds the capacity, depth bits and workspace it was
// recorded with; a new plan drops it (gs_batch_launch then fails until the
// next capture).
void batch_drop_graph(gs_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// the tables the kernels read, copied into the workspace (stream-ordered)
hipError_t batch_upload(const gs_batch* b, char* ws, hipStream_t st) {
  const BatchLayout L = batch_layout(b, b->capacity);
  hipError_t e = hipMemcpyAsync(ws + L.camk, b->host + b->host_camk,
                                b->camk.size() * sizeof(gs::CamK), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.viewk, b->host + b->host_viewk, b->viewk.size() * sizeof(gs::ViewK),
                       hipMemcpyHostToDevice, st);
  return e;
}

gs::SetK batch_setk(const gs_batch* b, const char* ws) {
  gs::SetK sk = make_setk(&b->cams[0], &b->set);
  sk.tiles_x = b->TX;
  sk.tiles_y = b->TY;
  sk.views = reinterpret_cast<const gs::ViewK*>(ws + batch_layout(b, b->capacity).viewk);
  sk.n_views = b->V;
  return sk;
}

// preprocess of every view and asset, and the global counts
hipError_t batch_preprocess(const gs_batch* b, char* ws, hipStream_t st) {
  const BatchLayout L = batch_layout(b, b->capacity);
  const gs::SetK sk = batch_setk(b, ws);
  hipError_t e = gs::launch_preprocess_views(
      b->pre, b->V, b->means, b->log_scales, b->quats, b->logits, b->sh, b->deg,
      reinterpret_cast<const gs::CamK*>(ws + L.camk), sk, reinterpret_cast<gs_splat*>(ws + L.recs),
      reinterpret_cast<uint32_t*>(ws + L.dkeys), reinterpret_cast<uint32_t*>(ws + L.rects),
      reinterpret_cast<uint4*>(ws + L.partial), st);
  if (e == hipSuccess)
    e = gs::launch_count_finalize(reinterpret_cast<const uint4*>(ws + L.partial),
                                  b->V * b->pre.block0[b->A], reinterpret_cast<uint32_t*>(ws + L.counts),
                                  st);
  return e;
}

// the whole batch: preprocess, one global sort, compositing; with targets
// the L1 gradient, compositing backward and the chain rule over all views
int32_t batch_enqueue(const gs_batch* b, char* ws, float* images, float* d_means,
                      float* d_log_scales, float* d_quats, float* d_opacity_logits, float* d_sh,
                      uint32_t* status_flag, hipStream_t st) {
  const BatchLayout L = batch_layout(b, b->capacity);
  auto U = [&](size_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  const gs::SetK sk = batch_setk(b, ws);
  hipError_t e = batch_preprocess(b, ws, st);
  if (e != hipSuccess) return hip_fail(e);
  const gs_splat* recs = reinterpret_cast<const gs_splat*>(ws + L.recs);
  int32_t r = sort_impl((int64_t)b->V * b->n, recs, U(L.dkeys), U(L.rects), U(L.counts), b->TX,
                        b->TY, &b->set, b->capacity, nullptr, U(L.values), U(L.ranges),
                        status_flag, ws + L.sort, st);
  if (r) return r;
  gs::trace_mark(st, "raster");
  e = gs::launch_rasterize(recs, U(L.values), U(L.ranges), sk, 0, 0, nullptr, nullptr, images,
                           reinterpret_cast<float*>(ws + L.T), U(L.last), nullptr, st);
  if (e != hipSuccess) return hip_fail(e);
  if (!b->targets) {
    gs::trace_mark(st, "");
    return GS_OK;
  }
  float* dL = reinterpret_cast<float*>(ws + L.dL);
  float* g2d = reinterpret_cast<float*>(ws + L.g2d);
  e = gs::launch_l1_grad(reinterpret_cast<const gs::ViewK*>(ws + L.viewk), b->V, b->max_pix, images,
                         b->targets, dL, st);
  gs::trace_mark(st, "bwd_clear");
  if (e == hipSuccess)
    e = gs::launch_fill_u32(U(L.g2d), 0u, (int64_t)b->V * b->n * gs::kGrad2dStride, st);
  gs::trace_mark(st, "raster_bwd");
  if (e == hipSuccess)
    e = gs::launch_rasterize_backward(recs, U(L.values), U(L.ranges), sk, 0, 0, nullptr,
                                      reinterpret_cast<const float*>(ws + L.T), U(L.last), dL, g2d,
                                      st);
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "preprocess_bwd");
  const int K3 = (b->deg + 1) * (b->deg + 1) * 3;
  const gs::SetK sk1 = make_setk(&b->cams[0], &b->set);
  for (int a = 0; a < b->A && e == hipSuccess; ++a) {
    const int64_t o = b->assets[a].offset, c = b->assets[a].count;
    if (c == 0) continue;
    for (int v0 = 0; v0 < b->V && e == hipSuccess; v0 += gs::kBwdViews) {
      gs::ViewsK vk;
      vk.nv = b->V - v0 < gs::kBwdViews ? b->V - v0 : gs::kBwdViews;
      for (int k = 0; k < gs::kBwdViews; ++k) {
        const int v = v0 + (k < vk.nv ? k : 0);
        vk.cam[k] = b->camk[(size_t)v * b->A + a];
        vk.g2d[k] = k < vk.nv ? g2d + gs::kGrad2dStride * ((int64_t)v * b->n + o) : nullptr;
      }
      e = gs::launch_preprocess_backward_views(
          (int)c, b->means + 3 * o, b->log_scales + 3 * o, b->quats + 4 * o, b->logits + o,
          b->sh + K3 * o, b->deg, vk, sk1, d_means + 3 * o, d_log_scales + 3 * o, d_quats + 4 * o,
          d_opacity_logits + o, d_sh + K3 * o, v0 > 0 ? 1 : 0, st);
    }
  }
  if (e != hipSuccess) return hip_fail(e);
  gs::trace_mark(st, "");
  return GS_OK;
}

int32_t batch_check_run(const gs_batch* b, void* workspace, size_t bytes, float* images,
                        float* d_means, float* d_log_scales, float* d_quats,
                        float* d_opacity_logits, float* d_sh, uint32_t* status_flag) {
  int32_t r;
  if (!b) return GS_ERR_INVALID_ARGUMENT;
  if (b->capacity < 0) return GS_ERR_INVALID_ARGUMENT;  // not planned
  if (bytes < batch_layout(b, b->capacity).bytes) return GS_ERR_WORKSPACE;
  if ((r = check_dev(workspace)) || (r = check_dev(images))) return r;
  if ((r = check_dev(status_flag, false))) return r;
  if (b->targets && ((r = check_dev(d_means)) || (r = check_dev(d_log_scales)) ||
                     (r = check_dev(d_quats)) || (r = check_dev(d_opacity_logits)) ||
                     (r = check_dev(d_sh))))
    return r;
  return GS_OK;
}
}  // namespace

int32_t gs_batch_create(const gs_batch_desc* d, const gs_settings* set, gs_batch** out) {
  int32_t r;
  if (!d || !out) return GS_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if ((r = check_settings(set))) return r;
  if (d->n_views < 1 || d->n_views > kMaxBatchViews || !d->cams) return GS_ERR_INVALID_ARGUMENT;
  if ((r = check_inputs(d->n, d->means, d->log_scales, d->quats, d->opacity_logits, d->sh,
                        d->sh_degree)))
    return r;
  if ((r = check_assets(d->n_assets, d->assets, d->n))) return r;
  if ((r = check_dev(d->targets, false))) return r;
  if (d->n < 1 || (int64_t)d->n_views * d->n >= kMaxN) return GS_ERR_INVALID_ARGUMENT;
  auto b = new gs_batch();
  b->V = d->n_views;
  b->A = d->n_assets;
  b->deg = d->sh_degree;
  b->n = d->n;
  b->means = d->means; b->log_scales = d->log_scales; b->quats = d->quats;
  b->logits = d->opacity_logits; b->sh = d->sh; b->targets = d->targets;
  b->set = *set;
  b->cams.assign(d->cams, d->cams + d->n_views);
  b->assets.assign(d->assets, d->assets + d->n_assets);
  b->models.resize(d->n_assets);
  // the batch's tile grid: each view a band of tile rows, as wide as the
  // widest view
  int row = 0;
  int64_t pix = 0;
  for (int v = 0; v < b->V; ++v) {
    if ((r = check_camera(&b->cams[v], set))) { delete b; return r; }
    gs::ViewK k{};
    k.row = row;
    k.tiles_x = tiles_x_of(&b->cams[v], set);
    k.tiles_y = tiles_y_of(&b->cams[v], set);
    k.W = b->cams[v].width;
    k.H = b->cams[v].height;
    k.pix = (size_t)pix;
    b->viewk.push_back(k);
    row += k.tiles_y;
    pix += (int64_t)k.W * k.H;
    b->TX = k.tiles_x > b->TX ? k.tiles_x : b->TX;
    b->max_pix = k.W * k.H > b->max_pix ? k.W * k.H : b->max_pix;
  }
  b->TY = row;
  b->pixels = pix;
  if (b->TY > 0xFFFF || (int64_t)b->TX * b->TY >= ((int64_t)1 << 26)) {
    delete b;
    return GS_ERR_UNSUPPORTED;
  }
  b->pre.n = d->n;
  b->pre.n_assets = d->n_assets;
  int blocks = 0;
  for (int a = 0; a < d->n_assets; ++a) {
    b->pre.block0[a] = blocks;
    b->pre.offset[a] = d->assets[a].offset;
    b->pre.count[a] = (int)d->assets[a].count;
    blocks += gs::preprocess_blocks(d->assets[a].count);
    if (d->assets[a].model) {
      std::memcpy(b->models[a].data(), d->assets[a].model, 12 * sizeof(float));
      b->assets[a].model = b->models[a].data();
    }
  }
  b->pre.block0[d->n_assets] = blocks;
  b->camk.resize((size_t)b->V * b->A);
  for (int v = 0; v < b->V; ++v)
    for (int a = 0; a < b->A; ++a) {
      gs::CamK& ck = b->camk[(size_t)v * b->A + a];
      if ((r = make_camk(&b->cams[v], set, b->assets[a].model, &ck))) { delete b; return r; }
      ck.tile_row = b->viewk[v].row;
    }
  *out = b;
  return GS_OK;
}

void gs_batch_destroy(gs_batch* b) { delete b; }

int64_t gs_batch_pixels(const gs_batch* b) { return b ? b->pixels : -1; }

int64_t gs_batch_pixel_offset(const gs_batch* b, int32_t view) {
  if (!b || view < 0 || view >= b->V) return -1;
  return (int64_t)b->viewk[view].pix;
}

int64_t gs_batch_capacity(const gs_batch* b) { return b ? b->capacity : -1; }

size_t gs_batch_workspace_size(const gs_batch* b, int64_t capacity) {
  if (!b || capacity < 0 || capacity > kMaxInstances) return 0;
  return batch_layout(b, capacity).bytes;
}

int32_t gs_batch_plan(gs_batch* b, float headroom, void* workspace, size_t workspace_bytes,
                      int64_t* capacity, void* stream) {
  int32_t r;
  if (!b || !capacity || !(headroom >= 1.f) || !(headroom <= 4.f)) return GS_ERR_INVALID_ARGUMENT;
  if (workspace_bytes < batch_layout(b, 0).bytes) return GS_ERR_WORKSPACE;
  if ((r = check_dev(workspace))) return r;
  if ((r = batch_host(b))) return r;
  batch_drop_graph(b);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const int64_t keep = b->capacity;
  b->capacity = 0;
  hipError_t e = batch_upload(b, ws, st);
  if (e == hipSuccess) e = batch_preprocess(b, ws, st);
  uint32_t* c = reinterpret_cast<uint32_t*>(b->host + b->host_counts);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c, ws + batch_layout(b, 0).counts, 16, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    b->capacity = keep;
    return hip_fail(e);
  }
  // the instance capacity and the depth key bits, with headroom for
  // parameter updates between plans (a frame that outgrows them raises
  // bit 0 or bit 1 of the status flag)
  int64_t cap = (int64_t)std::ceil((double)c[0] * headroom);
  cap = cap < 256 ? 256 : cap;
  if (cap > kMaxInstances) return GS_ERR_CAPACITY;
  int db = 0;
  if (c[1] > 0) {
    const uint32_t range = c[3] - c[2];
    while (db < 32 && ((uint64_t)range >> db) != 0) ++db;
    db = db + 1 < 32 ? db + 1 : 32;
  }
  b->set.depth_bits = db;
  b->capacity = cap;
  *capacity = cap;
  return GS_OK;
}

int32_t gs_batch_run(gs_batch* b, void* workspace, size_t workspace_bytes, float* images,
                     float* d_means, float* d_log_scales, float* d_quats, float* d_opacity_logits,
                     float* d_sh, uint32_t* status_flag, void* stream) {
  int32_t r;
  if ((r = batch_check_run(b, workspace, workspace_bytes, images, d_means, d_log_scales, d_quats,
                           d_opacity_logits, d_sh, status_flag)))
    return r;
  if ((r = batch_host(b))) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = batch_upload(b, static_cast<char*>(workspace), st);
  if (e != hipSuccess) return hip_fail(e);
  return batch_enqueue(b, static_cast<char*>(workspace), images, d_means, d_log_scales, d_quats,
                       d_opacity_logits, d_sh, status_flag, st);
}

int32_t gs_batch_capture(gs_batch* b, void* workspace, size_t workspace_bytes, float* images,
                         float* d_means, float* d_log_scales, float* d_quats,
                         float* d_opacity_logits, float* d_sh, uint32_t* status_flag,
                         void* stream) {
  int32_t r;
  if ((r = batch_check_run(b, workspace, workspace_bytes, images, d_means, d_log_scales, d_quats,
                           d_opacity_logits, d_sh, status_flag)))
    return r;
  if (!stream) return GS_ERR_INVALID_ARGUMENT;  // the legacy stream cannot be captured
  if ((r = batch_host(b))) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  // the tables go to the workspace before the capture (the graph reads
  // them there)
  hipError_t e = batch_upload(b, ws, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  batch_drop_graph(b);
  e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e);
  r = batch_enqueue(b, ws, images, d_means, d_log_scales, d_quats, d_opacity_logits, d_sh,
                    status_flag, st);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(st, &g);
  if (r) {
    if (g) hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) return hip_fail(e);
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return hip_fail(e);
  }
  b->graph = g;
  return GS_OK;
}

int32_t gs_batch_launch(gs_batch* b, void* stream) {
  if (!b || !b->exec) return GS_ERR_INVALID_ARGUMENT;
  const hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GS_OK : hip_fail(e);
}

int32_t gs_autotune(const gs_batch_desc* desc, const gs_settings* base,
                    const gs_autotune_space* space, int32_t reps, float headroom, void* workspace,
                    size_t workspace_bytes, float* images, float* d_means, float* d_log_scales,
                    float* d_quats, float* d_opacity_logits, float* d_sh, uint32_t* status_flag,
                    gs_settings* best, float* best_ms, int32_t* evaluated, void* stream) {
  int32_t r;
  if (!desc || !base || !space || !best || !best_ms || reps < 1 || reps > 100)
    return GS_ERR_INVALID_ARGUMENT;
  if (space->n_tiles < 0 || space->n_tiles > 16 || space->n_bits < 0 || space->n_bits > 8 ||
      space->n_modes < 0 || space->n_modes > 2 || space->n_orders < 0 || space->n_orders > 6)
    return GS_ERR_INVALID_ARGUMENT;
  if ((r = check_settings(base))) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t ev[2];
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e != hipSuccess) return hip_fail(e);
  int nev = 0;
  // time one candidate: plan, one warm batch, then `reps` timed batches
  auto measure = [&](const gs_settings& s, float* ms) -> int32_t {
    *ms = INFINITY;
    if (check_settings(&s)) return GS_OK;  // not a valid candidate
    gs_batch* b = nullptr;
    int32_t q = gs_batch_create(desc, &s, &b);
    if (q) return q == GS_ERR_UNSUPPORTED ? GS_OK : q;
    int64_t cap = 0;
    q = gs_batch_plan(b, headroom, workspace, workspace_bytes, &cap, stream);
    if (q == GS_OK && batch_layout(b, cap).bytes <= workspace_bytes) {
      q = gs_batch_run(b, workspace, workspace_bytes, images, d_means, d_log_scales, d_quats,
                       d_opacity_logits, d_sh, status_flag, stream);
      hipError_t he = hipEventRecord(ev[0], st);
      for (int k = 0; k < reps && q == GS_OK; ++k)
        q = batch_enqueue(b, static_cast<char*>(workspace), images, d_means, d_log_scales,
                          d_quats, d_opacity_logits, d_sh, status_flag, st);
      if (he == hipSuccess) he = hipEventRecord(ev[1], st);
      if (he == hipSuccess) he = hipEventSynchronize(ev[1]);
      float t = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&t, ev[0], ev[1]);
      if (he != hipSuccess && q == GS_OK) q = hip_fail(he);
      if (q == GS_OK) {
        *ms = t / reps;
        ++nev;
      }
    } else if (q == GS_ERR_WORKSPACE || q == GS_OK) {
      q = GS_OK;  // does not fit the workspace: skipped
    }
    gs_batch_destroy(b);
    return q;
  };
  gs_settings cur = *base;
  float cur_ms = INFINITY;
  r = measure(cur, &cur_ms);
  // coordinate search: tile shape, digit width, sort mode, compositing order
  for (int dim = 0; dim < 4 && r == GS_OK; ++dim) {
    const int cnt = dim == 0 ? space->n_tiles : dim == 1 ? space->n_bits
                    : dim == 2 ? space->n_modes : space->n_orders;
    for (int k = 0; k < cnt && r == GS_OK; ++k) {
      gs_settings s = cur;
      if (dim == 0) { s.tile_w = space->tiles[2 * k]; s.tile_h = space->tiles[2 * k + 1]; }
      else if (dim == 1) s.radix_bits = space->bits[k];
      else if (dim == 2) s.sort_mode = space->modes[k];
      else s.raster_order = space->orders[k];
      if (s.tile_w == cur.tile_w && s.tile_h == cur.tile_h && s.radix_bits == cur.radix_bits &&
          s.sort_mode == cur.sort_mode && s.raster_order == cur.raster_order)
        continue;
      float ms;
      r = measure(s, &ms);
      if (r == GS_OK && ms < cur_ms) {
        cur = s;
        cur_ms = ms;
      }
    }
  }
  hipEventDestroy(ev[0]);
  hipEventDestroy(ev[1]);
  if (r) return r;
  *best = cur;
  best->depth_bits = base->depth_bits;
  *best_ms = cur_ms;
  if (evaluated) *evaluated = nev;
  return std::isfinite(cur_ms) ? GS_OK : GS_ERR_WORKSPACE;
}

}  // extern "C"
