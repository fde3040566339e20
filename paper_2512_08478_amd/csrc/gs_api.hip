// C ABI of libgs: argument validation, workspace layout and launch order.
// Every check runs before the first HIP call.
#include <cmath>
#include <cstring>
#include <mutex>

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
  if (s->raster_order != 0 && s->raster_order != 1) return GS_ERR_UNSUPPORTED;
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
  k.tiles_x = tiles_x_of(c, s);
  k.tiles_y = tiles_y_of(c, s);
  k.raster_order = s->raster_order;
  k.eps2d = s->eps2d;
  k.tau = s->alpha_min;
  k.log2_tau = (float)std::log2((double)s->alpha_min);
  k.amax = s->alpha_max;
  k.t_eps = s->t_eps;
  for (int i = 0; i < 3; ++i) k.bg[i] = s->bg[i];
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

int32_t gs_sort(int64_t n, const gs_splat* splats, const uint32_t* depth_keys,
                const uint32_t* tile_rects, const uint32_t* counts, const gs_camera* cam,
                const gs_settings* set,
                int64_t capacity, uint64_t* keys, uint32_t* values, uint32_t* tile_ranges,
                uint32_t* status_flag, void* workspace, size_t workspace_bytes, void* stream) {
  int32_t r;
  if ((r = check_settings(set)) || (r = check_camera(cam, set))) return r;
  if (n < 0 || n >= kMaxN || capacity < 0 || capacity > kMaxInstances) return GS_ERR_INVALID_ARGUMENT;
  if ((r = check_dev(counts)) || (r = check_dev(tile_ranges))) return r;
  if (n > 0 && ((r = check_dev(splats)) || (r = check_dev(depth_keys)) ||
                (r = check_dev(tile_rects))))
    return r;
  if (capacity > 0 && (r = check_dev(values))) return r;
  if ((r = check_dev(keys, false)) || (r = check_dev(status_flag, false))) return r;
  const int tiles_all = tiles_x_of(cam, set) * tiles_y_of(cam, set);
  const gs::SortLayout L = gs::sort_layout(n, capacity, tiles_all);
  if (workspace_bytes < L.bytes) return GS_ERR_WORKSPACE;
  if ((r = check_dev(workspace))) return r;
  const int bits = set->radix_bits, mode = set->sort_mode;
  const bool heavy_first = set->raster_order == 1;
  const int tile_bits = key_bits_of(cam, set) - 32;
  // depth passes: all 32 bits in radix_bits-wide passes, or (depth_bits > 0)
  // depth_bits bits of the keys relative to the smallest visible key, in
  // balanced passes of at most 9 bits (mode 0) or radix_bits (mode 1)
  const int db = set->depth_bits;
  int widths[gs::kMaxPassTotal] = {};
  int pd;
  if (db > 0 && mode == 0) {
    pd = (db + 8) / 9;
    for (int p = 0; p < pd; ++p) {
      const int w = db / pd + (p < db % pd ? 1 : 0);
      widths[p] = w < 6 ? 6 : w;
    }
  } else {
    pd = ((db > 0 ? db : 32) + bits - 1) / bits;
    for (int p = 0; p < pd; ++p) widths[p] = bits;
  }
  const int pt = tile_bits > 0 ? (tile_bits + bits - 1) / bits : 1;
  const int tiles_x = tiles_x_of(cam, set), tiles = tiles_x * tiles_y_of(cam, set);
  char* ws = static_cast<char*>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto U = [&](size_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  uint32_t* count = U(L.count);
  gs::trace_mark(st, "sort_init");
  hipError_t e = gs::launch_sort_init(L, ws, mode, tile_ranges, tiles, status_flag, counts,
                                      capacity, st, heavy_first ? U(L.tcls) : nullptr, db);
  if (e != hipSuccess) return hip_fail(e);
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

}  // extern "C"
