// FP16 pre-pack and the preprocess that reads it (Algorithm 1's Pre-pack
// step and Section 3.4's FP16 layout), and the linear-blend-skinning
// pre-decoder that deforms packed canonical Gaussians (Section 3.3).
//
// Pre-pack, once per asset: the covariance Sigma = R diag(s^2) R^T is formed
// from scale and rotation, and the mean, the activated opacity, the upper
// triangle of Sigma and the SH coefficients are stored as binary16, two to
// a 32-bit word.  Per frame, the packed preprocess reads 20 + 2*S bytes per
// Gaussian (S halves of SH, 48 at degree 3) instead of 48 + 4*3K, and
// writes the same records, depth keys and tile rects as the raw-parameter
// preprocess, so sorting and compositing are shared.
//
// Layout (n Gaussians, little-endian halves):
//   posop  n x 4  (mu_x, mu_y, mu_z, alpha)                 8 bytes
//   cov    n x 6  (xx, xy, xz, yy, yz, zz) of Sigma          12 bytes
//   sh16   n x S  the 3K coefficients, coefficient-major, RGB innermost,
//                 zero-padded to S = 3K rounded up to a multiple of 4
//                 (4, 12, 28, 48 halves for degrees 0..3)
//
// Opacity and covariance are computed in float64 and rounded once to the
// nearest binary16 (ties to even): float64 -> float32 rounds to odd, which
// makes the second rounding, float32 -> binary16, exact-nearest.  Means and
// SH are float32 inputs rounded directly.
//
// The packed preprocess forms the 2-D covariance S = P Sigma P^T (P = J W,
// 2x3) and its determinant in float64: Sigma arrives as a matrix, not as
// factors, so the Cauchy-Binet form of the raw path is not available and
// det = ac - b^2 would cancel in float32 for thin splats seen edge-on.
#include "gs_device.h"
#include "gs_internal.h"
#include "gs_project.h"

namespace gs {
namespace {

__device__ __forceinline__ uint16_t f32_to_f16(float f) {
  return __builtin_bit_cast(uint16_t, static_cast<_Float16>(f));
}

__device__ __forceinline__ float f16_to_f32(uint32_t h) {
  return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(h & 0xFFFFu)));
}

// Nearest binary16 of a float64 value, ties to even.  Rounding to float32
// by round-to-odd first (truncate, then set the last bit if anything was
// cut off) keeps enough information for the final rounding to be correct.
__device__ __forceinline__ uint16_t f64_to_f16(double d) {
  float f = static_cast<float>(d);
  const double back = static_cast<double>(f);
  if (back != d && d == d) {
    uint32_t u = __float_as_uint(f);
    if (fabs(back) > fabs(d)) u -= 1u;  // rounded away from zero: step back
    f = __uint_as_float(u | 1u);
  }
  return f32_to_f16(f);
}

__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) {
  return (uint32_t)lo | ((uint32_t)hi << 16);
}

template <int DEG>
struct ShPack {
  static constexpr int K3 = (DEG + 1) * (DEG + 1) * 3;
  static constexpr int S = (K3 + 3) / 4 * 4;  // halves per packed row
  static constexpr int U2 = S / 4;            // 8-byte words per packed row
};

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_prepack(
    int n, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, uint2* __restrict__ posop, uint32_t* __restrict__ cov,
    uint2* __restrict__ sh16) {
  using P = ShPack<DEG>;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double o = 1.0 / (1.0 + exp(-(double)logits[i]));
  posop[i] = make_uint2(pack2(f32_to_f16(means[3 * i]), f32_to_f16(means[3 * i + 1])),
                        pack2(f32_to_f16(means[3 * i + 2]), f64_to_f16(o)));
  // Sigma = M M^T with M = R diag(s)
  const float4 q = quats[i];
  double qw = q.x, qx = q.y, qy = q.z, qz = q.w;
  const double inv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= inv; qx *= inv; qy *= inv; qz *= inv;
  const double R[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz),
                       2.0 * (qx * qz + qw * qy),       2.0 * (qx * qy + qw * qz),
                       1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                       2.0 * (qx * qz - qw * qy),       2.0 * (qy * qz + qw * qx),
                       1.0 - 2.0 * (qx * qx + qy * qy)};
  const double s[3] = {exp((double)log_scales[3 * i]), exp((double)log_scales[3 * i + 1]),
                       exp((double)log_scales[3 * i + 2])};
  double M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) M[3 * r + c] = R[3 * r + c] * s[c];
  auto sig = [&](int r, int c) {
    return M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
  };
  cov[3 * i] = pack2(f64_to_f16(sig(0, 0)), f64_to_f16(sig(0, 1)));
  cov[3 * i + 1] = pack2(f64_to_f16(sig(0, 2)), f64_to_f16(sig(1, 1)));
  cov[3 * i + 2] = pack2(f64_to_f16(sig(1, 2)), f64_to_f16(sig(2, 2)));
  const float* row = sh + (size_t)i * P::K3;
  uint2* out = sh16 + (size_t)i * P::U2;
#pragma unroll
  for (int w = 0; w < P::U2; ++w) {
    uint16_t h[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = 4 * w + k;
      h[k] = e < P::K3 ? f32_to_f16(row[e]) : (uint16_t)0;
    }
    out[w] = make_uint2(pack2(h[0], h[1]), pack2(h[2], h[3]));
  }
}

// Packed SH row of Gaussian i, loaded whole: 16-byte loads when a row is a
// whole number of 16-byte vectors (degree 3: 96 bytes), else 8-byte loads.
template <int DEG>
struct ShRow {
  static constexpr int S = ShPack<DEG>::S;
  static constexpr bool V16 = (S % 8) == 0;
  static constexpr int WORDS = S / 2;  // 32-bit words
  uint32_t w[WORDS];
  __device__ __forceinline__ void load(const uint2* __restrict__ sh16, int i) {
    if constexpr (V16) {
      const uint4* row = reinterpret_cast<const uint4*>(sh16) + (size_t)i * (S / 8);
#pragma unroll
      for (int k = 0; k < S / 8; ++k) {
        const uint4 u = row[k];
        w[4 * k] = u.x; w[4 * k + 1] = u.y; w[4 * k + 2] = u.z; w[4 * k + 3] = u.w;
      }
    } else {
      const uint2* row = sh16 + (size_t)i * (S / 4);
#pragma unroll
      for (int k = 0; k < S / 4; ++k) {
        const uint2 u = row[k];
        w[2 * k] = u.x; w[2 * k + 1] = u.y;
      }
    }
  }
  __device__ __forceinline__ float at(int e) const {
    return f16_to_f32(e & 1 ? w[e >> 1] >> 16 : w[e >> 1]);
  }
};

// Eq. 1 from the packed layout.  The packed SH row is loaded together with
// the mean, opacity and covariance, before the culls: one round trip to
// memory per Gaussian instead of two (the loads of a culled Gaussian's row
// are wasted, which costs less than a second dependent round trip).
template <int DEG>
__global__ __launch_bounds__(kBlock) void k_preprocess_packed(
    int n, const uint2* __restrict__ posop, const uint32_t* __restrict__ cov,
    const uint2* __restrict__ sh16, CamK cam, SetK set, gs_splat* __restrict__ splats,
    uint32_t* __restrict__ depth_keys, uint2* __restrict__ rects, uint4* __restrict__ partial) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int i = blockIdx.x * kBlock + threadIdx.x;
  uint32_t tiles = 0, dkey = 0xFFFFFFFFu;
  if (i < n) {
    const uint2 po = posop[i];
    const uint32_t c0 = cov[3 * i], c1 = cov[3 * i + 1], c2 = cov[3 * i + 2];
    ShRow<DEG> shr;
    shr.load(sh16, i);
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    uint32_t rect_lo = 0x0000FFFFu, rect_hi = 0u;  // empty pixel bbox
    uint2 trect = make_uint2(0x0000FFFFu, 0u);      // empty tile rect
    float dir[3] = {0.f, 0.f, 0.f};
    const float o = f16_to_f32(po.y >> 16);
    float w[3];
    double t[3];
    place_mean(f16_to_f32(po.x), f16_to_f32(po.x >> 16), f16_to_f32(po.y), cam, w, t);
    const float tx = (float)t[0], ty = (float)t[1], tz = (float)t[2];
    if ((tz > cam.znear) && (o >= set.tau) && __builtin_isfinite(tx) && __builtin_isfinite(ty)) {
      const double sxx = f16_to_f32(c0), sxy = f16_to_f32(c0 >> 16), sxz = f16_to_f32(c1),
                   syy = f16_to_f32(c1 >> 16), syz = f16_to_f32(c2), szz = f16_to_f32(c2 >> 16);
      // Jacobian of the perspective division at t (x/z, y/z clamped)
      const float iz = 1.f / tz;
      const float xt = fminf(cam.limx, fmaxf(-cam.limx, tx * iz));
      const float yt = fminf(cam.limy, fmaxf(-cam.limy, ty * iz));
      const double j00 = cam.fx * iz, j02 = -cam.fx * xt * iz;
      const double j11 = cam.fy * iz, j12 = -cam.fy * yt * iz;
      // P = J T3 (rows p, r); then Sigma p, Sigma r
      double p[3], r[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        p[c] = j00 * (double)cam.T3[c] + j02 * (double)cam.T3[6 + c];
        r[c] = j11 * (double)cam.T3[3 + c] + j12 * (double)cam.T3[6 + c];
      }
      const double sp0 = sxx * p[0] + sxy * p[1] + sxz * p[2];
      const double sp1 = sxy * p[0] + syy * p[1] + syz * p[2];
      const double sp2 = sxz * p[0] + syz * p[1] + szz * p[2];
      const double aa = p[0] * sp0 + p[1] * sp1 + p[2] * sp2;
      const double b = r[0] * sp0 + r[1] * sp1 + r[2] * sp2;
      const double cc = r[0] * (sxx * r[0] + sxy * r[1] + sxz * r[2]) +
                        r[1] * (sxy * r[0] + syy * r[1] + syz * r[2]) +
                        r[2] * (sxz * r[0] + syz * r[1] + szz * r[2]);
      const double e = set.eps2d;
      const double a = aa + e, c = cc + e;
      const double D = a * c - b * b;
      tiles = footprint(t, iz, w[0], w[1], w[2], (float)a, (float)b, (float)c, (float)D, o,
                        cam, set, r0, r1, rect_lo, rect_hi, trect, dir);
      if (tiles) {
        float Y[16];
        sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
        float acc[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int k = 0; k < K; ++k) {
          acc[0] = fmaf(shr.at(3 * k), Y[k], acc[0]);
          acc[1] = fmaf(shr.at(3 * k + 1), Y[k], acc[1]);
          acc[2] = fmaf(shr.at(3 * k + 2), Y[k], acc[2]);
        }
        r1.z = fmaxf(acc[0], 0.f);
        r1.w = fmaxf(acc[1], 0.f);
        r2.x = fmaxf(acc[2], 0.f);
      }
    }
    r2.y = tz;
    r2.z = __uint_as_float(rect_lo);
    r2.w = __uint_as_float(rect_hi);
    dkey = tiles ? __float_as_uint(tz) : 0xFFFFFFFFu;
    depth_keys[i] = dkey;
    rects[i] = trect;
    float4* dst = reinterpret_cast<float4*>(splats + i);
    dst[0] = r0;
    dst[1] = r1;
    dst[2] = r2;
  }
  block_counts(tiles, dkey, partial);
}

// Linear blend skinning of pre-packed canonical Gaussians (the avatar
// pre-decoder of Section 3.3, Eqs. 5-6): T_i = sum_k w_ik M_k = [R_i | t_i],
// mu_i = R_i mu^_i + t_i, Sigma_i = R_i Sigma^_i R_i^T.  The joint
// transforms are staged in LDS, followed by one all-zero transform that
// every index >= n_joints is clamped to (it contributes nothing); the
// blend and both products run in float64 from the exactly decoded
// canonical values and are rounded once to binary16, so the identity pose
// reproduces the canonical values.  Opacity is copied.  Each thread skins
// kLbsItems Gaussians a block-width apart, with all their loads issued
// before the first is computed, which also spreads the LDS staging over
// more Gaussians.
constexpr int kMaxJoints = 256;
constexpr int kInfluences = 4;
constexpr int kLbsItems = 4;

__global__ __launch_bounds__(kBlock) void k_lbs(
    int n, const uint2* __restrict__ canon_posop, const uint32_t* __restrict__ canon_cov,
    const uint32_t* __restrict__ joint_idx, const float4* __restrict__ joint_w, int n_joints,
    const float* __restrict__ joints, uint2* __restrict__ posop, uint32_t* __restrict__ cov) {
  __shared__ float s_m[(kMaxJoints + 1) * 12];
  for (int e = threadIdx.x; e < (n_joints + 1) * 12; e += kBlock)
    s_m[e] = e < n_joints * 12 ? joints[e] : 0.f;
  __syncthreads();
  const int base = blockIdx.x * kBlock * kLbsItems + threadIdx.x;
  uint2 po[kLbsItems];
  uint32_t c0[kLbsItems], c1[kLbsItems], c2[kLbsItems], ji[kLbsItems];
  float4 wv[kLbsItems];
#pragma unroll
  for (int u = 0; u < kLbsItems; ++u) {
    const int i = min(base + u * kBlock, n - 1);  // clamped: past-the-end items are not stored
    po[u] = canon_posop[i];
    c0[u] = canon_cov[3 * i];
    c1[u] = canon_cov[3 * i + 1];
    c2[u] = canon_cov[3 * i + 2];
    ji[u] = joint_idx[i];
    wv[u] = joint_w[i];
  }
#pragma unroll
  for (int u = 0; u < kLbsItems; ++u) {
    const int i = base + u * kBlock;
    if (i >= n) break;
    const float wk[kInfluences] = {wv[u].x, wv[u].y, wv[u].z, wv[u].w};
    double T[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) T[e] = 0.0;
#pragma unroll
    for (int k = 0; k < kInfluences; ++k) {
      const int j = min((int)((ji[u] >> (8 * k)) & 0xFFu), n_joints);
      const float* m = s_m + 12 * j;
      const double w = wk[k];
#pragma unroll
      for (int e = 0; e < 12; ++e) T[e] += w * (double)m[e];
    }
    const double mu[3] = {f16_to_f32(po[u].x), f16_to_f32(po[u].x >> 16), f16_to_f32(po[u].y)};
    double md[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      md[r] = T[4 * r] * mu[0] + T[4 * r + 1] * mu[1] + T[4 * r + 2] * mu[2] + T[4 * r + 3];
    const double S[9] = {f16_to_f32(c0[u]),       f16_to_f32(c0[u] >> 16), f16_to_f32(c1[u]),
                         f16_to_f32(c0[u] >> 16), f16_to_f32(c1[u] >> 16), f16_to_f32(c2[u]),
                         f16_to_f32(c1[u]),       f16_to_f32(c2[u]),       f16_to_f32(c2[u] >> 16)};
    // RS = R Sigma^, then Sigma = RS R^T (upper triangle)
    double RS[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        RS[3 * r + c] = T[4 * r] * S[c] + T[4 * r + 1] * S[3 + c] + T[4 * r + 2] * S[6 + c];
    auto sig = [&](int r, int c) {
      return RS[3 * r] * T[4 * c] + RS[3 * r + 1] * T[4 * c + 1] + RS[3 * r + 2] * T[4 * c + 2];
    };
    posop[i] = make_uint2(pack2(f64_to_f16(md[0]), f64_to_f16(md[1])),
                          pack2(f64_to_f16(md[2]), (uint16_t)(po[u].y >> 16)));
    cov[3 * i] = pack2(f64_to_f16(sig(0, 0)), f64_to_f16(sig(0, 1)));
    cov[3 * i + 1] = pack2(f64_to_f16(sig(0, 2)), f64_to_f16(sig(1, 1)));
    cov[3 * i + 2] = pack2(f64_to_f16(sig(1, 2)), f64_to_f16(sig(2, 2)));
  }
}

}  // namespace

int packed_sh_stride(int degree) {
  switch (degree) {
    case 0: return ShPack<0>::S;
    case 1: return ShPack<1>::S;
    case 2: return ShPack<2>::S;
    case 3: return ShPack<3>::S;
    default: return -1;
  }
}

hipError_t launch_prepack(int n, const float* means, const float* log_scales, const float* quats,
                          const float* logits, const float* sh, int degree, uint16_t* posop,
                          uint16_t* cov, uint16_t* sh16, hipStream_t st) {
  if (n > 0) {
    trace_mark(st, "prepack");
    const dim3 grid((n + kBlock - 1) / kBlock);
    const float4* q4 = reinterpret_cast<const float4*>(quats);
    uint2* po = reinterpret_cast<uint2*>(posop);
    uint32_t* cv = reinterpret_cast<uint32_t*>(cov);
    uint2* s16 = reinterpret_cast<uint2*>(sh16);
#define GS_PP(D) hipLaunchKernelGGL(k_prepack<D>, grid, dim3(kBlock), 0, st, n, means, log_scales, q4, logits, sh, po, cv, s16)
    switch (degree) {
      case 0: GS_PP(0); break;
      case 1: GS_PP(1); break;
      case 2: GS_PP(2); break;
      default: GS_PP(3); break;
    }
#undef GS_PP
  }
  return hipGetLastError();
}

hipError_t launch_lbs(int n, const uint16_t* canon_posop, const uint16_t* canon_cov,
                      const uint8_t* joint_idx, const float* joint_w, int n_joints,
                      const float* joints, uint16_t* posop, uint16_t* cov, hipStream_t st) {
  if (n > 0) {
    trace_mark(st, "lbs");
    const int per_block = kBlock * kLbsItems;
    hipLaunchKernelGGL(k_lbs, dim3((n + per_block - 1) / per_block), dim3(kBlock), 0, st, n,
                       reinterpret_cast<const uint2*>(canon_posop),
                       reinterpret_cast<const uint32_t*>(canon_cov),
                       reinterpret_cast<const uint32_t*>(joint_idx),
                       reinterpret_cast<const float4*>(joint_w), n_joints, joints,
                       reinterpret_cast<uint2*>(posop), reinterpret_cast<uint32_t*>(cov));
  }
  return hipGetLastError();
}

hipError_t launch_preprocess_packed(int n, const uint16_t* posop, const uint16_t* cov,
                                    const uint16_t* sh16, int degree, const CamK& cam,
                                    const SetK& set, gs_splat* splats, uint32_t* depth_keys,
                                    uint32_t* tile_rects, uint4* partial, hipStream_t st) {
  const int blocks = preprocess_blocks(n);
  if (n > 0) {
    trace_mark(st, "preprocess_packed");
    const uint2* po = reinterpret_cast<const uint2*>(posop);
    const uint32_t* cv = reinterpret_cast<const uint32_t*>(cov);
    const uint2* s16 = reinterpret_cast<const uint2*>(sh16);
    uint2* tr = reinterpret_cast<uint2*>(tile_rects);
#define GS_PK(D) hipLaunchKernelGGL(k_preprocess_packed<D>, dim3(blocks), dim3(kBlock), 0, st, n, po, cv, s16, cam, set, splats, depth_keys, tr, partial)
    switch (degree) {
      case 0: GS_PK(0); break;
      case 1: GS_PK(1); break;
      case 2: GS_PK(2); break;
      default: GS_PK(3); break;
    }
#undef GS_PK
  }
  return hipGetLastError();
}

}  // namespace gs
