// Per-Gaussian preprocess (Section 3.2 Eq. 1, Algorithm 1's Preprocess
// procedure): activations, covariance from scale and rotation, per-model
// transform, camera transform, culls, EWA footprint, SH colour, tile rect.
//
// One thread per Gaussian, 256-thread blocks.  Every input attribute is an
// array of its own (means, log-scales, quaternions, logits, SH), so each
// wave reads contiguous spans; the SH rows are read only for Gaussians that
// survive the culls.
#include "gs_device.h"
#include "gs_internal.h"
#include "gs_project.h"

// The forward projection takes no implicit FMAs either (see gs_project.h):
// the one-view and the batch kernels must write bitwise-equal records.
#pragma float_control(push)
#pragma clang fp contract(off)

namespace gs {
namespace {

// rgb = sum_k sh_k Y_k + 1/2 for Gaussian i (before the clamp at 0).
template <int DEG>
__device__ __forceinline__ void sh_colour(const float* __restrict__ sh, int i, const float* Y,
                                          float* rgb) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  float acc[3] = {0.5f, 0.5f, 0.5f};
  if constexpr (DEG == 1 || DEG == 3) {
    // rows are 48 or 192 bytes: 16-byte aligned float4 loads
    const float4* row = reinterpret_cast<const float4*>(sh + (size_t)i * K * 3);
    float v[K * 3];
#pragma unroll
    for (int j = 0; j < K * 3 / 4; ++j) {
      const float4 f = row[j];
      v[4 * j] = f.x; v[4 * j + 1] = f.y; v[4 * j + 2] = f.z; v[4 * j + 3] = f.w;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      acc[0] = fmaf(v[3 * k], Y[k], acc[0]);
      acc[1] = fmaf(v[3 * k + 1], Y[k], acc[1]);
      acc[2] = fmaf(v[3 * k + 2], Y[k], acc[2]);
    }
  } else {
    const float* row = sh + (size_t)i * K * 3;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      acc[0] = fmaf(row[3 * k], Y[k], acc[0]);
      acc[1] = fmaf(row[3 * k + 1], Y[k], acc[1]);
      acc[2] = fmaf(row[3 * k + 2], Y[k], acc[2]);
    }
  }
  rgb[0] = acc[0]; rgb[1] = acc[1]; rgb[2] = acc[2];
}

// Eq. 1 and the colour for Gaussian i; fills its record r0..r2 and returns
// the number of tiles it touches (0 if culled).  With STAGED_SH the colour
// is left to the caller, which gets the SH view direction in dir[].
template <int DEG, bool STAGED_SH>
__device__ __forceinline__ uint32_t project_one(
    int i, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, const CamK& cam, const SetK& set, float4& r0, float4& r1,
    float4& r2, uint2& trect, float* dir) {
  const float4 q = quats[i];
  const float lg = logits[i];
  float w[3];
  double t[3];
  place_mean(means[3 * i], means[3 * i + 1], means[3 * i + 2], cam, w, t);
  const float tx = (float)t[0], ty = (float)t[1], tz = (float)t[2];

  const float o = 1.f / (1.f + expf(-lg));
  const float qn2 = q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w;

  r0 = make_float4(0.f, 0.f, 0.f, 0.f);
  r1 = r0;
  r2 = r0;
  uint32_t tiles = 0;
  // empty rects: x0 = 0xFFFF, y0 = 0 | x1 = 0, y1 = 0
  uint32_t rect_lo = 0x0000FFFFu, rect_hi = 0u;  // pixel bbox
  trect = make_uint2(0x0000FFFFu, 0u);            // tile rect

  const bool ok = (tz > cam.znear) && (o >= set.tau) && (qn2 > 0.f) &&
                  __builtin_isfinite(tx) && __builtin_isfinite(ty) && __builtin_isfinite(qn2);
  if (ok) {
    // Sigma = R diag(s^2) R^T; with N = T3 R diag(s), camera-space
    // covariance is N N^T and S = J N N^T J^T + eps I = M M^T + eps I.
    const float s0 = expf(log_scales[3 * i]), s1 = expf(log_scales[3 * i + 1]),
                s2 = expf(log_scales[3 * i + 2]);
    const float inv = 1.f / sqrtf(qn2);
    const float qw = q.x * inv, qx = q.y * inv, qy = q.z * inv, qz = q.w * inv;
    float R[9];
    R[0] = 1.f - 2.f * (qy * qy + qz * qz); R[1] = 2.f * (qx * qy - qw * qz); R[2] = 2.f * (qx * qz + qw * qy);
    R[3] = 2.f * (qx * qy + qw * qz); R[4] = 1.f - 2.f * (qx * qx + qz * qz); R[5] = 2.f * (qy * qz - qw * qx);
    R[6] = 2.f * (qx * qz - qw * qy); R[7] = 2.f * (qy * qz + qw * qx); R[8] = 1.f - 2.f * (qx * qx + qy * qy);
    float N[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        N[3 * r + c] = fmaf(cam.T3[3 * r], R[c], fmaf(cam.T3[3 * r + 1], R[3 + c], cam.T3[3 * r + 2] * R[6 + c]));
    N[0] *= s0; N[3] *= s0; N[6] *= s0;
    N[1] *= s1; N[4] *= s1; N[7] *= s1;
    N[2] *= s2; N[5] *= s2; N[8] *= s2;
    // Jacobian of the perspective division at t (x/z, y/z clamped)
    const float iz = 1.f / tz;
    const float xt = fminf(cam.limx, fmaxf(-cam.limx, tx * iz));
    const float yt = fminf(cam.limy, fmaxf(-cam.limy, ty * iz));
    const float j00 = cam.fx * iz, j02 = -cam.fx * xt * iz;
    const float j11 = cam.fy * iz, j12 = -cam.fy * yt * iz;
    float m0[3], m1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      m0[c] = fmaf(j00, N[c], j02 * N[6 + c]);
      m1[c] = fmaf(j11, N[3 + c], j12 * N[6 + c]);
    }
    const float aa = fmaf(m0[0], m0[0], fmaf(m0[1], m0[1], m0[2] * m0[2]));
    const float cc = fmaf(m1[0], m1[0], fmaf(m1[1], m1[1], m1[2] * m1[2]));
    const float b = fmaf(m0[0], m1[0], fmaf(m0[1], m1[1], m0[2] * m1[2]));
    // det S = |m0 x m1|^2 + eps (|m0|^2 + |m1|^2) + eps^2 (Cauchy-Binet):
    // a sum of non-negative terms, so no cancellation.
    const float x0 = det2(m0[1], m0[2], m1[1], m1[2]);
    const float x1 = det2(m0[2], m0[0], m1[2], m1[0]);
    const float x2 = det2(m0[0], m0[1], m1[0], m1[1]);
    const float D = fmaf(x0, x0, fmaf(x1, x1, x2 * x2)) +
                    set.eps2d * (aa + cc) + set.eps2d * set.eps2d;
    tiles = footprint(t, iz, w[0], w[1], w[2], aa + set.eps2d, b, cc + set.eps2d, D, o, cam,
                      set, r0, r1, rect_lo, rect_hi, trect, dir);
    if (!STAGED_SH && tiles) {
      float Y[16];
      sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
      float rgb[3];
      sh_colour<DEG>(sh, i, Y, rgb);
      r1.z = fmaxf(rgb[0], 0.f);
      r1.w = fmaxf(rgb[1], 0.f);
      r2.x = fmaxf(rgb[2], 0.f);
    }
  }
  r2.y = tz;
  r2.z = __uint_as_float(rect_lo);
  r2.w = __uint_as_float(rect_hi);
  return tiles;
}

// SH rows per wave staged through LDS at a time (half a wave's Gaussians).
constexpr int kShRows = 32;

// Record of Gaussian i and its depth sort key (float32 bits of the
// camera-space depth; the largest key when culled, so culled Gaussians sort
// last).  Each workgroup writes its tile and visible counts to its own
// slot of `partial`; k_count_finalize sums the slots.
//
// At SH degrees 1 and 3 a Gaussian's SH row is a whole number of 16-byte
// vectors (48 or 192 bytes).  Instead of each lane reading its own row (a
// wave-wide load then touches one 16-byte piece of each of 64 rows), the
// wave copies the rows of its visible Gaussians into LDS with contiguous
// 16-byte loads, 32 rows at a time, and each lane reads its row from LDS.
template <int DEG>
__device__ __forceinline__ void preprocess_block(
    int blk, int n, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, const CamK& cam, const SetK& set, gs_splat* __restrict__ splats,
    uint32_t* __restrict__ depth_keys, uint2* __restrict__ rects, uint4* __restrict__ partial) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  constexpr bool STAGED = DEG == 1 || DEG == 3;
  constexpr int F4 = STAGED ? K * 3 / 4 : 1;  // float4 per SH row
  __shared__ float4 s_sh[STAGED ? kBlock / 64 : 1][kShRows * F4];
  const int i = blk * kBlock + threadIdx.x;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t tiles = 0, dkey = 0xFFFFFFFFu;
  float4 r0, r1, r2;
  uint2 trect;
  float dir[3] = {0.f, 0.f, 0.f};
  if (i < n) {
    tiles = project_one<DEG, STAGED>(i, means, log_scales, quats, logits, sh, cam, set, r0, r1,
                                     r2, trect, dir);
    dkey = tiles ? __float_as_uint(r2.y) : 0xFFFFFFFFu;
    depth_keys[i] = dkey;
    rects[i] = trect;
  }
  if constexpr (STAGED) {
    const uint64_t need = ballot(tiles > 0);
    const int i0 = blk * kBlock + wave * 64;  // this wave's first Gaussian
    const float4* sh4 = reinterpret_cast<const float4*>(sh);
    float4* buf = s_sh[wave];
    // both halves' rows are read from HBM at once (one round trip per
    // wave), then staged through LDS half by half
    constexpr int LPH = (kShRows * F4 + 63) / 64;  // 16-byte loads per lane and half
    float4 pre[64 / kShRows][LPH];
#pragma unroll
    for (int h = 0; h < 64 / kShRows; ++h)
#pragma unroll
      for (int k = 0; k < LPH; ++k) {
        const int f = lane + 64 * k, row = f / F4;
        pre[h][k] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (f < kShRows * F4 && ((need >> (h * kShRows + row)) & 1ull))
          pre[h][k] = sh4[(size_t)(i0 + h * kShRows + row) * F4 + f % F4];
      }
#pragma unroll
    for (int h = 0; h < 64 / kShRows; ++h) {
#pragma unroll
      for (int k = 0; k < LPH; ++k) {
        const int f = lane + 64 * k;
        if (f < kShRows * F4) buf[f] = pre[h][k];
      }
      if (tiles > 0 && lane / kShRows == h) {
        const float4* rowp = buf + (lane - h * kShRows) * F4;
        float v[K * 3];
#pragma unroll
        for (int j = 0; j < F4; ++j) {
          const float4 q = rowp[j];
          v[4 * j] = q.x; v[4 * j + 1] = q.y; v[4 * j + 2] = q.z; v[4 * j + 3] = q.w;
        }
        float Y[16];
        sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
        float acc[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int k = 0; k < K; ++k) {
          acc[0] = fmaf(v[3 * k], Y[k], acc[0]);
          acc[1] = fmaf(v[3 * k + 1], Y[k], acc[1]);
          acc[2] = fmaf(v[3 * k + 2], Y[k], acc[2]);
        }
        r1.z = fmaxf(acc[0], 0.f);
        r1.w = fmaxf(acc[1], 0.f);
        r2.x = fmaxf(acc[2], 0.f);
      }
    }
  }
  if (i < n) {
    float4* dst = reinterpret_cast<float4*>(splats + i);
    dst[0] = r0;
    dst[1] = r1;
    dst[2] = r2;
  }
  block_counts(tiles, dkey, partial);
}

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_preprocess(
    int n, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, CamK cam, SetK set, gs_splat* __restrict__ splats,
    uint32_t* __restrict__ depth_keys, uint2* __restrict__ rects, uint4* __restrict__ partial) {
  preprocess_block<DEG>(blockIdx.x, n, means, log_scales, quats, logits, sh, cam, set, splats,
                        depth_keys, rects, partial);
}

// Every view of a batch and every asset in one launch: blockIdx.x runs over
// the assets' blocks (asset a owns blocks [B.block0[a], B.block0[a + 1])),
// blockIdx.y over chunks of kViewsPerBlock views, which the workgroup
// projects one after the other: its Gaussians' inputs come from HBM for the
// first view and from the cache for the others, instead of once per view.
// View v's records, depth keys and tile rects start at v * B.n; view v's
// partial counts of workgroup b go to slot v * B.block0[n_assets] + b.
// cams[v * n_assets + a] places asset a in view v.
template <int DEG>
// 4 waves per SIMD (124 VGPRs, no spill once the inputs are not kept live
// across the views; 194 VGPRs and 2 waves otherwise): 5.7 -> 5.4 ms per
// batch of 32 views x 4.5 M Gaussians.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_preprocess_views(
    BatchPreK B, int n_views, const float* __restrict__ means,
    const float* __restrict__ log_scales, const float4* __restrict__ quats,
    const float* __restrict__ logits, const float* __restrict__ sh,
    const CamK* __restrict__ cams, SetK set, gs_splat* __restrict__ splats,
    uint32_t* __restrict__ depth_keys, uint2* __restrict__ rects, uint4* __restrict__ partial) {
  constexpr int K3 = (DEG + 1) * (DEG + 1) * 3;
  const int b = blockIdx.x;
  int a = 0;
  while (a + 1 < B.n_assets && B.block0[a + 1] <= b) ++a;
  const int64_t o = B.offset[a];
  const int v0 = blockIdx.y * kViewsPerBlock;
  const int v1 = min(n_views, v0 + kViewsPerBlock);
  for (int v = v0; v < v1; ++v) {
    const int64_t vo = (int64_t)v * B.n + o;
    // opaque input pointers: each view reads its inputs again (from the
    // cache) instead of the compiler keeping them, and all that derives
    // from them, live across the views
    const float* m = means + 3 * o;
    const float* ls = log_scales + 3 * o;
    const float4* qt = quats + o;
    const float* lg = logits + o;
    asm volatile("" : "+s"(m), "+s"(ls), "+s"(qt), "+s"(lg));
    preprocess_block<DEG>(b - B.block0[a], B.count[a], m, ls, qt, lg, sh + K3 * o,
                          cams[v * B.n_assets + a], set,
                          splats + vo, depth_keys + vo, rects + vo,
                          partial + (size_t)v * B.block0[B.n_assets]);  // slot blockIdx.x
    __syncthreads();  // the next view reuses the LDS of this one
  }
}

#pragma float_control(pop)
#pragma float_control(push)

// counts[0] = total instances, counts[1] = visible Gaussians, counts[2] and
// counts[3] = the smallest and largest depth key of a visible Gaussian
// (all ones and 0 when none is visible).
__global__ __launch_bounds__(kBlock) void k_count_finalize(const uint4* __restrict__ partial,
                                                           int blocks, uint32_t* __restrict__ counts) {
  __shared__ uint32_t s_a[kBlock / 64], s_b[kBlock / 64], s_lo[kBlock / 64], s_hi[kBlock / 64];
  // 16 independent loads in flight per thread and step: one workgroup
  // reads tens of thousands of slots, so load latency, not bandwidth, rules
  constexpr int U = 16;
  uint32_t a = 0, b = 0, lo = 0xFFFFFFFFu, hi = 0u;
  for (int base = 0; base < blocks; base += kBlock * U) {
    // branch-free loads (past the end: the last slot, ignored), so that
    // all U are in flight together
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = partial[min(base + u * kBlock + (int)threadIdx.x, blocks - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (base + u * kBlock + (int)threadIdx.x < blocks) {
        a += v[u].x;
        b += v[u].y;
        lo = min(lo, v[u].z);
        hi = max(hi, v[u].w);
      }
    }
  }
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  a = wave_sum_u32(a);
  b = wave_sum_u32(b);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    lo = min(lo, shfl_u32(lo, lane ^ d));
    hi = max(hi, shfl_u32(hi, lane ^ d));
  }
  if (lane == 0) {
    s_a[wave] = a;
    s_b[wave] = b;
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ta = 0, tb = 0, tlo = 0xFFFFFFFFu, thi = 0u;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      ta += s_a[w];
      tb += s_b[w];
      tlo = min(tlo, s_lo[w]);
      thi = max(thi, s_hi[w]);
    }
    counts[0] = ta;
    counts[1] = tb;
    counts[2] = tlo;
    counts[3] = thi;
  }
}

// dY/d(x, y, z) of the basis above, accumulated against per-basis weights
// wk: returns sum_k wk[k] * grad Y_k.
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, const float* wk,
                                              float* g) {
  float gx = 0.f, gy = 0.f, gz = 0.f;
  if (DEG >= 1) {
    gy -= kC1 * wk[1];
    gz += kC1 * wk[2];
    gx -= kC1 * wk[3];
  }
  if (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    gx += kC2a * y * wk[4]; gy += kC2a * x * wk[4];
    gy -= kC2a * z * wk[5]; gz -= kC2a * y * wk[5];
    gx -= 2.f * kC2b * x * wk[6]; gy -= 2.f * kC2b * y * wk[6]; gz += 4.f * kC2b * z * wk[6];
    gx -= kC2a * z * wk[7]; gz -= kC2a * x * wk[7];
    gx += 2.f * kC2c * x * wk[8]; gy -= 2.f * kC2c * y * wk[8];
    if (DEG >= 3) {
      gx -= 6.f * kC3a * x * y * wk[9]; gy -= 3.f * kC3a * (xx - yy) * wk[9];
      gx += kC3b * y * z * wk[10]; gy += kC3b * x * z * wk[10]; gz += kC3b * x * y * wk[10];
      gx += 2.f * kC3c * x * y * wk[11]; gy -= kC3c * (4.f * zz - xx - 3.f * yy) * wk[11];
      gz -= 8.f * kC3c * y * z * wk[11];
      gx -= 6.f * kC3d * x * z * wk[12]; gy -= 6.f * kC3d * y * z * wk[12];
      gz += kC3d * (6.f * zz - 3.f * xx - 3.f * yy) * wk[12];
      gx -= kC3c * (4.f * zz - 3.f * xx - yy) * wk[13]; gy += 2.f * kC3c * x * y * wk[13];
      gz -= 8.f * kC3c * x * z * wk[13];
      gx += 2.f * kC3e * x * z * wk[14]; gy -= 2.f * kC3e * y * z * wk[14];
      gz += kC3e * (xx - yy) * wk[14];
      gx -= 3.f * kC3a * (xx - yy) * wk[15]; gy += 6.f * kC3a * x * y * wk[15];
    }
  }
  g[0] = gx; g[1] = gy; g[2] = gz;
}

// Chain rule for Gaussian i under one camera: from its 2-D gradient record
// G = d(mean2d, qa, qb, qc, opacity, rgb) back to the raw inputs,
// recomputing the forward quantities; the input gradients are added to
// gp, gls, gq, glogit and gsh.
template <int DEG>
__device__ __forceinline__ void chain_one(
    int i, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, const CamK& cam, const SetK& set, const float* G, float* gp,
    float* gls, float* gq, float& glogit, float* gsh) {
  constexpr int K = (DEG + 1) * (DEG + 1);
    const float gmx = G[0], gmy = G[1], gqa = G[2], gqb = G[3], gqc = G[4], gop = G[5];
  const float grgb[3] = {G[6], G[7], G[8]};

  // ---- recompute the forward quantities
  const float p0 = means[3 * i], p1 = means[3 * i + 1], p2 = means[3 * i + 2];
  const float4 q = quats[i];
  const float lg = logits[i];
  float w0 = p0, w1 = p1, w2 = p2;
  if (cam.has_model) {
    w0 = fmaf(cam.A[0], p0, fmaf(cam.A[1], p1, fmaf(cam.A[2], p2, cam.A[3])));
    w1 = fmaf(cam.A[4], p0, fmaf(cam.A[5], p1, fmaf(cam.A[6], p2, cam.A[7])));
    w2 = fmaf(cam.A[8], p0, fmaf(cam.A[9], p1, fmaf(cam.A[10], p2, cam.A[11])));
  }
  const float tx = fmaf(cam.V[0], w0, fmaf(cam.V[1], w1, fmaf(cam.V[2], w2, cam.V[3])));
  const float ty = fmaf(cam.V[4], w0, fmaf(cam.V[5], w1, fmaf(cam.V[6], w2, cam.V[7])));
  const float tz = fmaf(cam.V[8], w0, fmaf(cam.V[9], w1, fmaf(cam.V[10], w2, cam.V[11])));
  const float o = 1.f / (1.f + expf(-lg));
  const float s[3] = {expf(log_scales[3 * i]), expf(log_scales[3 * i + 1]),
                      expf(log_scales[3 * i + 2])};
  const float qn2 = q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w;
  const float inv = 1.f / sqrtf(qn2);
  const float qw = q.x * inv, qx = q.y * inv, qy = q.z * inv, qz = q.w * inv;
  float R[9];
  R[0] = 1.f - 2.f * (qy * qy + qz * qz); R[1] = 2.f * (qx * qy - qw * qz); R[2] = 2.f * (qx * qz + qw * qy);
  R[3] = 2.f * (qx * qy + qw * qz); R[4] = 1.f - 2.f * (qx * qx + qz * qz); R[5] = 2.f * (qy * qz - qw * qx);
  R[6] = 2.f * (qx * qz - qw * qy); R[7] = 2.f * (qy * qz + qw * qx); R[8] = 1.f - 2.f * (qx * qx + qy * qy);
  float P[9];  // T3 R
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      P[3 * r + c] = fmaf(cam.T3[3 * r], R[c], fmaf(cam.T3[3 * r + 1], R[3 + c], cam.T3[3 * r + 2] * R[6 + c]));
  float N[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) N[3 * r + c] = P[3 * r + c] * s[c];
  const float iz = 1.f / tz;
  const float xr = tx * iz, yr = ty * iz;
  const bool xclamp = xr < -cam.limx || xr > cam.limx;
  const bool yclamp = yr < -cam.limy || yr > cam.limy;
  const float xt = fminf(cam.limx, fmaxf(-cam.limx, xr));
  const float yt = fminf(cam.limy, fmaxf(-cam.limy, yr));
  const float j00 = cam.fx * iz, j02 = -cam.fx * xt * iz;
  const float j11 = cam.fy * iz, j12 = -cam.fy * yt * iz;
  float m0[3], m1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    m0[c] = fmaf(j00, N[c], j02 * N[6 + c]);
    m1[c] = fmaf(j11, N[3 + c], j12 * N[6 + c]);
  }
  const float aa = fmaf(m0[0], m0[0], fmaf(m0[1], m0[1], m0[2] * m0[2]));
  const float cc = fmaf(m1[0], m1[0], fmaf(m1[1], m1[1], m1[2] * m1[2]));
  const float b = fmaf(m0[0], m1[0], fmaf(m0[1], m1[1], m0[2] * m1[2]));
  const float c = cc + set.eps2d;
  const float x0 = det2(m0[1], m0[2], m1[1], m1[2]);
  const float x1 = det2(m0[2], m0[0], m1[2], m1[0]);
  const float x2 = det2(m0[0], m0[1], m1[0], m1[1]);
  const float D = fmaf(x0, x0, fmaf(x1, x1, x2 * x2)) +
                  set.eps2d * (aa + cc) + set.eps2d * set.eps2d;
  const float qa = c / D, qb = b / c, qc = 1.f / c;

  // ---- colour: rgb = max(0, sum_k sh_k Y_k(dl) + 1/2)
  float v0 = w0 - cam.campos[0], v1 = w1 - cam.campos[1], v2 = w2 - cam.campos[2];
  const float vn = sqrtf(v0 * v0 + v1 * v1 + v2 * v2);
  const float ivn = 1.f / vn;
  const float d0 = v0 * ivn, d1 = v1 * ivn, d2 = v2 * ivn;
  float e0 = d0, e1 = d1, e2 = d2;
  if (cam.has_model) {
    e0 = cam.Rk[0] * d0 + cam.Rk[3] * d1 + cam.Rk[6] * d2;
    e1 = cam.Rk[1] * d0 + cam.Rk[4] * d1 + cam.Rk[7] * d2;
    e2 = cam.Rk[2] * d0 + cam.Rk[5] * d1 + cam.Rk[8] * d2;
  }
  float Y[16];
  sh_basis<DEG>(e0, e1, e2, Y);
  float rgb[3];
  sh_colour<DEG>(sh, i, Y, rgb);
  float graw[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) graw[ch] = rgb[ch] > 0.f ? grgb[ch] : 0.f;
  float wk[16];
  const float* shrow = sh + (size_t)i * K * 3;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    gsh[3 * k] += graw[0] * Y[k];
    gsh[3 * k + 1] += graw[1] * Y[k];
    gsh[3 * k + 2] += graw[2] * Y[k];
    wk[k] = graw[0] * shrow[3 * k] + graw[1] * shrow[3 * k + 1] + graw[2] * shrow[3 * k + 2];
  }
  float gdl[3];
  sh_basis_grad<DEG>(e0, e1, e2, wk, gdl);
  float gd0 = gdl[0], gd1 = gdl[1], gd2 = gdl[2];
  if (cam.has_model) {  // dl = Rk^T d  ->  dL/dd = Rk dL/ddl
    gd0 = cam.Rk[0] * gdl[0] + cam.Rk[1] * gdl[1] + cam.Rk[2] * gdl[2];
    gd1 = cam.Rk[3] * gdl[0] + cam.Rk[4] * gdl[1] + cam.Rk[5] * gdl[2];
    gd2 = cam.Rk[6] * gdl[0] + cam.Rk[7] * gdl[1] + cam.Rk[8] * gdl[2];
  }
  const float dd = gd0 * d0 + gd1 * d1 + gd2 * d2;
  float gw[3] = {(gd0 - dd * d0) * ivn, (gd1 - dd * d1) * ivn, (gd2 - dd * d2) * ivn};

  // ---- opacity
  glogit += gop * o * (1.f - o);

  // ---- (qa, qb, qc) -> S = [[a, b], [b, c]]
  const float ga = -gqa * qa * qa;
  const float gb = 2.f * gqa * qa * qa * qb + gqb * qc;
  const float gc = -gqa * qa * qa * qb * qb - gqb * qb * qc - gqc * qc * qc;
  // ---- S = M M^T + eps I
  float gm0[3], gm1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gm0[k] = 2.f * ga * m0[k] + gb * m1[k];
    gm1[k] = gb * m0[k] + 2.f * gc * m1[k];
  }
  // ---- M = J N  (rows m0 = j00 N0 + j02 N2, m1 = j11 N1 + j12 N2)
  float gj00 = 0.f, gj02 = 0.f, gj11 = 0.f, gj12 = 0.f;
  float gN[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gj00 += gm0[k] * N[k];
    gj02 += gm0[k] * N[6 + k];
    gj11 += gm1[k] * N[3 + k];
    gj12 += gm1[k] * N[6 + k];
    gN[k] = j00 * gm0[k];
    gN[3 + k] = j11 * gm1[k];
    gN[6 + k] = j02 * gm0[k] + j12 * gm1[k];
  }
  // ---- N = P diag(s), P = T3 R
  float gR[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float gs = gN[c] * P[c] + gN[3 + c] * P[3 + c] + gN[6 + c] * P[6 + c];
    gls[c] += gs * s[c];
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)  // dL/dR_rc = sum_i T3_ir gP_ic, gP_ic = gN_ic s_c
      gR[3 * r + c] = (cam.T3[r] * gN[c] + cam.T3[3 + r] * gN[3 + c] + cam.T3[6 + r] * gN[6 + c]) * s[c];
  // ---- R(q^) -> q^
  const float gqw = 2.f * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
  const float gqx = 2.f * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.f * qx * gR[4] - qw * gR[5] +
                           qz * gR[6] + qw * gR[7] - 2.f * qx * gR[8]);
  const float gqy = 2.f * (-2.f * qy * gR[0] + qx * gR[1] + qw * gR[2] + qx * gR[3] + qz * gR[5] -
                           qw * gR[6] + qz * gR[7] - 2.f * qy * gR[8]);
  const float gqz = 2.f * (-2.f * qz * gR[0] - qw * gR[1] + qx * gR[2] + qw * gR[3] - 2.f * qz * gR[4] +
                           qy * gR[5] + qx * gR[6] + qy * gR[7]);
  // ---- normalisation q^ = q/|q|
  const float qd = gqw * qw + gqx * qx + gqy * qy + gqz * qz;
  gq[0] += (gqw - qd * qw) * inv;
  gq[1] += (gqx - qd * qx) * inv;
  gq[2] += (gqy - qd * qy) * inv;
  gq[3] += (gqz - qd * qz) * inv;
  // ---- J and mean2d -> camera-space t
  const float iz2 = iz * iz;
  float gtx = gmx * cam.fx * iz, gty = gmy * cam.fy * iz;
  float gtz = -(gmx * cam.fx * tx + gmy * cam.fy * ty) * iz2;
  gtz += -gj00 * cam.fx * iz2 - gj11 * cam.fy * iz2;
  if (xclamp) {
    gtz += gj02 * cam.fx * xt * iz2;
  } else {
    gtx += -gj02 * cam.fx * iz2;
    gtz += 2.f * gj02 * cam.fx * tx * iz2 * iz;
  }
  if (yclamp) {
    gtz += gj12 * cam.fy * yt * iz2;
  } else {
    gty += -gj12 * cam.fy * iz2;
    gtz += 2.f * gj12 * cam.fy * ty * iz2 * iz;
  }
  // ---- t = V w + v  ->  w; w = A p + t_k  ->  p
#pragma unroll
  for (int k = 0; k < 3; ++k) gw[k] += cam.V[k] * gtx + cam.V[4 + k] * gty + cam.V[8 + k] * gtz;
  if (cam.has_model) {
#pragma unroll
    for (int k = 0; k < 3; ++k) gp[k] += cam.A[k] * gw[0] + cam.A[4 + k] * gw[1] + cam.A[8 + k] * gw[2];
  } else {
    gp[0] += gw[0]; gp[1] += gw[1]; gp[2] += gw[2];
  }
}

// Chain rule from the 2-D gradient record d(mean2d, qa, qb, qc, opacity,
// rgb) back to the raw inputs, recomputing the forward quantities.
template <int DEG>
__global__ __launch_bounds__(kBlock) void k_preprocess_bwd(
    int n, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, CamK cam, SetK set, const gs_splat* __restrict__ splats,
    const float* __restrict__ grad2d, float* __restrict__ d_means,
    float* __restrict__ d_log_scales, float4* __restrict__ d_quats,
    float* __restrict__ d_logits, float* __restrict__ d_sh, int accumulate) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float gp[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
  float glogit = 0.f;
  float gsh[K * 3];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) gsh[k] = 0.f;

  const float4 r2 = reinterpret_cast<const float4*>(splats + i)[2];
  const uint32_t rl = __float_as_uint(r2.z), rh = __float_as_uint(r2.w);
  const bool visible = (rh & 0xFFFFu) >= (rl & 0xFFFFu);
  // a culled Gaussian's gradient is zero: adding it changes nothing
  if (accumulate && !visible) return;
  if (visible) {
    chain_one<DEG>(i, means, log_scales, quats, logits, sh, cam, set,
                   grad2d + (size_t)i * kGrad2dStride, gp, gls, gq, glogit, gsh);
  }

  if (accumulate) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d_means[3 * i + k] += gp[k];
      d_log_scales[3 * i + k] += gls[k];
    }
    float4 dq = d_quats[i];
    dq.x += gq[0]; dq.y += gq[1]; dq.z += gq[2]; dq.w += gq[3];
    d_quats[i] = dq;
    d_logits[i] += glogit;
#pragma unroll
    for (int k = 0; k < K * 3; ++k) d_sh[(size_t)i * K * 3 + k] += gsh[k];
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d_means[3 * i + k] = gp[k];
      d_log_scales[3 * i + k] = gls[k];
    }
    d_quats[i] = make_float4(gq[0], gq[1], gq[2], gq[3]);
    d_logits[i] = glogit;
#pragma unroll
    for (int k = 0; k < K * 3; ++k) d_sh[(size_t)i * K * 3 + k] = gsh[k];
  }
}

// The same chain rule for several views at once: per Gaussian the inputs
// are read once, the chain runs for every view whose 2-D gradient record
// is non-zero (a view that culled the Gaussian, or to whose pixels it
// contributed nothing, has an all-zero record), and the input gradients
// are written, or added, once.  Compared with one backward per view, the
// 236-byte gradient of a degree-3 Gaussian is read and written once per
// kBwdViews views instead of once per view.
template <int DEG>
// 3 waves per SIMD: the 59 gradient accumulators stay live across the
// views, the inputs are read again per view (opaque pointers); 181 VGPRs
// and 2 waves otherwise (5.9 -> 5.5 ms per batch of 32 views x 4.5 M).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_preprocess_bwd_views(
    int n, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float4* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, ViewsK views, SetK set, float* __restrict__ d_means,
    float* __restrict__ d_log_scales, float4* __restrict__ d_quats,
    float* __restrict__ d_logits, float* __restrict__ d_sh, int accumulate) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float gp[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
  float glogit = 0.f;
  float gsh[K * 3];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) gsh[k] = 0.f;
  bool any = false;
  for (int v = 0; v < views.nv; ++v) {
    const float4* row = reinterpret_cast<const float4*>(views.g2d[v] + (size_t)i * kGrad2dStride);
    const float4 a = row[0], b = row[1];
    const float c = row[2].x;
    const float G[9] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c};
    bool nz = false;
#pragma unroll
    for (int k = 0; k < 9; ++k) nz = nz || G[k] != 0.f;
    if (!nz) continue;
    any = true;
    // opaque input pointers: read again per view rather than kept live
    const float* m = means;
    const float* ls = log_scales;
    const float4* qt = quats;
    const float* lg = logits;
    const float* shp = sh;
    asm volatile("" : "+s"(m), "+s"(ls), "+s"(qt), "+s"(lg), "+s"(shp));
    chain_one<DEG>(i, m, ls, qt, lg, shp, views.cam[v], set, G, gp, gls, gq, glogit, gsh);
  }
  if (accumulate && !any) return;
  if (accumulate) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d_means[3 * i + k] += gp[k];
      d_log_scales[3 * i + k] += gls[k];
    }
    float4 dq = d_quats[i];
    dq.x += gq[0]; dq.y += gq[1]; dq.z += gq[2]; dq.w += gq[3];
    d_quats[i] = dq;
    d_logits[i] += glogit;
#pragma unroll
    for (int k = 0; k < K * 3; ++k) d_sh[(size_t)i * K * 3 + k] += gsh[k];
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d_means[3 * i + k] = gp[k];
      d_log_scales[3 * i + k] = gls[k];
    }
    d_quats[i] = make_float4(gq[0], gq[1], gq[2], gq[3]);
    d_logits[i] = glogit;
#pragma unroll
    for (int k = 0; k < K * 3; ++k) d_sh[(size_t)i * K * 3 + k] = gsh[k];
  }
}

}  // namespace

int preprocess_blocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// one partial slot per block of every asset: at most blocks(n) + assets
size_t preprocess_ws_bytes(int64_t n) {
  return align_up((size_t)(preprocess_blocks(n) + kMaxAssets) * 16, 256);
}

hipError_t launch_preprocess(int n, const float* means, const float* log_scales,
                             const float* quats, const float* logits, const float* sh,
                             int degree, const CamK& cam, const SetK& set,
                             gs_splat* splats, uint32_t* depth_keys, uint32_t* tile_rects,
                             uint4* partial, hipStream_t st) {
  const int blocks = preprocess_blocks(n);
  if (n > 0) {
    trace_mark(st, "preprocess");
    const float4* q4 = reinterpret_cast<const float4*>(quats);
#define GS_PRE(D) hipLaunchKernelGGL(k_preprocess<D>, dim3(blocks), dim3(kBlock), 0, st, n, means, log_scales, q4, logits, sh, cam, set, splats, depth_keys, reinterpret_cast<uint2*>(tile_rects), partial)
    switch (degree) {
      case 0: GS_PRE(0); break;
      case 1: GS_PRE(1); break;
      case 2: GS_PRE(2); break;
      default: GS_PRE(3); break;
    }
#undef GS_PRE
  }
  return hipGetLastError();
}

hipError_t launch_preprocess_views(const BatchPreK& B, int n_views, const float* means,
                                   const float* log_scales, const float* quats,
                                   const float* logits, const float* sh, int degree,
                                   const CamK* cams, const SetK& set, gs_splat* splats,
                                   uint32_t* depth_keys, uint32_t* tile_rects, uint4* partial,
                                   hipStream_t st) {
  const int blocks = B.block0[B.n_assets];
  if (blocks > 0 && n_views > 0) {
    trace_mark(st, "preprocess_views");
    const float4* q4 = reinterpret_cast<const float4*>(quats);
    const int chunks = (n_views + kViewsPerBlock - 1) / kViewsPerBlock;
#define GS_PREV(D) hipLaunchKernelGGL(k_preprocess_views<D>, dim3(blocks, chunks), dim3(kBlock), 0, st, B, n_views, means, log_scales, q4, logits, sh, cams, set, splats, depth_keys, reinterpret_cast<uint2*>(tile_rects), partial)
    switch (degree) {
      case 0: GS_PREV(0); break;
      case 1: GS_PREV(1); break;
      case 2: GS_PREV(2); break;
      default: GS_PREV(3); break;
    }
#undef GS_PREV
  }
  return hipGetLastError();
}

hipError_t launch_count_finalize(const uint4* partial, int blocks, uint32_t* counts,
                                 hipStream_t st) {
  trace_mark(st, "count_finalize");
  hipLaunchKernelGGL(k_count_finalize, dim3(1), dim3(kBlock), 0, st, partial, blocks, counts);
  return hipGetLastError();
}

hipError_t launch_preprocess_backward(int n, const float* means, const float* log_scales,
                                      const float* quats, const float* logits, const float* sh,
                                      int degree, const CamK& cam, const SetK& set,
                                      const gs_splat* splats, const float* grad2d,
                                      float* d_means, float* d_log_scales, float* d_quats,
                                      float* d_logits, float* d_sh, int accumulate,
                                      hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 grid((n + kBlock - 1) / kBlock), block(kBlock);
  const float4* q4 = reinterpret_cast<const float4*>(quats);
  float4* dq4 = reinterpret_cast<float4*>(d_quats);
#define GS_PBWD(D) hipLaunchKernelGGL(k_preprocess_bwd<D>, grid, block, 0, st, n, means, log_scales, q4, logits, sh, cam, set, splats, grad2d, d_means, d_log_scales, dq4, d_logits, d_sh, accumulate)
  switch (degree) {
    case 0: GS_PBWD(0); break;
    case 1: GS_PBWD(1); break;
    case 2: GS_PBWD(2); break;
    default: GS_PBWD(3); break;
  }
#undef GS_PBWD
  return hipGetLastError();
}

hipError_t launch_preprocess_backward_views(int n, const float* means, const float* log_scales,
                                            const float* quats, const float* logits,
                                            const float* sh, int degree, const ViewsK& views,
                                            const SetK& set, float* d_means, float* d_log_scales,
                                            float* d_quats, float* d_logits, float* d_sh,
                                            int accumulate, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const dim3 grid((n + kBlock - 1) / kBlock), block(kBlock);
  const float4* q4 = reinterpret_cast<const float4*>(quats);
  float4* dq4 = reinterpret_cast<float4*>(d_quats);
#define GS_PBWDV(D) hipLaunchKernelGGL(k_preprocess_bwd_views<D>, grid, block, 0, st, n, means, log_scales, q4, logits, sh, views, set, d_means, d_log_scales, dq4, d_logits, d_sh, accumulate)
  switch (degree) {
    case 0: GS_PBWDV(0); break;
    case 1: GS_PBWDV(1); break;
    case 2: GS_PBWDV(2); break;
    default: GS_PBWDV(3); break;
  }
#undef GS_PBWDV
  return hipGetLastError();
}

}  // namespace gs

#pragma float_control(pop)
