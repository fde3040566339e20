// Device helpers shared by the raw-parameter and pre-packed preprocess
// kernels: the real SH basis, the camera placement of a mean and the
// common tail of the projection (Section 3.2 Eq. 1, Algorithm 1's
// Preprocess procedure).
#pragma once

#include "gs_device.h"
#include "gs_internal.h"

// No implicit fusion of a multiply and an add into an FMA in the projection
// (the FMAs it wants are written out): which products the compiler would
// fuse depends on the code around the inlined functions (a loop over views
// hoists the view-independent products out of the loop body, where they
// cannot fuse), and a record must not depend on the kernel that computed it.
#pragma float_control(push)
#pragma clang fp contract(off)

namespace gs {

// Real SH normalisation constants (degree <= 3), with the sign of the
// Condon-Shortley phase folded in; each is the closed form noted beside it.
constexpr float kC0 = 0.28209479177387814f;   // 1/2 sqrt(1/pi)
constexpr float kC1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
constexpr float kC2a = 1.0925484305920792f;   // 1/2 sqrt(15/pi)
constexpr float kC2b = 0.31539156525252005f;  // 1/4 sqrt(5/pi)
constexpr float kC2c = 0.54627421529603959f;  // 1/4 sqrt(15/pi)
constexpr float kC3a = 0.59004358992664352f;  // 1/4 sqrt(35/(2 pi))
constexpr float kC3b = 2.8906114426405538f;   // 1/2 sqrt(105/pi)
constexpr float kC3c = 0.45704579946446572f;  // 1/4 sqrt(21/(2 pi))
constexpr float kC3d = 0.37317633259011540f;  // 1/4 sqrt(7/pi)
constexpr float kC3e = 1.4453057213202769f;   // 1/4 sqrt(105/pi)

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kC0;
  if (DEG >= 1) {
    Y[1] = -kC1 * y;
    Y[2] = kC1 * z;
    Y[3] = -kC1 * x;
  }
  if (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kC2a * x * y;
    Y[5] = -kC2a * y * z;
    Y[6] = kC2b * (2.f * zz - xx - yy);
    Y[7] = -kC2a * x * z;
    Y[8] = kC2c * (xx - yy);
    if (DEG >= 3) {
      Y[9] = -kC3a * y * (3.f * xx - yy);
      Y[10] = kC3b * x * y * z;
      Y[11] = -kC3c * y * (4.f * zz - xx - yy);
      Y[12] = kC3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
      Y[13] = -kC3c * x * (4.f * zz - xx - yy);
      Y[14] = kC3e * z * (xx - yy);
      Y[15] = -kC3a * x * (xx - 3.f * yy);
    }
  }
}

// Shared tail of the projection.  From the camera-space mean t (float64;
// 1/t_z in iz), the world-space mean w, the 2-D covariance S = [[a, b],
// [b, c]] (eps2d included) with determinant D and the opacity o: the 2-D
// mean, the whitened form, the opacity-aware pixel bbox and tile rect (r0,
// r1.xy, rect_lo/hi, trect) and the unit view direction for the colour, in
// the asset's frame.  Returns the number of tiles touched (0: nothing
// drawn).
//
// The 2-D mean is formed in float64 and stored relative to the pixel bbox's
// top-left corner (px0, py0): a pixel's offset from the mean is then an
// exact small integer minus a float32 fraction, accurate to ~1e-7 px
// anywhere in the image instead of the ~1e-4 px that a float32 absolute
// position carries at x ~ 2000 (which moves the weight near alpha_min by
// ~1e-4 relative for sharp splats).
__device__ __forceinline__ uint32_t footprint(const double* t, float iz, float w0, float w1,
                                              float w2, float a, float b, float c, float D,
                                              float o, const CamK& cam, const SetK& set,
                                              float4& r0, float4& r1, uint32_t& rect_lo,
                                              uint32_t& rect_hi, uint2& trect, float* dir) {
  const double mxd = (double)cam.fx * (t[0] / t[2]) + (double)cam.cx;
  const double myd = (double)cam.fy * (t[1] / t[2]) + (double)cam.cy;
  const bool ok = D > 0.f && c > 0.f && __builtin_isfinite(D) && __builtin_isfinite(a) &&
                  __builtin_isfinite(mxd) && __builtin_isfinite(myd) && fabs(mxd) < 1e9 &&
                  fabs(myd) < 1e9;
  if (!ok) return 0;
  const float qa = c / D, qb = b / c, qc = 1.f / c;
  // Opacity-aware bbox: o exp(-Q/2) >= tau inside the ellipse
  // Q <= 2 ln(o/tau), whose bbox half-extents are sqrt(qmax a),
  // sqrt(qmax c).  Inflated slightly so that rounding can only add
  // tiles (an added tile holds no pixel with weight >= tau).
  const float qmax = 2.f * (logf(o) - logf(set.tau));
  const double rx = (double)(sqrtf(qmax * a) * (1.f + 1e-5f) + 1e-3f);
  const double ry = (double)(sqrtf(qmax * c) * (1.f + 1e-5f) + 1e-3f);
  double fx0 = ceil(mxd - rx - 0.5), fx1 = floor(mxd + rx - 0.5);
  double fy0 = ceil(myd - ry - 0.5), fy1 = floor(myd + ry - 0.5);
  fx0 = fmax(fx0, 0.0); fy0 = fmax(fy0, 0.0);
  fx1 = fmin(fx1, (double)(cam.W - 1)); fy1 = fmin(fy1, (double)(cam.H - 1));
  if (!(fx0 <= fx1 && fy0 <= fy1)) return 0;
  const int px0 = (int)fx0, px1 = (int)fx1, py0 = (int)fy0, py1 = (int)fy1;
  // tile of a pixel: the tile sides are powers of 2 and the pixel bbox is
  // clamped to the image, so a shift is the division
  const int tx0 = px0 >> set.tile_w_shift, tx1 = px1 >> set.tile_w_shift;
  const int ty0 = (py0 >> set.tile_h_shift) + cam.tile_row;
  const int ty1 = (py1 >> set.tile_h_shift) + cam.tile_row;
  rect_lo = (uint32_t)px0 | ((uint32_t)py0 << 16);
  rect_hi = (uint32_t)px1 | ((uint32_t)py1 << 16);
  trect = make_uint2((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)tx1 | ((uint32_t)ty1 << 16));
  // view direction for the colour, in the asset's frame
  float d0 = w0 - cam.campos[0], d1 = w1 - cam.campos[1], d2 = w2 - cam.campos[2];
  const float dn = 1.f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
  d0 *= dn; d1 *= dn; d2 *= dn;
  if (cam.has_model) {
    const float e0 = cam.Rk[0] * d0 + cam.Rk[3] * d1 + cam.Rk[6] * d2;
    const float e1 = cam.Rk[1] * d0 + cam.Rk[4] * d1 + cam.Rk[7] * d2;
    const float e2 = cam.Rk[2] * d0 + cam.Rk[5] * d1 + cam.Rk[8] * d2;
    d0 = e0; d1 = e1; d2 = e2;
  }
  r0 = make_float4((float)(mxd - fx0), (float)(myd - fy0), qa, qb);
  r1 = make_float4(qc, o, 0.f, 0.f);
  dir[0] = d0; dir[1] = d1; dir[2] = d2;
  return (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
}

// Asset-to-world (Algorithm 1's M_k) and world-to-camera transforms of a
// mean.  The camera-space mean t is formed in float64: its float32 rounding
// is the depth sort key (so keys are correctly rounded depths), and the 2-D
// mean is projected from it.  w (the world mean, for the SH view
// direction) is float32.
__device__ __forceinline__ void place_mean(float p0, float p1, float p2, const CamK& cam,
                                           float* w, double* t) {
  double w0 = p0, w1 = p1, w2 = p2;
  if (cam.has_model) {
    w0 = fma((double)cam.A[0], (double)p0, fma((double)cam.A[1], (double)p1,
             fma((double)cam.A[2], (double)p2, (double)cam.A[3])));
    w1 = fma((double)cam.A[4], (double)p0, fma((double)cam.A[5], (double)p1,
             fma((double)cam.A[6], (double)p2, (double)cam.A[7])));
    w2 = fma((double)cam.A[8], (double)p0, fma((double)cam.A[9], (double)p1,
             fma((double)cam.A[10], (double)p2, (double)cam.A[11])));
  }
  w[0] = (float)w0; w[1] = (float)w1; w[2] = (float)w2;
  t[0] = fma((double)cam.V[0], w0, fma((double)cam.V[1], w1, fma((double)cam.V[2], w2, (double)cam.V[3])));
  t[1] = fma((double)cam.V[4], w0, fma((double)cam.V[5], w1, fma((double)cam.V[6], w2, (double)cam.V[7])));
  t[2] = fma((double)cam.V[8], w0, fma((double)cam.V[9], w1, fma((double)cam.V[10], w2, (double)cam.V[11])));
}

// Each workgroup's (instances, visible) totals into its slot of `partial`
// (summed later by k_count_finalize); tiles = this thread's tile count.
__device__ __forceinline__ void block_counts(uint32_t tiles, uint32_t dkey, uint4* __restrict__ partial) {
  __shared__ uint32_t s_vis[kBlock / 64], s_til[kBlock / 64], s_min[kBlock / 64], s_max[kBlock / 64];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const uint32_t wv = (uint32_t)__builtin_popcountll(ballot(tiles > 0));
  const uint32_t wt = wave_sum_u32(tiles);
  // depth key range of the visible Gaussians (culled keys are all ones)
  uint32_t kmin = dkey, kmax = tiles > 0 ? dkey : 0u;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    kmin = min(kmin, shfl_u32(kmin, lane ^ d));
    kmax = max(kmax, shfl_u32(kmax, lane ^ d));
  }
  if (lane == 0) {
    s_vis[wave] = wv;
    s_til[wave] = wt;
    s_min[wave] = kmin;
    s_max[wave] = kmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t bv = 0, bt = 0, bmin = 0xFFFFFFFFu, bmax = 0u;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      bv += s_vis[w];
      bt += s_til[w];
      bmin = min(bmin, s_min[w]);
      bmax = max(bmax, s_max[w]);
    }
    partial[blockIdx.x] = make_uint4(bt, bv, bmin, bmax);
  }
}

}  // namespace gs

#pragma float_control(pop)
