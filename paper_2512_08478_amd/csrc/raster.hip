// Tile compositing (Section 3.2 Eqs. 2-3) forward and backward.
//
// One workgroup per tile, one thread per pixel.  The tile's splats (already
// in (depth, index) order) are staged through LDS in batches of one record
// per thread; every pixel walks the batch front to back.  A pixel stops
// after the blend that takes its transmittance below t_eps; a wave whose
// 64 pixels have all stopped skips the batch loop, and the workgroup leaves
// once every pixel has stopped.
//
// Tiles are assigned XCD-major: the hardware deals consecutive workgroups
// round-robin to the 8 XCDs, so workgroup b works on tile
// (b % 8) * ceil(tiles/8) + b / 8 and each XCD's L2 sees one contiguous band
// of tiles, whose splats it shares.
#include "gs_device.h"
#include "gs_internal.h"

namespace gs {
namespace {

constexpr float kHalfLog2e = 0.72134752044448170f;  // log2(e) / 2
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_tile(int b, int tiles) {
  const int chunk = (tiles + kXcds - 1) / kXcds;
  return (b % kXcds) * chunk + b / kXcds;
}

inline int xcd_grid(int tiles) { return ((tiles + kXcds - 1) / kXcds) * kXcds; }

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_raster(const gs_splat* __restrict__ splats,
                                                   const uint32_t* __restrict__ values,
                                                   const uint32_t* __restrict__ ranges,
                                                   SetK set, int W, int H,
                                                   float* __restrict__ image,
                                                   float* __restrict__ T_final,
                                                   uint32_t* __restrict__ last) {
  constexpr int NT = TW * TH;
  __shared__ float4 s_a[NT];  // mean_x, mean_y, qa*log2e/2, qb
  __shared__ float4 s_b[NT];  // qc*log2e/2, log2(opacity), r, g
  __shared__ float s_c[NT];   // b
  const int tiles = set.tiles_x * set.tiles_y;
  const int tile = xcd_tile(blockIdx.x, tiles);
  if (tile >= tiles) return;
  const int tid = threadIdx.x;
  const int px = (tile % set.tiles_x) * TW + tid % TW;
  const int py = (tile / set.tiles_x) * TH + tid / TW;
  const bool inside = px < W && py < H;
  const float fx = px + 0.5f, fy = py + 0.5f;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];

  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  uint32_t lastc = 0;
  bool done = !inside;
  for (uint32_t bs = start; bs < end; bs += NT) {
    if (__syncthreads_count(done) == NT) break;
    const uint32_t idx = bs + tid;
    if (idx < end) {
      const float4* rec = reinterpret_cast<const float4*>(splats + values[idx]);
      float4 a = rec[0], b = rec[1];
      const float c = rec[2].x;
      a.z *= kHalfLog2e;
      b.x *= kHalfLog2e;
      b.y = log2f(b.y);
      s_a[tid] = a;
      s_b[tid] = b;
      s_c[tid] = c;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)NT, end - bs);
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        const float4 a = s_a[j];
        const float4 b = s_b[j];
        const float dx = fx - a.x, dy = fy - a.y;
        const float u = fmaf(-a.w, dy, dx);
        // log2 of o*exp(-Q/2), Q = qa u^2 + qc dy^2
        const float e = b.y - fmaf(a.z, u * u, b.x * (dy * dy));
        if (e < set.log2_tau) continue;  // weight below alpha_min: skipped
        const float alpha = fminf(set.amax, exp2f(e));
        const float w = alpha * T;
        C0 = fmaf(w, b.z, C0);
        C1 = fmaf(w, b.w, C1);
        C2 = fmaf(w, s_c[j], C2);
        T = T * (1.f - alpha);
        lastc = bs + j + 1 - start;
        if (T < set.t_eps) {
          done = true;
          break;
        }
      }
    }
  }
  if (inside) {
    const int p = py * W + px;
    reinterpret_cast<float4*>(image)[p] =
        make_float4(fmaf(T, set.bg[0], C0), fmaf(T, set.bg[1], C1), fmaf(T, set.bg[2], C2), 1.f - T);
    T_final[p] = T;
    last[p] = lastc;
  }
}

// Backward: walk each pixel's blended splats back to front from `last`,
// recovering T_i = T_{i+1} / (1 - alpha_i) from T_final.  With
//   S_i = colour composited behind i (normalised by T_{i+1}),
//   B_i = T_final / T_{i+1},
// dC/dalpha_i = T_i (c_i - S_i - B_i bg) and dA/dalpha_i = T_i B_i.
// Per splat the 9 partial derivatives are summed over the wave first and
// added to the Gaussian's 2-D gradient record with one atomic per value.
template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_raster_bwd(const gs_splat* __restrict__ splats,
                                                       const uint32_t* __restrict__ values,
                                                       const uint32_t* __restrict__ ranges,
                                                       SetK set, int W, int H,
                                                       const float* __restrict__ T_final,
                                                       const uint32_t* __restrict__ last,
                                                       const float* __restrict__ dL_dimage,
                                                       float* __restrict__ grad2d) {
  constexpr int NT = TW * TH;
  // staged exactly as in the forward kernel, so that every skip decision
  // (log2 weight < log2 alpha_min) is taken on identical arithmetic
  __shared__ float4 s_a[NT];  // mean_x, mean_y, qa*log2e/2, qb
  __shared__ float4 s_b[NT];  // qc*log2e/2, log2(opacity), r, g
  __shared__ float2 s_c[NT];  // b, opacity
  __shared__ uint32_t s_g[NT];
  __shared__ uint32_t s_maxlast;
  const int tiles = set.tiles_x * set.tiles_y;
  const int tile = xcd_tile(blockIdx.x, tiles);
  if (tile >= tiles) return;
  const int tid = threadIdx.x;
  const int px = (tile % set.tiles_x) * TW + tid % TW;
  const int py = (tile / set.tiles_x) * TH + tid / TW;
  const bool inside = px < W && py < H;
  const float fx = px + 0.5f, fy = py + 0.5f;
  const uint32_t start = ranges[2 * tile];

  float T = 1.f, dC0 = 0.f, dC1 = 0.f, dC2 = 0.f, dA = 0.f;
  uint32_t mylast = 0;
  if (inside) {
    const int p = py * W + px;
    T = T_final[p];
    mylast = last[p];
    const float4 g = reinterpret_cast<const float4*>(dL_dimage)[p];
    dC0 = g.x; dC1 = g.y; dC2 = g.z; dA = g.w;
  }
  if (tid == 0) s_maxlast = 0;
  __syncthreads();
  if (mylast) atomicMax(&s_maxlast, mylast);
  __syncthreads();
  const uint32_t nlast = s_maxlast;
  const float bgdot = dC0 * set.bg[0] + dC1 * set.bg[1] + dC2 * set.bg[2];
  float S0 = 0.f, S1 = 0.f, S2 = 0.f, B = 1.f;
  constexpr float kLn2 = 0.69314718055994531f;

  // batches cover positions [0, nlast) of the tile's range, last batch first
  const int nb = (int)((nlast + NT - 1) / NT);
  for (int bi = nb - 1; bi >= 0; --bi) {
    const uint32_t bs = (uint32_t)bi * NT;
    __syncthreads();
    const uint32_t pos = bs + tid;
    if (pos < nlast) {
      const uint32_t g = values[start + pos];
      const float4* rec = reinterpret_cast<const float4*>(splats + g);
      float4 a = rec[0], b = rec[1];
      const float c = rec[2].x;
      const float o = b.y;
      a.z *= kHalfLog2e;
      b.x *= kHalfLog2e;
      b.y = log2f(b.y);
      s_a[tid] = a;
      s_b[tid] = b;
      s_c[tid] = make_float2(c, o);
      s_g[tid] = g;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)NT, nlast - bs);
    for (int j = cnt - 1; j >= 0; --j) {
      const float4 a = s_a[j];
      const float4 b = s_b[j];
      float gmx = 0.f, gmy = 0.f, gqa = 0.f, gqb = 0.f, gqc = 0.f, gop = 0.f;
      float gr = 0.f, gg = 0.f, gb = 0.f;
      bool contrib = false;
      if (bs + j < mylast) {
        const float dx = fx - a.x, dy = fy - a.y;
        const float u = fmaf(-a.w, dy, dx);
        const float e = b.y - fmaf(a.z, u * u, b.x * (dy * dy));
        if (e >= set.log2_tau) {
          contrib = true;
          const float2 c2 = s_c[j];
          const float gw = exp2f(e);
          const float alpha = fminf(set.amax, gw);
          const float om = 1.f - alpha;
          const float Ti = T / om;
          const float cr = b.z, cg = b.w, cb = c2.x;
          const float w = alpha * Ti;
          gr = dC0 * w; gg = dC1 * w; gb = dC2 * w;
          const float dalpha = Ti * (dC0 * (cr - S0) + dC1 * (cg - S1) + dC2 * (cb - S2) -
                                     B * bgdot + dA * B);
          S0 = fmaf(alpha, cr - S0, S0);
          S1 = fmaf(alpha, cg - S1, S1);
          S2 = fmaf(alpha, cb - S2, S2);
          B *= om;
          T = Ti;
          if (gw < set.amax) {
            // weight g = 2^e with e = log2(o) - Q', Q' = (log2e/2) Q
            gop = dalpha * gw / c2.y;
            const float dQ = -kLn2 * gw * dalpha;  // dL/dQ'
            const float qau = a.z * u;
            gqa = dQ * kHalfLog2e * (u * u);
            gqb = -2.f * dQ * qau * dy;
            gqc = dQ * kHalfLog2e * (dy * dy);
            gmx = -2.f * dQ * qau;
            gmy = 2.f * dQ * (qau * a.w - b.x * dy);
          }
        }
      }
      if (ballot(contrib)) {
        gmx = wave_sum_f32(gmx); gmy = wave_sum_f32(gmy);
        gqa = wave_sum_f32(gqa); gqb = wave_sum_f32(gqb); gqc = wave_sum_f32(gqc);
        gop = wave_sum_f32(gop);
        gr = wave_sum_f32(gr); gg = wave_sum_f32(gg); gb = wave_sum_f32(gb);
        if (lane_id() == 0) {
          float* dst = grad2d + (size_t)s_g[j] * kGrad2dStride;
          atomicAdd(dst + 0, gmx); atomicAdd(dst + 1, gmy);
          atomicAdd(dst + 2, gqa); atomicAdd(dst + 3, gqb); atomicAdd(dst + 4, gqc);
          atomicAdd(dst + 5, gop);
          atomicAdd(dst + 6, gr); atomicAdd(dst + 7, gg); atomicAdd(dst + 8, gb);
        }
      }
    }
  }
}

template <int TW, int TH>
void raster_fwd(const gs_splat* splats, const uint32_t* values, const uint32_t* ranges,
                const SetK& set, int W, int H, float* image, float* T_final, uint32_t* last,
                hipStream_t st) {
  const int tiles = set.tiles_x * set.tiles_y;
  hipLaunchKernelGGL((k_raster<TW, TH>), dim3(xcd_grid(tiles)), dim3(TW * TH), 0, st, splats,
                     values, ranges, set, W, H, image, T_final, last);
}

template <int TW, int TH>
void raster_bwd(const gs_splat* splats, const uint32_t* values, const uint32_t* ranges,
                const SetK& set, int W, int H, const float* T_final, const uint32_t* last,
                const float* dL_dimage, float* grad2d, hipStream_t st) {
  const int tiles = set.tiles_x * set.tiles_y;
  hipLaunchKernelGGL((k_raster_bwd<TW, TH>), dim3(xcd_grid(tiles)), dim3(TW * TH), 0, st,
                     splats, values, ranges, set, W, H, T_final, last, dL_dimage, grad2d);
}

}  // namespace

bool tile_shape_supported(int tw, int th) {
  return (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 16 && th == 16) ||
         (tw == 32 && th == 8) || (tw == 32 && th == 16);
}

hipError_t launch_rasterize(const gs_splat* splats, const uint32_t* values,
                            const uint32_t* ranges, const SetK& set, int W, int H,
                            float* image, float* T_final, uint32_t* last, hipStream_t st) {
  const int tw = set.tile_w, th = set.tile_h;
  if (tw == 8 && th == 8) raster_fwd<8, 8>(splats, values, ranges, set, W, H, image, T_final, last, st);
  else if (tw == 16 && th == 8) raster_fwd<16, 8>(splats, values, ranges, set, W, H, image, T_final, last, st);
  else if (tw == 16 && th == 16) raster_fwd<16, 16>(splats, values, ranges, set, W, H, image, T_final, last, st);
  else if (tw == 32 && th == 8) raster_fwd<32, 8>(splats, values, ranges, set, W, H, image, T_final, last, st);
  else raster_fwd<32, 16>(splats, values, ranges, set, W, H, image, T_final, last, st);
  return hipGetLastError();
}

hipError_t launch_rasterize_backward(const gs_splat* splats, const uint32_t* values,
                                     const uint32_t* ranges, const SetK& set, int W, int H,
                                     const float* T_final, const uint32_t* last,
                                     const float* dL_dimage, float* grad2d, hipStream_t st) {
  const int tw = set.tile_w, th = set.tile_h;
  if (tw == 8 && th == 8) raster_bwd<8, 8>(splats, values, ranges, set, W, H, T_final, last, dL_dimage, grad2d, st);
  else if (tw == 16 && th == 8) raster_bwd<16, 8>(splats, values, ranges, set, W, H, T_final, last, dL_dimage, grad2d, st);
  else if (tw == 16 && th == 16) raster_bwd<16, 16>(splats, values, ranges, set, W, H, T_final, last, dL_dimage, grad2d, st);
  else if (tw == 32 && th == 8) raster_bwd<32, 8>(splats, values, ranges, set, W, H, T_final, last, dL_dimage, grad2d, st);
  else raster_bwd<32, 16>(splats, values, ranges, set, W, H, T_final, last, dL_dimage, grad2d, st);
  return hipGetLastError();
}

}  // namespace gs
