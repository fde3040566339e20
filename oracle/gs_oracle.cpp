// Plain FP64 CPU oracle for the 3D Gaussian Splatting render path.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; it exists so that tests (and the CPU-baseline leg of the
// benchmark) can check the GPU library against a slow, obviously correct
// implementation of what the renderer computes.  It shares no code, header,
// table or helper with the GPU library.
//
// What it computes (paper: "Visionary", Section 3.2 Eqs. 1-3 and
// Algorithm 1 / Section 3.4), every step in float64:
//   * the per-Gaussian projection of Eq. 1: activations, Sigma from scale
//     and rotation (Algorithm 1, CovFromScaleRot), optional per-model
//     similarity transform, camera transform, near/opacity/frustum culls,
//     EWA footprint S = J W Sigma W^T J^T (+ eps I), its inverse, the 2-D
//     mean, and the view-dependent SH colour (Section 3.2 / 3.4); the same
//     projection from a Gaussian given by mean, activated opacity and upper
//     covariance triangle (the pre-packed form of Section 3.4);
//   * the per-pixel colour of Eq. 3 with the 2-D weight of Eq. 2, taken by
//     brute force over every surviving Gaussian in ascending (depth, index)
//     order -- no tiles, no sort keys;
//   * the (tile, depth) key list and a library stable sort, for the sort
//     contract;
//   * the real SH basis of degree <= 3, exposed for its own pins.
//
// Readings of what the paper leaves open (all settable through `set`):
//   camera: OpenCV pinhole, +z forward, pixel (i,j) samples (i+1/2, j+1/2);
//   J is the Jacobian of the perspective division at the camera-space mean
//     with x/z, y/z clamped to `clip` times the half-FoV tangent;
//   eps2d is added to the diagonal of S (a low-pass term);
//   tau: a Gaussian with opacity < tau is culled, a pixel weight < tau is
//     skipped; alpha is clamped to alpha_max; compositing blends and then
//     stops once the transmittance falls below t_eps;
//   near plane: t_z <= znear is culled; no far plane;
//   colour: rgb = max(0, sum_lm sh_lm Y_lm(d) + 1/2), d the unit vector
//     from the camera centre to the mean (rotated into the asset frame when
//     a model transform is given);
//   equal depths are ordered by Gaussian index.
//
// Build: g++ -O2 -std=c++17 -fopenmp -shared -fPIC (no fast-math).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <numeric>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Layout of the per-Gaussian record written by orc_preprocess.
enum RecD {
  D_MX = 0, D_MY = 1,                 // 2-D mean (pixels)
  D_SA = 2, D_SB = 3, D_SC = 4,       // S = [[a,b],[b,c]] incl. eps2d
  D_CA = 5, D_CB = 6, D_CC = 7,       // S^-1 = [[A,B],[B,C]]
  D_DEPTH = 8,                        // camera-space z
  D_R = 9, D_G = 10, D_B = 11,        // colour after the clamp at 0
  D_RR = 12, D_RG = 13, D_RB = 14,    // colour before the clamp
  D_OPAC = 15,                        // activated opacity
  D_C3 = 16,                          // world Sigma: xx xy xz yy yz zz (6)
  D_QMAX = 22,                        // 2 ln(o / tau)
  D_TZ = 23,                          // camera-space z again (kept for margins)
  REC_D = 24
};
enum RecI {
  I_CULL = 0,                          // 0 visible; see CullCode
  I_PX0 = 1, I_PX1 = 2, I_PY0 = 3, I_PY1 = 4,  // inclusive pixel bbox
  I_TX0 = 5, I_TY0 = 6, I_TX1 = 7, I_TY1 = 8,  // inclusive tile rect
  I_TILES = 9,                         // tiles in the rect
  I_AMBIG = 10,                        // culled within a relative 1e-5 of a threshold
  REC_I = 11
};
enum CullCode { C_VISIBLE = 0, C_NEAR = 1, C_INVALID = 2, C_DET = 3,
                C_OPACITY = 4, C_OFFIMAGE = 5 };

struct Cam {
  double V[16];
  double fx, fy, cx, cy;
  int W, H;
  double znear;
};
struct Set {
  int tw, th;
  double eps2d, tau, amax, teps, clip;
  double bg[3];
};

Cam load_cam(const double* c) {
  Cam k;
  std::memcpy(k.V, c, 16 * sizeof(double));
  k.fx = c[16]; k.fy = c[17]; k.cx = c[18]; k.cy = c[19];
  k.W = (int)c[20]; k.H = (int)c[21]; k.znear = c[22];
  return k;
}
Set load_set(const double* s) {
  Set k;
  k.tw = (int)s[0]; k.th = (int)s[1];
  k.eps2d = s[2]; k.tau = s[3]; k.amax = s[4]; k.teps = s[5]; k.clip = s[6];
  k.bg[0] = s[7]; k.bg[1] = s[8]; k.bg[2] = s[9];
  return k;
}

// Real spherical harmonics of degree l <= 3, m = -l..l, evaluated on a unit
// vector.  The basis is sqrt(2) Re Y_l^m (m > 0), Y_l^0, sqrt(2) Im Y_l^|m|
// (m < 0) of the complex harmonics with the Condon-Shortley phase, written
// out as polynomials in (x, y, z); index k = l*l + l + m.
void sh_basis(int degree, double x, double y, double z, double* Y) {
  const double c0 = 0.5 * std::sqrt(1.0 / kPi);
  Y[0] = c0;
  if (degree < 1) return;
  const double c1 = std::sqrt(3.0 / (4.0 * kPi));
  Y[1] = -c1 * y;
  Y[2] = c1 * z;
  Y[3] = -c1 * x;
  if (degree < 2) return;
  const double c2a = 0.5 * std::sqrt(15.0 / kPi);
  const double c2b = 0.25 * std::sqrt(5.0 / kPi);
  const double c2c = 0.25 * std::sqrt(15.0 / kPi);
  Y[4] = c2a * x * y;
  Y[5] = -c2a * y * z;
  Y[6] = c2b * (2.0 * z * z - x * x - y * y);
  Y[7] = -c2a * x * z;
  Y[8] = c2c * (x * x - y * y);
  if (degree < 3) return;
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * kPi));
  const double c3b = 0.5 * std::sqrt(105.0 / kPi);
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * kPi));
  const double c3d = 0.25 * std::sqrt(7.0 / kPi);
  const double c3e = 0.25 * std::sqrt(105.0 / kPi);
  Y[9] = -c3a * y * (3.0 * x * x - y * y);
  Y[10] = c3b * x * y * z;
  Y[11] = -c3c * y * (4.0 * z * z - x * x - y * y);
  Y[12] = c3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
  Y[13] = -c3c * x * (4.0 * z * z - x * x - y * y);
  Y[14] = c3e * z * (x * x - y * y);
  Y[15] = -c3a * x * (x * x - 3.0 * y * y);
}

// Rotation matrix of a unit quaternion (w, x, y, z), row-major.
void quat_to_rot(double w, double x, double y, double z, double R[9]) {
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

void matmul3(const double* A, const double* B, double* C) {  // C = A B
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}
void matmul3_bt(const double* A, const double* B, double* C) {  // C = A B^T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * j + k];
      C[3 * i + j] = s;
    }
}

bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// One Gaussian from its raw parameters: activations and the covariance
// Sigma = R diag(s^2) R^T (Algorithm 1, CovFromScaleRot; Section 3.2), then
// the common projection below.  Real is float (the library's input type)
// or double (finite differences).
template <typename Real>
void preprocess_one(int64_t i, const Real* means, const Real* log_scales,
                    const Real* quats, const Real* logits, const Real* sh,
                    int degree, const double* model, const Cam& cam,
                    const Set& set, double* d, int32_t* iv);

// Eq. 1 and the colour for one Gaussian with mean mu, activated opacity o,
// world covariance Sig (asset frame) and SH row sh_row, with every cull of
// Algorithm 1.
template <typename ShT>
void project_gaussian(const double* mu, double o, const double* Sig, const ShT* sh_row,
                      int degree, const double* model, const Cam& cam, const Set& set,
                      double* d, int32_t* iv) {
  const int K = (degree + 1) * (degree + 1);
  // Per-model similarity transform A = s_k R_k, translation t_k
  // (Algorithm 1, ModelParams; Section 3.4 step (i)).
  double A[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, tk[3] = {0, 0, 0}, Rk[9];
  double sk = 1.0;
  if (model) {
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) A[3 * r + c] = model[4 * r + c];
      tk[r] = model[4 * r + 3];
    }
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    sk = std::cbrt(det);
  }
  for (int k = 0; k < 9; ++k) Rk[k] = A[k] / sk;
  double muw[3], SA[9], Sigw[9];
  for (int r = 0; r < 3; ++r)
    muw[r] = A[3 * r] * mu[0] + A[3 * r + 1] * mu[1] + A[3 * r + 2] * mu[2] + tk[r];
  matmul3(A, Sig, SA);
  matmul3_bt(SA, A, Sigw);
  d[D_C3 + 0] = Sigw[0]; d[D_C3 + 1] = Sigw[1]; d[D_C3 + 2] = Sigw[2];
  d[D_C3 + 3] = Sigw[4]; d[D_C3 + 4] = Sigw[5]; d[D_C3 + 5] = Sigw[8];

  // Camera transform t = V mu_w  (Algorithm 1, x_c = V x_w)
  const double* V = cam.V;
  double t[3];
  for (int r = 0; r < 3; ++r)
    t[r] = V[4 * r] * muw[0] + V[4 * r + 1] * muw[1] + V[4 * r + 2] * muw[2] + V[4 * r + 3];
  d[D_DEPTH] = t[2];
  d[D_TZ] = t[2];
  int cull = C_VISIBLE;
  bool ambiguous = false;
  if (!(t[2] > cam.znear)) {
    cull = C_NEAR;
    if (std::fabs(t[2] - cam.znear) <= 1e-5 * cam.znear) ambiguous = true;
  }

  // Colour: view direction from the camera centre to the mean
  // (Section 3.2: colour encoded by SH; Algorithm 1: evaluate color).
  double Vr[9] = {V[0], V[1], V[2], V[4], V[5], V[6], V[8], V[9], V[10]};
  double campos[3];
  for (int c = 0; c < 3; ++c)
    campos[c] = -(Vr[c] * V[3] + Vr[3 + c] * V[7] + Vr[6 + c] * V[11]);
  double dir[3] = {muw[0] - campos[0], muw[1] - campos[1], muw[2] - campos[2]};
  double dn = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  for (int c = 0; c < 3; ++c) dir[c] /= dn;
  double dl[3];  // into the asset frame: R_k^T d
  for (int c = 0; c < 3; ++c) dl[c] = Rk[c] * dir[0] + Rk[3 + c] * dir[1] + Rk[6 + c] * dir[2];
  double Y[16];
  sh_basis(degree, dl[0], dl[1], dl[2], Y);
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc += (double)sh_row[k * 3 + ch] * Y[k];
    acc += 0.5;
    d[D_RR + ch] = acc;
    d[D_R + ch] = acc > 0.0 ? acc : 0.0;
  }

  // EWA footprint, Eq. 1: S = J W Sigma_w W^T J^T + eps I.
  if (t[2] > 0.0) {
    const double tz = t[2];
    const double limx = set.clip * (0.5 * cam.W) / cam.fx;
    const double limy = set.clip * (0.5 * cam.H) / cam.fy;
    double xt = std::min(limx, std::max(-limx, t[0] / tz));
    double yt = std::min(limy, std::max(-limy, t[1] / tz));
    double J[6] = {cam.fx / tz, 0.0, -cam.fx * xt / tz, 0.0, cam.fy / tz, -cam.fy * yt / tz};
    double WS[9], Sc[9];
    matmul3(Vr, Sigw, WS);
    matmul3_bt(WS, Vr, Sc);  // W Sigma_w W^T
    double JS[6];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c)
        JS[3 * r + c] = J[3 * r] * Sc[c] + J[3 * r + 1] * Sc[3 + c] + J[3 * r + 2] * Sc[6 + c];
    double S[4];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c)
        S[2 * r + c] = JS[3 * r] * J[3 * c] + JS[3 * r + 1] * J[3 * c + 1] + JS[3 * r + 2] * J[3 * c + 2];
    const double a = S[0] + set.eps2d, b = 0.5 * (S[1] + S[2]), c = S[3] + set.eps2d;
    d[D_SA] = a; d[D_SB] = b; d[D_SC] = c;
    const double det = a * c - b * b;
    d[D_MX] = cam.fx * t[0] / tz + cam.cx;
    d[D_MY] = cam.fy * t[1] / tz + cam.cy;
    if (!(det > 0.0) || !std::isfinite(det)) {
      if (cull == C_VISIBLE) cull = C_DET;
    } else {
      d[D_CA] = c / det; d[D_CB] = -b / det; d[D_CC] = a / det;
    }
    if (!finite_all(d, D_C3) && cull == C_VISIBLE) cull = C_INVALID;
  } else if (cull == C_VISIBLE) {
    cull = C_NEAR;
  }

  // Opacity cull (Algorithm 1: alpha < alpha_min).
  if (o < set.tau) {
    if (cull == C_VISIBLE) cull = C_OPACITY;
    if (o >= set.tau * (1.0 - 1e-5)) ambiguous = true;
  }

  // Exact bbox of the ellipse {x : (x-m)^T S^-1 (x-m) <= 2 ln(o/tau)}: outside
  // it every pixel weight is below tau.  Pixel centres sit at +1/2.
  const bool have_shape = (t[2] > 0.0) && d[D_CA] != 0.0;
  if (have_shape) {
    double qmax = 2.0 * std::log(o / set.tau);
    if (ambiguous && qmax <= 0.0) qmax = 1e-6;  // keep a footprint for margin checks
    d[D_QMAX] = qmax;
    if (qmax > 0.0) {
      const double rx = std::sqrt(qmax * d[D_SA]), ry = std::sqrt(qmax * d[D_SC]);
      const double mx = d[D_MX], my = d[D_MY];
      double fx0 = std::ceil(mx - rx - 0.5), fx1 = std::floor(mx + rx - 0.5);
      double fy0 = std::ceil(my - ry - 0.5), fy1 = std::floor(my + ry - 0.5);
      fx0 = std::max(fx0, 0.0); fy0 = std::max(fy0, 0.0);
      fx1 = std::min(fx1, (double)(cam.W - 1)); fy1 = std::min(fy1, (double)(cam.H - 1));
      if (fx0 <= fx1 && fy0 <= fy1) {
        iv[I_PX0] = (int)fx0; iv[I_PX1] = (int)fx1; iv[I_PY0] = (int)fy0; iv[I_PY1] = (int)fy1;
        iv[I_TX0] = iv[I_PX0] / set.tw; iv[I_TX1] = iv[I_PX1] / set.tw;
        iv[I_TY0] = iv[I_PY0] / set.th; iv[I_TY1] = iv[I_PY1] / set.th;
      } else if (cull == C_VISIBLE) {
        cull = C_OFFIMAGE;
      }
    } else if (cull == C_VISIBLE) {
      cull = C_OPACITY;
    }
  }
  iv[I_CULL] = cull;
  iv[I_AMBIG] = (cull != C_VISIBLE && ambiguous && iv[I_PX1] >= iv[I_PX0]) ? 1 : 0;
  if (cull == C_VISIBLE)
    iv[I_TILES] = (iv[I_TX1] - iv[I_TX0] + 1) * (iv[I_TY1] - iv[I_TY0] + 1);
}

void clear_record(double* d, int32_t* iv) {
  for (int k = 0; k < REC_D; ++k) d[k] = 0.0;
  for (int k = 0; k < REC_I; ++k) iv[k] = 0;
  iv[I_PX0] = iv[I_PY0] = iv[I_TX0] = iv[I_TY0] = 0;
  iv[I_PX1] = iv[I_PY1] = iv[I_TX1] = iv[I_TY1] = -1;
}

template <typename Real>
void preprocess_one(int64_t i, const Real* means, const Real* log_scales,
                    const Real* quats, const Real* logits, const Real* sh,
                    int degree, const double* model, const Cam& cam,
                    const Set& set, double* d, int32_t* iv) {
  clear_record(d, iv);
  const int K = (degree + 1) * (degree + 1);
  double mu[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
  double s[3] = {std::exp((double)log_scales[3 * i]), std::exp((double)log_scales[3 * i + 1]),
                 std::exp((double)log_scales[3 * i + 2])};
  double q[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
  double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double o = 1.0 / (1.0 + std::exp(-(double)logits[i]));
  d[D_OPAC] = o;
  if (!(qn > 0.0) || !std::isfinite(qn) || !finite_all(mu, 3) || !finite_all(s, 3) ||
      !std::isfinite(o)) {
    iv[I_CULL] = C_INVALID;
    return;
  }
  for (int k = 0; k < 4; ++k) q[k] /= qn;
  double R[9], M[9], Sig[9];
  quat_to_rot(q[0], q[1], q[2], q[3], R);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[3 * r + c] = R[3 * r + c] * s[c];
  matmul3_bt(M, M, Sig);
  project_gaussian(mu, o, Sig, sh + (size_t)i * K * 3, degree, model, cam, set, d, iv);
}

// One Gaussian given directly by its mean, activated opacity and the upper
// triangle (xx, xy, xz, yy, yz, zz) of its covariance: the input of the
// pre-packed layout (Algorithm 1, Pre-pack; Section 3.4).
void preprocess_cov_one(int64_t i, const double* means, const double* opac, const double* cov6,
                        const double* sh, int degree, const double* model, const Cam& cam,
                        const Set& set, double* d, int32_t* iv) {
  clear_record(d, iv);
  const int K = (degree + 1) * (degree + 1);
  const double mu[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
  const double* u = cov6 + 6 * i;
  const double Sig[9] = {u[0], u[1], u[2], u[1], u[3], u[4], u[2], u[4], u[5]};
  const double o = opac[i];
  d[D_OPAC] = o;
  if (!finite_all(mu, 3) || !finite_all(Sig, 9) || !std::isfinite(o)) {
    iv[I_CULL] = C_INVALID;
    return;
  }
  project_gaussian(mu, o, Sig, sh + (size_t)i * K * 3, degree, model, cam, set, d, iv);
}

inline double pixel_weight(const double* d, double px, double py) {
  // Eq. 2 without the alpha clamp: o * exp(-1/2 dx^T S^-1 dx)
  const double dx = px - d[D_MX], dy = py - d[D_MY];
  const double Q = d[D_CA] * dx * dx + 2.0 * d[D_CB] * dx * dy + d[D_CC] * dy * dy;
  return d[D_OPAC] * std::exp(-0.5 * Q);
}

}  // namespace

extern "C" {

int orc_rec_layout(int32_t* out) {
  out[0] = REC_D;
  out[1] = REC_I;
  return 0;
}

// Real SH basis values for n unit directions (n x 3) -> out (n x 16); entries
// above the degree are left 0.
int orc_sh_basis(int degree, int64_t n, const double* dirs, double* out) {
  if (degree < 0 || degree > 3) return 1;
  for (int64_t i = 0; i < n; ++i) {
    double Y[16] = {0};
    sh_basis(degree, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], Y);
    for (int k = 0; k < 16; ++k) out[16 * i + k] = Y[k];
  }
  return 0;
}

// Per-Gaussian records (REC_D doubles + REC_I ints each) for one asset.
// cam: viewmat[16] (row-major world->camera), fx, fy, cx, cy, W, H, znear.
// set: tile_w, tile_h, eps2d, tau, alpha_max, t_eps, clip, bg[3].
// model: NULL or 3x4 row-major similarity transform [s R | t].
int orc_preprocess(int64_t n, const float* means, const float* log_scales,
                   const float* quats, const float* logits, const float* sh,
                   int degree, const double* model, const double* cam_in,
                   const double* set_in, double* rec_d, int32_t* rec_i) {
  if (n < 0 || degree < 0 || degree > 3) return 1;
  const Cam cam = load_cam(cam_in);
  const Set set = load_set(set_in);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    preprocess_one<float>(i, means, log_scales, quats, logits, sh, degree, model, cam, set,
                          rec_d + (size_t)i * REC_D, rec_i + (size_t)i * REC_I);
  return 0;
}

// Same with float64 inputs (used for central finite differences).
int orc_preprocess_f64(int64_t n, const double* means, const double* log_scales,
                       const double* quats, const double* logits, const double* sh,
                       int degree, const double* model, const double* cam_in,
                       const double* set_in, double* rec_d, int32_t* rec_i) {
  if (n < 0 || degree < 0 || degree > 3) return 1;
  const Cam cam = load_cam(cam_in);
  const Set set = load_set(set_in);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    preprocess_one<double>(i, means, log_scales, quats, logits, sh, degree, model, cam, set,
                           rec_d + (size_t)i * REC_D, rec_i + (size_t)i * REC_I);
  return 0;
}

// From the pre-packed representation: means (n*3), activated opacities (n),
// upper covariance triangles (n*6: xx, xy, xz, yy, yz, zz) and SH (n*K*3),
// all float64 (the caller decodes whatever rounded values it packs).
int orc_preprocess_cov(int64_t n, const double* means, const double* opac, const double* cov6,
                       const double* sh, int degree, const double* model, const double* cam_in,
                       const double* set_in, double* rec_d, int32_t* rec_i) {
  if (n < 0 || degree < 0 || degree > 3) return 1;
  const Cam cam = load_cam(cam_in);
  const Set set = load_set(set_in);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    preprocess_cov_one(i, means, opac, cov6, sh, degree, model, cam, set,
                       rec_d + (size_t)i * REC_D, rec_i + (size_t)i * REC_I);
  return 0;
}

// Eq. 3 by brute force at npix pixels (x, y pairs).  Every visible Gaussian
// is visited in ascending (depth, index) order.
// Outputs per pixel: rgba (4), final transmittance T, number of blended
// Gaussians, the smallest relative margin to any discrete decision taken
// (pixel skip alpha<tau, clamp at alpha_max, stop at T<t_eps), and flags:
//   1 = two blended Gaussians closer in depth than a relative 1e-6;
//   2 = a Gaussian culled within a relative 1e-5 of a threshold covers it;
//   4 = a Gaussian with weight >= tau lies within a relative 1e-5 of the
//       mesh depth.
// Mesh depth composition (Algorithm 1, DrawSplatsWithMeshDepth; Section
// 3.4): with mesh_depth (one value per requested pixel, camera-space z of
// the mesh surface; +inf where there is none), a Gaussian whose depth is
// greater than the pixel's mesh depth is hidden by the mesh, and so is
// every Gaussian after it in depth order; mesh_rgb (three values per
// pixel) replaces the background colour behind the Gaussians.  Either may
// be NULL.
int orc_render_pixels(int64_t n, const double* rec_d, const int32_t* rec_i,
                      const double* cam_in, const double* set_in, int64_t npix,
                      const int32_t* pix, const double* mesh_depth, const double* mesh_rgb,
                      double* rgba, double* T_out, int32_t* n_blend, double* margin,
                      int32_t* flags) {
  const Cam cam = load_cam(cam_in);
  const Set set = load_set(set_in);
  std::vector<int64_t> order;
  std::vector<int64_t> ambig;
  order.reserve((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    if (rec_i[(size_t)i * REC_I + I_CULL] == C_VISIBLE) order.push_back(i);
    else if (rec_i[(size_t)i * REC_I + I_AMBIG]) ambig.push_back(i);
  }
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    const double da = rec_d[(size_t)a * REC_D + D_DEPTH], db = rec_d[(size_t)b * REC_D + D_DEPTH];
    if (da != db) return da < db;
    return a < b;
  });
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < npix; ++p) {
    const int x = pix[2 * p], y = pix[2 * p + 1];
    const double px = x + 0.5, py = y + 0.5;
    double C[3] = {0, 0, 0}, T = 1.0, mrg = std::numeric_limits<double>::infinity();
    int32_t nb = 0, fl = 0;
    double last_depth = -1.0;
    const double D = mesh_depth ? mesh_depth[p] : std::numeric_limits<double>::infinity();
    for (int64_t idx : order) {
      const double* d = rec_d + (size_t)idx * REC_D;
      const double g = pixel_weight(d, px, py);
      if (std::isfinite(D) && g >= set.tau && std::fabs(d[D_DEPTH] - D) <= 1e-5 * std::fabs(D))
        fl |= 4;
      if (d[D_DEPTH] > D) break;  // hidden by the mesh, as is everything behind
      mrg = std::min(mrg, std::fabs(g - set.tau) / set.tau);
      if (g < set.tau) continue;
      mrg = std::min(mrg, std::fabs(g - set.amax) / set.amax);
      const double a = std::min(set.amax, g);
      for (int c = 0; c < 3; ++c) C[c] += T * a * d[D_R + c];
      T *= (1.0 - a);
      ++nb;
      if (last_depth >= 0.0 && std::fabs(d[D_DEPTH] - last_depth) <= 1e-6 * d[D_DEPTH]) fl |= 1;
      last_depth = d[D_DEPTH];
      mrg = std::min(mrg, std::fabs(T - set.teps) / set.teps);
      if (T < set.teps) break;
    }
    for (int64_t idx : ambig) {
      const int32_t* iv = rec_i + (size_t)idx * REC_I;
      if (x >= iv[I_PX0] && x <= iv[I_PX1] && y >= iv[I_PY0] && y <= iv[I_PY1]) {
        fl |= 2;
        mrg = 0.0;
      }
    }
    for (int c = 0; c < 3; ++c)
      rgba[4 * p + c] = C[c] + T * (mesh_rgb ? mesh_rgb[3 * p + c] : set.bg[c]);
    rgba[4 * p + 3] = 1.0 - T;
    T_out[p] = T;
    n_blend[p] = nb;
    margin[p] = mrg;
    flags[p] = fl;
  }
  return 0;
}

// Number of (Gaussian, tile) instances of the visible Gaussians.
int64_t orc_count_instances(int64_t n, const int32_t* rec_i) {
  int64_t total = 0;
  for (int64_t i = 0; i < n; ++i)
    if (rec_i[(size_t)i * REC_I + I_CULL] == C_VISIBLE) total += rec_i[(size_t)i * REC_I + I_TILES];
  return total;
}

// Key list: for each visible Gaussian in index order, each tile of its rect
// in row-major order: key = tile_id << 32 | bits(float32(depth)),
// value = Gaussian index.
int orc_keys(int64_t n, const double* rec_d, const int32_t* rec_i, int tiles_x,
             uint64_t* keys, uint32_t* values) {
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* iv = rec_i + (size_t)i * REC_I;
    if (iv[I_CULL] != C_VISIBLE) continue;
    const float z = (float)rec_d[(size_t)i * REC_D + D_DEPTH];
    uint32_t zb;
    std::memcpy(&zb, &z, 4);
    for (int ty = iv[I_TY0]; ty <= iv[I_TY1]; ++ty)
      for (int tx = iv[I_TX0]; tx <= iv[I_TX1]; ++tx) {
        keys[k] = ((uint64_t)(uint32_t)(ty * tiles_x + tx) << 32) | (uint64_t)zb;
        values[k] = (uint32_t)i;
        ++k;
      }
  }
  return 0;
}

// Largest unclamped weight o*exp(-Q/2) of Gaussian g over the pixel centres
// of tile `tile` (row-major id) inside the image, for each of npairs pairs.
int orc_pair_max_weight(int64_t npairs, const uint32_t* g, const uint32_t* tile,
                        const double* rec_d, const double* cam_in, const double* set_in,
                        double* out) {
  const Cam cam = load_cam(cam_in);
  const Set set = load_set(set_in);
  const int tiles_x = (cam.W + set.tw - 1) / set.tw;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < npairs; ++p) {
    const double* d = rec_d + (size_t)g[p] * REC_D;
    const int tx = (int)(tile[p] % (uint32_t)tiles_x), ty = (int)(tile[p] / (uint32_t)tiles_x);
    double best = 0.0;
    for (int y = ty * set.th; y < std::min(cam.H, (ty + 1) * set.th); ++y)
      for (int x = tx * set.tw; x < std::min(cam.W, (tx + 1) * set.tw); ++x)
        best = std::max(best, pixel_weight(d, x + 0.5, y + 0.5));
    out[p] = best;
  }
  return 0;
}

// Stable sort of (key, value) pairs by key (library std::stable_sort).
int orc_stable_sort_pairs(int64_t n, uint64_t* keys, uint32_t* values) {
  std::vector<int64_t> perm((size_t)n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int64_t a, int64_t b) { return keys[a] < keys[b]; });
  std::vector<uint64_t> k2((size_t)n);
  std::vector<uint32_t> v2((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    k2[i] = keys[perm[i]];
    v2[i] = values[perm[i]];
  }
  std::copy(k2.begin(), k2.end(), keys);
  std::copy(v2.begin(), v2.end(), values);
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
