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
//     order -- no tiles, no sort keys -- and the same walk over per-tile
//     candidate lists (orc_render_tiled), which is exactly equal and fast
//     enough for whole 1080p frames; each pixel also reports the decisions
//     its float64 walk took close to a threshold (the tolerance protocol) and the
//     jump that taking each of them the other way would cause;
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
  D_UNUSED = 23,                      // (zero)
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

// Relative margins below which a decision is near: a weight against tau
// (skip, an ambiguous Gaussian's include) within 3e-5 -- twice the largest
// float32 error of a pixel weight measured near tau (1.6e-5 over the ~10^5
// near-threshold pairs of the 1M frame) -- and the transmittance against
// t_eps within 1e-4, since T's float32 error compounds over the blends
// through factors 1 - alpha.
constexpr double kNearRel = 3e-5;
constexpr double kNearStop = 1e-4;

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

// Pixels whose centres (i + 1/2, j + 1/2) lie in the bounding box of the
// ellipse {x : (x - m)^T S^-1 (x - m) <= q} -- half-extents sqrt(q S00) and
// sqrt(q S11) -- clipped to the image: box = (x0, x1, y0, y1), inclusive.
// False when it holds no pixel centre.
bool pixel_bbox(const double* d, double q, const Cam& cam, int* box) {
  const double rx = std::sqrt(q * d[D_SA]), ry = std::sqrt(q * d[D_SC]);
  const double mx = d[D_MX], my = d[D_MY];
  double x0 = std::ceil(mx - rx - 0.5), x1 = std::floor(mx + rx - 0.5);
  double y0 = std::ceil(my - ry - 0.5), y1 = std::floor(my + ry - 0.5);
  x0 = std::max(x0, 0.0); y0 = std::max(y0, 0.0);
  x1 = std::min(x1, (double)(cam.W - 1)); y1 = std::min(y1, (double)(cam.H - 1));
  if (!(x0 <= x1 && y0 <= y1)) return false;
  box[0] = (int)x0; box[1] = (int)x1; box[2] = (int)y0; box[3] = (int)y1;
  return true;
}

void set_bbox(const int* box, const Set& set, int32_t* iv) {
  iv[I_PX0] = box[0]; iv[I_PX1] = box[1]; iv[I_PY0] = box[2]; iv[I_PY1] = box[3];
  iv[I_TX0] = box[0] / set.tw; iv[I_TX1] = box[1] / set.tw;
  iv[I_TY0] = box[2] / set.th; iv[I_TY1] = box[3] / set.th;
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
  int box[4];
  if (have_shape) {
    const double qmax = 2.0 * std::log(o / set.tau);
    d[D_QMAX] = qmax;
    if (cull == C_VISIBLE) {
      if (!(qmax > 0.0)) {
        cull = C_OPACITY;
      } else if (pixel_bbox(d, qmax, cam, box)) {
        set_bbox(box, set, iv);
      } else {
        cull = C_OFFIMAGE;
        // the support misses every pixel centre; it is a near decision when
        // the region where the weight reaches tau (1 - kNearRel) does not
        ambiguous = true;
      }
    }
    // A culled Gaussian counts as ambiguous when some pixel centre sees a
    // weight within kNearRel of tau, were it kept; its bbox is then that
    // region's.
    if (cull != C_VISIBLE && ambiguous) {
      const double qn = 2.0 * std::log(o / (set.tau * (1.0 - kNearRel)));
      if (qn > 0.0 && pixel_bbox(d, qn, cam, box)) set_bbox(box, set, iv);
      else ambiguous = false;
    }
  }
  iv[I_CULL] = cull;
  iv[I_AMBIG] = (cull != C_VISIBLE && ambiguous) ? 1 : 0;
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

// ---------------------------------------------------------------------------
// Per-pixel compositing, Eqs. 2-3.  A pixel walks its candidates -- the
// visible Gaussians and the ambiguous culled ones -- in ascending (depth,
// index) order: alpha = min(alpha_max, o exp(-Q/2)); a weight below tau is
// skipped; C += T alpha rgb; T *= 1 - alpha; the walk stops once T < t_eps.
//
// Tolerance protocol.  The GPU computes in float32, so it may take a
// discrete decision the other way where the float64 value lies close to the
// threshold (a "near" decision; bands kNearRel, kNearStop): the skip
// (weight vs tau), the stop (T vs t_eps), the order of two blended Gaussians whose
// depths agree within float32 rounding (or of the Gaussian the walk stops
// on and the next one that would blend), keeping a Gaussian culled within 1e-5
// of a threshold, and the mesh depth test.  The walk records each near
// decision; the pixel's jump is the sum, over its near decisions, of the
// largest change of any output channel when that one decision is taken the
// other way (the pixel re-walked with it forced).

// Two depths are a near tie when they differ by at most 2^-22 times the sum
// of their magnitudes (two to four float32 spacings): the sort key is the
// float32 rounding of the depth, and depths that round to the same or
// neighbouring float32 values may be ordered either way.
constexpr double kTieRel = 1.0 / 4194304.0;
constexpr int kMaxNear = 64;       // more near decisions: the jump is not bounded

struct Cand {
  int64_t idx;  // Gaussian
  bool ambig;   // culled within a relative 1e-5 of a threshold
};

enum NearKind { N_TAKE = 1, N_STOP = 2, N_SWAP = 3, N_INCLUDE = 4, N_HIDE = 5 };

struct Near {
  int kind;
  int64_t k, k2;  // walk positions (k2: the other Gaussian of a swap)
};

struct WalkOut {
  double C[3], T, mrg;
  int32_t nb, fl;
  std::vector<Near> near;
};

// One walk over the candidate list L (in walk order).  `force` (or NULL)
// takes one decision the other way; only the unforced walk records margins,
// flags and near decisions.  D is the pixel's mesh depth (+inf: none).
void walk_pixel(const std::vector<Cand>& L, const double* rec_d, const Set& set,
                double px, double py, double D, const Near* force, WalkOut& o) {
  const bool rec = force == nullptr;
  o.C[0] = o.C[1] = o.C[2] = 0.0;
  o.T = 1.0;
  o.mrg = 1.0;
  o.nb = 0;
  o.fl = 0;
  o.near.clear();
  int64_t prev = -1;
  double prev_depth = 0.0;
  const int64_t n = (int64_t)L.size();
  for (int64_t k = 0; k < n; ++k) {
    int64_t at = k;  // the swap force exchanges two positions of the walk
    if (force && force->kind == N_SWAP) {
      if (k == force->k) at = force->k2;
      else if (k == force->k2) at = force->k;
    }
    const bool forced = force && force->kind != N_SWAP && force->k == k;
    const Cand& c = L[(size_t)at];
    const double* d = rec_d + (size_t)c.idx * REC_D;
    const double g = pixel_weight(d, px, py);
    const double depth = d[D_DEPTH];
    if (std::isfinite(D)) {
      // mesh depth test: hidden when deeper than the mesh, and so is every
      // Gaussian after it in depth order
      bool hidden = depth > D;
      if (rec && g >= set.tau && std::fabs(depth - D) <= 1e-5 * std::fabs(D)) {
        o.fl |= 4;
        o.near.push_back({N_HIDE, k, -1});
      }
      if (forced && force->kind == N_HIDE) hidden = !hidden;
      if (hidden) break;
    }
    bool take;
    if (c.ambig) {
      // culled, but kept by a float32 computation it would be blended where
      // its weight reaches tau within the near band
      const bool could = g >= set.tau * (1.0 - kNearRel);
      if (rec && could) {
        o.fl |= 2;
        o.mrg = 0.0;
        o.near.push_back({N_INCLUDE, k, -1});
      }
      take = forced && force->kind == N_INCLUDE && could;
    } else {
      const double m = std::fabs(g - set.tau) / set.tau;
      if (rec) {
        o.mrg = std::min(o.mrg, m);
        if (m < kNearRel) o.near.push_back({N_TAKE, k, -1});
      }
      take = g >= set.tau;
      if (forced && force->kind == N_TAKE) take = !take;
    }
    if (!take) continue;
    if (rec) o.mrg = std::min(o.mrg, std::fabs(g - set.amax) / set.amax);
    const double a = std::min(set.amax, g);
    for (int ch = 0; ch < 3; ++ch) o.C[ch] += o.T * a * d[D_R + ch];
    o.T *= (1.0 - a);
    ++o.nb;
    if (rec && prev >= 0 &&
        std::fabs(depth - prev_depth) <= kTieRel * (std::fabs(depth) + std::fabs(prev_depth))) {
      o.fl |= 1;
      o.near.push_back({N_SWAP, prev, k});
    }
    prev = k;
    prev_depth = depth;
    const double m3 = std::fabs(o.T - set.teps) / set.teps;
    if (rec) {
      o.mrg = std::min(o.mrg, m3);
      if (m3 < kNearStop) o.near.push_back({N_STOP, k, -1});
    }
    bool stop = o.T < set.teps;
    if (forced && force->kind == N_STOP) stop = !stop;
    if (stop) {
      // The Gaussian the walk stops on may tie in depth with the next one
      // that would blend; ordered the other way, that one blends first.
      if (rec) {
        for (int64_t j = k + 1; j < n; ++j) {
          const double* dj = rec_d + (size_t)L[(size_t)j].idx * REC_D;
          if (dj[D_DEPTH] - depth > kTieRel * (std::fabs(depth) + std::fabs(dj[D_DEPTH]))) break;
          if (L[(size_t)j].ambig || dj[D_DEPTH] > D) continue;
          if (pixel_weight(dj, px, py) >= set.tau) {
            o.fl |= 1;
            o.near.push_back({N_SWAP, k, j});
            break;
          }
        }
      }
      break;
    }
  }
}

// The outputs of one pixel from its candidate list: rgba = (C + T B, 1 - T)
// with B the background (or the mesh colour), T, the blend count, margin,
// flags and jump (see above; +inf when more than kMaxNear near decisions).
void composite_pixel(const std::vector<Cand>& L, const double* rec_d, const Set& set,
                     double px, double py, double D, const double* B, double* rgba,
                     double* T_out, int32_t* nb, double* margin, int32_t* flags,
                     double* jump) {
  WalkOut base, alt;
  walk_pixel(L, rec_d, set, px, py, D, nullptr, base);
  for (int ch = 0; ch < 3; ++ch) rgba[ch] = base.C[ch] + base.T * B[ch];
  rgba[3] = 1.0 - base.T;
  *T_out = base.T;
  *nb = base.nb;
  *margin = base.mrg;
  *flags = base.fl | (base.near.empty() ? 0 : 8);
  if (!jump) return;
  if ((int)base.near.size() > kMaxNear) {
    *jump = std::numeric_limits<double>::infinity();
    return;
  }
  double J = 0.0;
  for (const Near& nd : base.near) {
    walk_pixel(L, rec_d, set, px, py, D, &nd, alt);
    double m = std::fabs(alt.T - base.T);
    for (int ch = 0; ch < 3; ++ch)
      m = std::max(m, std::fabs((alt.C[ch] + alt.T * B[ch]) - rgba[ch]));
    J += m;
  }
  *jump = J;
}

// Candidates in walk order: ascending depth, then index.
void sort_walk_order(std::vector<Cand>& L, const double* rec_d) {
  std::sort(L.begin(), L.end(), [&](const Cand& a, const Cand& b) {
    const double da = rec_d[(size_t)a.idx * REC_D + D_DEPTH];
    const double db = rec_d[(size_t)b.idx * REC_D + D_DEPTH];
    if (da != db) return da < db;
    return a.idx < b.idx;
  });
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

// Eq. 3 by brute force at npix pixels (x, y pairs): every pixel walks every
// visible Gaussian (and every ambiguous culled one) in ascending (depth,
// index) order.
// Outputs per pixel: rgba (4), final transmittance T, number of blended
// Gaussians, the smallest relative margin to any discrete decision taken
// (skip at tau, clamp at alpha_max, stop at t_eps; capped at 1), flags:
//   1 = two blended Gaussians whose depths agree within float32 rounding
//       (a near tie, see kTieRel);
//   2 = a Gaussian culled within a relative 1e-5 of a threshold (or whose
//       footprint misses every pixel centre by less than the weight band)
//       would reach tau within the weight band here;
//   4 = a Gaussian with weight >= tau lies within a relative 1e-5 of the
//       mesh depth;
//   8 = the walk took at least one near decision (see walk_pixel);
// and, if `jump` is not NULL, the jump the pixel's near decisions straddle.
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
                      int32_t* flags, double* jump) {
  const Cam cam = load_cam(cam_in);
  const Set set = load_set(set_in);
  (void)cam;
  std::vector<Cand> L;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* iv = rec_i + (size_t)i * REC_I;
    if (iv[I_CULL] == C_VISIBLE) L.push_back({i, false});
    else if (iv[I_AMBIG]) L.push_back({i, true});
  }
  sort_walk_order(L, rec_d);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < npix; ++p) {
    const double D = mesh_depth ? mesh_depth[p] : std::numeric_limits<double>::infinity();
    composite_pixel(L, rec_d, set, pix[2 * p] + 0.5, pix[2 * p + 1] + 0.5, D,
                    mesh_rgb ? mesh_rgb + 3 * p : set.bg, rgba + 4 * p, T_out + p, n_blend + p,
                    margin + p, flags + p, jump ? jump + p : nullptr);
  }
  return 0;
}

// Eq. 3 by tiles: the same per-pixel walk over a shorter candidate list.
// Each visible or ambiguous Gaussian is listed in every tile (set.tw x
// set.th pixels) that its bounding box of {weight >= tau (1 - 1e-3)}
// overlaps; a tile's list is in ascending (depth, index) order.  A Gaussian
// missing from a pixel's list has weight below tau (1 - 1e-3) there, so the
// walk skips it in the brute-force list too, and it could only raise the
// margin above 1e-3: rgba, T, blend counts, flags and jumps equal the
// brute-force ones exactly, and margins equal them wherever either is below
// 1e-3.  Same arguments and outputs as orc_render_pixels.
int orc_render_tiled(int64_t n, const double* rec_d, const int32_t* rec_i,
                     const double* cam_in, const double* set_in, int64_t npix,
                     const int32_t* pix, const double* mesh_depth, const double* mesh_rgb,
                     double* rgba, double* T_out, int32_t* n_blend, double* margin,
                     int32_t* flags, double* jump) {
  const Cam cam = load_cam(cam_in);
  const Set set = load_set(set_in);
  const int tiles_x = (cam.W + set.tw - 1) / set.tw;
  const int tiles_y = (cam.H + set.th - 1) / set.th;
  const int64_t tiles = (int64_t)tiles_x * tiles_y;
  // tile rect of each candidate's listing bbox (empty: not listed)
  std::vector<int32_t> rect((size_t)n * 4, -1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* iv = rec_i + (size_t)i * REC_I;
    if (iv[I_CULL] != C_VISIBLE && !iv[I_AMBIG]) continue;
    const double* d = rec_d + (size_t)i * REC_D;
    const double q = 2.0 * std::log(d[D_OPAC] / (set.tau * (1.0 - 1e-3)));
    int box[4];
    if (!(q > 0.0) || !pixel_bbox(d, q, cam, box)) continue;
    int32_t* r = rect.data() + 4 * i;
    r[0] = box[0] / set.tw; r[1] = box[1] / set.tw;
    r[2] = box[2] / set.th; r[3] = box[3] / set.th;
  }
  std::vector<std::vector<Cand>> lists((size_t)tiles);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* r = rect.data() + 4 * i;
    if (r[0] < 0) continue;
    const bool amb = rec_i[(size_t)i * REC_I + I_CULL] != C_VISIBLE;
    for (int ty = r[2]; ty <= r[3]; ++ty)
      for (int tx = r[0]; tx <= r[1]; ++tx) lists[(size_t)ty * tiles_x + tx].push_back({i, amb});
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < tiles; ++t) sort_walk_order(lists[(size_t)t], rec_d);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t p = 0; p < npix; ++p) {
    const int x = pix[2 * p], y = pix[2 * p + 1];
    const double D = mesh_depth ? mesh_depth[p] : std::numeric_limits<double>::infinity();
    const std::vector<Cand>& L = lists[(size_t)(y / set.th) * tiles_x + x / set.tw];
    composite_pixel(L, rec_d, set, x + 0.5, y + 0.5, D, mesh_rgb ? mesh_rgb + 3 * p : set.bg,
                    rgba + 4 * p, T_out + p, n_blend + p, margin + p, flags + p,
                    jump ? jump + p : nullptr);
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

// Number of OpenMP threads later calls use (for timing on one core).
int orc_set_num_threads(int k) {
#ifdef _OPENMP
  if (k > 0) omp_set_num_threads(k);
#endif
  return 0;
}

}  // extern "C"
