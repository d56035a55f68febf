// FP64 CPU oracle for the online 3DGS optimize step -- TEST INFRASTRUCTURE ONLY.
//
// Only the test suite, the smoke check and the benchmark's CPU baseline may
// load this library.  It shares no code, header, table or constant with the
// HIP path.  It is deliberately plain: every pixel composites the Gaussians
// whose 3-sigma ellipse covers its centre, in depth order, as the definition
// says; no tiles are used for images.
//
// What it follows:
//  * the optimize loop: render the model from reference views, compare with
//    ground truth under the configured loss, update the parameters with the
//    configured learning rates (Sec. 3.1, overview);
//  * the optimized quantities are those of prior 3DGS work (Sec. 3.2.3):
//    means, log-scales, quaternions, opacities, SH coefficients (Sec. 3.1);
//    EWA projection and front-to-back alpha compositing are the standard
//    mathematics of that lineage (no formula is printed in the paper);
//  * tensor deltas relative to the previously transmitted state, grouped per
//    attribute, in Gaussian-ID order (Sec. 3.5);
//  * snapshot bookkeeping: baselines := current, epoch += 1 (Sec. 3.5).
//
// Readings where the paper is silent (all documented with the build):
//  constants are the FP32 values promoted to FP64; depth key is an FP32
//  expression without FMA; pixel membership is the 3-sigma ellipse test;
//  SH basis is the orthonormal real basis with the (-1)^m sign; L1 loss.
//
// Precision: FP64 throughout except the depth key, which is FP32 by definition.
// Build: g++ -O2 -fopenmp -ffp-contract=off -std=c++17 -shared -fPIC.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

// ---- thresholds: FP32 values promoted exactly ------------------------------
const double K_NEAR = (double)0.2f;
const double EPS_DIL = (double)0.3f;
const double ALPHA_MAX = (double)0.99f;
const double ALPHA_MIN = (double)(1.0f / 255.0f);
const double T_MIN = (double)1e-4f;
const double GUARD = (double)1.3f;
const double CUTOFF = -4.5;
// decision margins used to flag near-threshold events
const double M_CUTOFF = 1e-4;   // |P + 4.5|
const double M_AMIN = 1e-4;     // relative, |o e^P - alpha_min|
const double M_TMIN = 1e-4;     // relative, |T' - T_min|
const double M_AMAX = 1e-5;     // relative, |o e^P - alpha_max| (gradient only)
const int MAX_FLAGS = 4;

struct Cam {
  float R[9], t[3], campos[3], fx, fy, cx, cy;
  int32_t width, height;
};
static_assert(sizeof(Cam) == 84, "camera record layout");

struct Params {
  const float* mean;   // [3][n]
  const float* lsc;    // [3][n]
  const float* quat;   // [4][n] (w,x,y,z)
  const float* opac;   // [n]
  const float* sh;     // [(D+1)^2*3][n]
  int64_t n;
  int deg;
};

inline int nk_of(int deg) { return (deg + 1) * (deg + 1); }
inline int nparam_of(int deg) { return 3 + 3 + 4 + 1 + 3 * nk_of(deg); }

// ---- real spherical harmonics, orthonormal, with the (-1)^m sign -----------
// Y_{l,m} at unit direction (x,y,z), index k = l*l + l + m.  Constants are the
// normalisations sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the Legendre
// polynomial factors, written out per function.
void sh_eval(int deg, double x, double y, double z, double* Y) {
  const double s = 1.0 / std::sqrt(M_PI);
  Y[0] = 0.5 * s;
  if (deg < 1) return;
  const double c1 = std::sqrt(3.0) / 2.0 * s;
  Y[1] = -c1 * y;
  Y[2] = c1 * z;
  Y[3] = -c1 * x;
  if (deg < 2) return;
  const double c2a = std::sqrt(15.0) / 2.0 * s;
  const double c2b = std::sqrt(5.0) / 4.0 * s;
  const double c2c = std::sqrt(15.0) / 4.0 * s;
  Y[4] = c2a * x * y;
  Y[5] = -c2a * y * z;
  Y[6] = c2b * (2.0 * z * z - x * x - y * y);
  Y[7] = -c2a * x * z;
  Y[8] = c2c * (x * x - y * y);
  if (deg < 3) return;
  const double c3a = std::sqrt(35.0 / 2.0) / 4.0 * s;
  const double c3b = std::sqrt(105.0) / 2.0 * s;
  const double c3c = std::sqrt(21.0 / 2.0) / 4.0 * s;
  const double c3d = std::sqrt(7.0) / 4.0 * s;
  const double c3e = std::sqrt(105.0) / 4.0 * s;
  Y[9] = -c3a * y * (3.0 * x * x - y * y);
  Y[10] = c3b * x * y * z;
  Y[11] = -c3c * y * (4.0 * z * z - x * x - y * y);
  Y[12] = c3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
  Y[13] = -c3c * x * (4.0 * z * z - x * x - y * y);
  Y[14] = c3e * z * (x * x - y * y);
  Y[15] = -c3a * x * (x * x - 3.0 * y * y);
}

// Gradient of each polynomial Y_k(x,y,z) with respect to (x,y,z).
void sh_grad(int deg, double x, double y, double z, double (*dY)[3]) {
  const double s = 1.0 / std::sqrt(M_PI);
  for (int k = 0; k < nk_of(deg); ++k) dY[k][0] = dY[k][1] = dY[k][2] = 0.0;
  if (deg < 1) return;
  const double c1 = std::sqrt(3.0) / 2.0 * s;
  dY[1][1] = -c1;
  dY[2][2] = c1;
  dY[3][0] = -c1;
  if (deg < 2) return;
  const double c2a = std::sqrt(15.0) / 2.0 * s;
  const double c2b = std::sqrt(5.0) / 4.0 * s;
  const double c2c = std::sqrt(15.0) / 4.0 * s;
  dY[4][0] = c2a * y; dY[4][1] = c2a * x;
  dY[5][1] = -c2a * z; dY[5][2] = -c2a * y;
  dY[6][0] = -2.0 * c2b * x; dY[6][1] = -2.0 * c2b * y; dY[6][2] = 4.0 * c2b * z;
  dY[7][0] = -c2a * z; dY[7][2] = -c2a * x;
  dY[8][0] = 2.0 * c2c * x; dY[8][1] = -2.0 * c2c * y;
  if (deg < 3) return;
  const double c3a = std::sqrt(35.0 / 2.0) / 4.0 * s;
  const double c3b = std::sqrt(105.0) / 2.0 * s;
  const double c3c = std::sqrt(21.0 / 2.0) / 4.0 * s;
  const double c3d = std::sqrt(7.0) / 4.0 * s;
  const double c3e = std::sqrt(105.0) / 4.0 * s;
  // Y9 = -c3a (3 x^2 y - y^3)
  dY[9][0] = -c3a * 6.0 * x * y; dY[9][1] = -c3a * (3.0 * x * x - 3.0 * y * y);
  // Y10 = c3b x y z
  dY[10][0] = c3b * y * z; dY[10][1] = c3b * x * z; dY[10][2] = c3b * x * y;
  // Y11 = -c3c (4 y z^2 - x^2 y - y^3)
  dY[11][0] = -c3c * (-2.0 * x * y);
  dY[11][1] = -c3c * (4.0 * z * z - x * x - 3.0 * y * y);
  dY[11][2] = -c3c * (8.0 * y * z);
  // Y12 = c3d (2 z^3 - 3 x^2 z - 3 y^2 z)
  dY[12][0] = c3d * (-6.0 * x * z); dY[12][1] = c3d * (-6.0 * y * z);
  dY[12][2] = c3d * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
  // Y13 = -c3c (4 x z^2 - x^3 - x y^2)
  dY[13][0] = -c3c * (4.0 * z * z - 3.0 * x * x - y * y);
  dY[13][1] = -c3c * (-2.0 * x * y);
  dY[13][2] = -c3c * (8.0 * x * z);
  // Y14 = c3e (x^2 z - y^2 z)
  dY[14][0] = c3e * 2.0 * x * z; dY[14][1] = -c3e * 2.0 * y * z; dY[14][2] = c3e * (x * x - y * y);
  // Y15 = -c3a (x^3 - 3 x y^2)
  dY[15][0] = -c3a * (3.0 * x * x - 3.0 * y * y); dY[15][1] = -c3a * (-6.0 * x * y);
}

// ---- small dense linear algebra --------------------------------------------
struct M3 { double m[3][3]; };
M3 mul(const M3& a, const M3& b) {
  M3 r{};
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
    double s = 0; for (int k = 0; k < 3; ++k) s += a.m[i][k] * b.m[k][j]; r.m[i][j] = s;
  }
  return r;
}
M3 tr(const M3& a) { M3 r{}; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[j][i]; return r; }

// Rotation matrix of a unit quaternion (w,x,y,z).
M3 quat_rot(double w, double x, double y, double z) {
  M3 R;
  R.m[0][0] = 1 - 2 * (y * y + z * z); R.m[0][1] = 2 * (x * y - w * z);     R.m[0][2] = 2 * (x * z + w * y);
  R.m[1][0] = 2 * (x * y + w * z);     R.m[1][1] = 1 - 2 * (x * x + z * z); R.m[1][2] = 2 * (y * z - w * x);
  R.m[2][0] = 2 * (x * z - w * y);     R.m[2][1] = 2 * (y * z + w * x);     R.m[2][2] = 1 - 2 * (x * x + y * y);
  return R;
}

// ---- projection of one Gaussian into one view (stage "project/cull") -------
struct Proj {
  int visible;
  uint32_t zbits;
  double x[3];            // camera-space mean
  double u, w;            // projected mean (pixel units)
  double A, B, C;         // screen covariance (with dilation)
  double a, b, c;         // conic = inverse screen covariance
  double o;               // opacity
  double col[3], pre[3];  // colour after / before the clamp at 0
  int px0, px1, py0, py1; // pixel rectangle (inclusive) of the 3-sigma box
  double Mcov[3][3];      // camera-space covariance W Sigma W^T
  double J[2][3];
  int clx, cly;           // guard-band clamp active
};

bool finite_all(const Params& P, int64_t i) {
  auto f = [](float v) { return std::isfinite(v); };
  for (int k = 0; k < 3; ++k) if (!f(P.mean[k * P.n + i]) || !f(P.lsc[k * P.n + i])) return false;
  for (int k = 0; k < 4; ++k) if (!f(P.quat[k * P.n + i])) return false;
  if (!f(P.opac[i])) return false;
  for (int k = 0; k < 3 * nk_of(P.deg); ++k) if (!f(P.sh[k * P.n + i])) return false;
  return true;
}

// Depth key: the camera-space z of the mean evaluated in FP32 in the fixed
// order ((R20 x + R21 y) + R22 z) + t2, every operation rounded separately.
float depth32(const Cam& c, float mx, float my, float mz) {
  float a = c.R[6] * mx;
  float b = c.R[7] * my;
  float s = a + b;
  float d = c.R[8] * mz;
  s = s + d;
  s = s + c.t[2];
  return s;
}

void project_one(const Params& P, int64_t i, const Cam& cam, Proj& pr) {
  std::memset(&pr, 0, sizeof(pr));
  pr.visible = 0;
  if (!finite_all(P, i)) return;
  const int64_t n = P.n;
  const float mx = P.mean[i], my = P.mean[n + i], mz = P.mean[2 * n + i];
  const float z32 = depth32(cam, mx, my, mz);
  if (!(z32 >= (float)0.2f)) return;   // near cull on the FP32 depth
  std::memcpy(&pr.zbits, &z32, 4);

  M3 W;
  for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) W.m[r][c] = cam.R[r * 3 + c];
  double mu[3] = {mx, my, mz};
  for (int r = 0; r < 3; ++r)
    pr.x[r] = W.m[r][0] * mu[0] + W.m[r][1] * mu[1] + W.m[r][2] * mu[2] + (double)cam.t[r];
  const double xz = pr.x[2];
  const double fx = cam.fx, fy = cam.fy;

  // rotation and scale -> world covariance
  double q[4] = {P.quat[i], P.quat[n + i], P.quat[2 * n + i], P.quat[3 * n + i]};
  double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(qn > 0)) return;
  M3 Rq = quat_rot(q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn);
  double sc2[3];
  for (int k = 0; k < 3; ++k) { double e = std::exp((double)P.lsc[k * n + i]); sc2[k] = e * e; }
  M3 Sig{};
  for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) {
    double s = 0; for (int k = 0; k < 3; ++k) s += Rq.m[r][k] * sc2[k] * Rq.m[c][k]; Sig.m[r][c] = s;
  }
  M3 Mc = mul(mul(W, Sig), tr(W));
  std::memcpy(pr.Mcov, Mc.m, sizeof(Mc.m));

  // perspective Jacobian with the guard band on the tangent
  const double limx = GUARD * (0.5 * cam.width) / fx;
  const double limy = GUARD * (0.5 * cam.height) / fy;
  double tx = pr.x[0] / xz, ty = pr.x[1] / xz;
  pr.clx = (tx < -limx || tx > limx);
  pr.cly = (ty < -limy || ty > limy);
  tx = std::min(limx, std::max(-limx, tx));
  ty = std::min(limy, std::max(-limy, ty));
  double J[2][3] = {{fx / xz, 0.0, -fx * tx / xz}, {0.0, fy / xz, -fy * ty / xz}};
  std::memcpy(pr.J, J, sizeof(J));
  double S2[2][2];
  for (int r = 0; r < 2; ++r) for (int c = 0; c < 2; ++c) {
    double s = 0;
    for (int k = 0; k < 3; ++k) for (int l = 0; l < 3; ++l) s += J[r][k] * Mc.m[k][l] * J[c][l];
    S2[r][c] = s;
  }
  pr.A = S2[0][0] + EPS_DIL;
  pr.B = S2[0][1];
  pr.C = S2[1][1] + EPS_DIL;
  const double det = pr.A * pr.C - pr.B * pr.B;
  if (!(det > 0) || !std::isfinite(det)) return;
  pr.a = pr.C / det;
  pr.b = -pr.B / det;
  pr.c = pr.A / det;
  pr.u = fx * pr.x[0] / xz + (double)cam.cx;
  pr.w = fy * pr.x[1] / xz + (double)cam.cy;
  if (!std::isfinite(pr.u) || !std::isfinite(pr.w)) return;

  // pixel rectangle of the 3-sigma box (tight axis-aligned bound, with slack)
  const double hx = 3.0 * std::sqrt(pr.A) * (1.0 + std::ldexp(1.0, -10));
  const double hy = 3.0 * std::sqrt(pr.C) * (1.0 + std::ldexp(1.0, -10));
  double lo_x = std::ceil(pr.u - hx - 0.5), hi_x = std::floor(pr.u + hx - 0.5);
  double lo_y = std::ceil(pr.w - hy - 0.5), hi_y = std::floor(pr.w + hy - 0.5);
  lo_x = std::max(lo_x, 0.0); lo_y = std::max(lo_y, 0.0);
  hi_x = std::min(hi_x, (double)(cam.width - 1)); hi_y = std::min(hi_y, (double)(cam.height - 1));
  if (lo_x > hi_x || lo_y > hi_y) return;
  pr.px0 = (int)lo_x; pr.px1 = (int)hi_x; pr.py0 = (int)lo_y; pr.py1 = (int)hi_y;

  pr.o = 1.0 / (1.0 + std::exp(-(double)P.opac[i]));

  // view-dependent colour
  double dv[3] = {mu[0] - cam.campos[0], mu[1] - cam.campos[1], mu[2] - cam.campos[2]};
  double dl = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  double Y[16];
  sh_eval(P.deg, dv[0] / dl, dv[1] / dl, dv[2] / dl, Y);
  for (int ch = 0; ch < 3; ++ch) {
    double s = 0.5;
    for (int k = 0; k < nk_of(P.deg); ++k) s += (double)P.sh[(k * 3 + ch) * n + i] * Y[k];
    pr.pre[ch] = s;
    pr.col[ch] = std::max(0.0, s);
  }
  pr.visible = 1;
}

// ---- per-pixel compositing ---------------------------------------------------
struct Contrib {
  int32_t j;       // index into the view's visible list
  double alpha, G; // alpha and Gaussian falloff e^P
  double dx, dy;   // pixel centre minus projected mean
  int clamped;     // alpha hit alpha_max (derivative w.r.t. o and P is 0)
};

struct PixResult {
  double C[3];
  double T;
  int n;
  int flags;       // near-threshold decisions met on this path (capped count)
};

struct ViewData {
  const Cam* cam;
  std::vector<int64_t> ids;          // Gaussian index per visible entry, depth order
  std::vector<Proj> pr;              // projection per visible entry
  std::vector<std::vector<int32_t>> rows;  // per image row: visible entries covering it
};

// Walks one pixel's candidates in depth order.  `mask` flips the k-th
// flagged decision (k < MAX_FLAGS) met on this path, giving the alternative
// outcomes of near-threshold events.
void composite_pixel(const ViewData& vd, int px, int py, const double bg[3], unsigned mask,
                     PixResult& res, std::vector<Contrib>* contribs) {
  double T = 1.0, Cc[3] = {0, 0, 0};
  int n = 0, nflag = 0;
  if (contribs) contribs->clear();
  const double cxp = px + 0.5, cyp = py + 0.5;
  auto decide = [&](bool exact, bool near) -> bool {
    if (!near) return exact;
    bool flip = false;
    if (nflag < MAX_FLAGS) flip = (mask >> nflag) & 1u;
    ++nflag;
    return flip ? !exact : exact;
  };
  for (int32_t e : vd.rows[py]) {
    const Proj& g = vd.pr[e];
    if (px < g.px0 || px > g.px1) continue;
    const double dx = cxp - g.u, dy = cyp - g.w;
    const double P = -0.5 * (g.a * dx * dx + g.c * dy * dy) - g.b * dx * dy;
    const bool outside = decide(P < CUTOFF, std::fabs(P - CUTOFF) < M_CUTOFF);
    if (outside) continue;
    const double G = std::exp(P);
    const double oG = g.o * G;
    const bool clamped = decide(oG >= ALPHA_MAX, std::fabs(oG - ALPHA_MAX) < M_AMAX * ALPHA_MAX);
    const double alpha = clamped ? ALPHA_MAX : oG;
    const bool skip = decide(alpha < ALPHA_MIN, std::fabs(oG - ALPHA_MIN) < M_AMIN * ALPHA_MIN);
    if (skip) continue;
    const double Tn = T * (1.0 - alpha);
    const bool stop = decide(Tn < T_MIN, std::fabs(Tn - T_MIN) < M_TMIN * T_MIN);
    if (stop) break;
    for (int ch = 0; ch < 3; ++ch) Cc[ch] += g.col[ch] * alpha * T;
    if (contribs) contribs->push_back({e, alpha, G, dx, dy, clamped ? 1 : 0});
    T = Tn;
    ++n;
  }
  for (int ch = 0; ch < 3; ++ch) res.C[ch] = Cc[ch] + T * bg[ch];
  res.T = T;
  res.n = n;
  res.flags = nflag;
}

// 2D adjoint of one pixel for upstream G (3-vector): per contributor, the
// derivative of the pixel with respect to (u, w, a, b, c, o, r, g, b).
void pixel_backward(const ViewData& vd, const std::vector<Contrib>& cs, double Tfinal,
                    const double bg[3], const double Gup[3], std::vector<std::pair<int32_t, std::array<double, 9>>>* out) {
  out->clear();
  double T = Tfinal;
  double S[3] = {bg[0], bg[1], bg[2]};
  for (int k = (int)cs.size() - 1; k >= 0; --k) {
    const Contrib& c = cs[k];
    const Proj& g = vd.pr[c.j];
    const double a = c.alpha;
    const double Tj = T / (1.0 - a);
    std::array<double, 9> d{};
    double dL_da = 0;
    for (int ch = 0; ch < 3; ++ch) {
      d[6 + ch] = a * Tj * Gup[ch];
      dL_da += Tj * (g.col[ch] - S[ch]) * Gup[ch];
    }
    if (!c.clamped) {
      const double dL_dP = dL_da * a;          // alpha = o e^P
      d[5] = dL_da * c.G;                      // d alpha / d o
      // P = -1/2 (a dx^2 + c dy^2) - b dx dy, dx = px - u, dy = py - w
      d[0] = dL_dP * (g.a * c.dx + g.b * c.dy);
      d[1] = dL_dP * (g.b * c.dx + g.c * c.dy);
      d[2] = dL_dP * (-0.5 * c.dx * c.dx);
      d[3] = dL_dP * (-c.dx * c.dy);
      d[4] = dL_dP * (-0.5 * c.dy * c.dy);
    }
    for (int ch = 0; ch < 3; ++ch) S[ch] = a * g.col[ch] + (1.0 - a) * S[ch];
    T = Tj;
    out->push_back({c.j, d});
  }
}

// Chain rule from 2D quantities to the Gaussian's parameters in one view:
// g3 (length nparam) += J^T g2.
void chain_rule(const Params& P, int64_t i, const Cam& cam, const Proj& pr, const double g2[9], double* g3) {
  const int64_t n = P.n;
  const double fx = cam.fx, fy = cam.fy;
  const double xz = pr.x[2];
  // opacity
  g3[10] += g2[5] * pr.o * (1.0 - pr.o);
  // colour -> SH coefficients and view direction
  double mu[3] = {P.mean[i], P.mean[n + i], P.mean[2 * n + i]};
  double dv[3] = {mu[0] - cam.campos[0], mu[1] - cam.campos[1], mu[2] - cam.campos[2]};
  double dl = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  double d[3] = {dv[0] / dl, dv[1] / dl, dv[2] / dl};
  double Y[16], dY[16][3];
  sh_eval(P.deg, d[0], d[1], d[2], Y);
  sh_grad(P.deg, d[0], d[1], d[2], dY);
  double dL_dd[3] = {0, 0, 0};
  for (int ch = 0; ch < 3; ++ch) {
    const double gc = pr.pre[ch] > 0 ? g2[6 + ch] : 0.0;
    for (int k = 0; k < nk_of(P.deg); ++k) {
      g3[11 + k * 3 + ch] += Y[k] * gc;
      const double f = P.sh[(k * 3 + ch) * n + i];
      for (int a = 0; a < 3; ++a) dL_dd[a] += gc * f * dY[k][a];
    }
  }
  double dL_dmu[3];
  {
    const double dd = d[0] * dL_dd[0] + d[1] * dL_dd[1] + d[2] * dL_dd[2];
    for (int a = 0; a < 3; ++a) dL_dmu[a] = (dL_dd[a] - d[a] * dd) / dl;
  }
  // conic (a,b,c) -> screen covariance: dL/dSigma2 = -Q (dL/dQ) Q, with the
  // symmetric matrix dL/dQ = [[ga, gb/2], [gb/2, gc]].
  const double Q[2][2] = {{pr.a, pr.b}, {pr.b, pr.c}};
  const double GQ[2][2] = {{g2[2], 0.5 * g2[3]}, {0.5 * g2[3], g2[4]}};
  double GS[2][2];
  for (int r = 0; r < 2; ++r) for (int c = 0; c < 2; ++c) {
    double s = 0;
    for (int k = 0; k < 2; ++k) for (int l = 0; l < 2; ++l) s += Q[r][k] * GQ[k][l] * Q[l][c];
    GS[r][c] = -s;
  }
  // Sigma2 = J M J^T + eps I: dL/dM = J^T GS J, dL/dJ = 2 GS J M
  double GM[3][3], GJ[2][3];
  for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) {
    double s = 0;
    for (int k = 0; k < 2; ++k) for (int l = 0; l < 2; ++l) s += pr.J[k][r] * GS[k][l] * pr.J[l][c];
    GM[r][c] = s;
  }
  for (int r = 0; r < 2; ++r) for (int c = 0; c < 3; ++c) {
    double s = 0;
    for (int k = 0; k < 2; ++k) for (int l = 0; l < 3; ++l) s += GS[r][k] * pr.J[k][l] * pr.Mcov[l][c];
    GJ[r][c] = 2.0 * s;
  }
  // camera-space mean: through u, w and through J
  double gx[3] = {0, 0, 0};
  gx[0] += g2[0] * fx / xz;
  gx[2] += -g2[0] * fx * pr.x[0] / (xz * xz);
  gx[1] += g2[1] * fy / xz;
  gx[2] += -g2[1] * fy * pr.x[1] / (xz * xz);
  // J = [[fx/z, 0, -fx tx/z], [0, fy/z, -fy ty/z]], tx = x/z unless clamped
  gx[2] += GJ[0][0] * (-fx / (xz * xz)) + GJ[1][1] * (-fy / (xz * xz));
  if (!pr.clx) {  // J02 = -fx x / z^2
    gx[0] += GJ[0][2] * (-fx / (xz * xz));
    gx[2] += GJ[0][2] * (2.0 * fx * pr.x[0] / (xz * xz * xz));
  } else {        // J02 = -fx c / z with c constant
    const double tcl = -pr.J[0][2] * xz / fx;
    gx[2] += GJ[0][2] * (fx * tcl / (xz * xz));
  }
  if (!pr.cly) {
    gx[1] += GJ[1][2] * (-fy / (xz * xz));
    gx[2] += GJ[1][2] * (2.0 * fy * pr.x[1] / (xz * xz * xz));
  } else {
    const double tcl = -pr.J[1][2] * xz / fy;
    gx[2] += GJ[1][2] * (fy * tcl / (xz * xz));
  }
  // x = W mu + t
  for (int a = 0; a < 3; ++a) {
    double s = 0;
    for (int r = 0; r < 3; ++r) s += (double)cam.R[r * 3 + a] * gx[r];
    g3[a] += s + dL_dmu[a];
  }
  // M = W Sigma W^T -> dL/dSigma = W^T GM W
  M3 Wm;
  for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) Wm.m[r][c] = cam.R[r * 3 + c];
  M3 GMm; std::memcpy(GMm.m, GM, sizeof(GM));
  M3 G3 = mul(mul(tr(Wm), GMm), Wm);
  // Sigma = Rq diag(e^{2s}) Rq^T
  double q[4] = {P.quat[i], P.quat[n + i], P.quat[2 * n + i], P.quat[3 * n + i]};
  double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double rw = q[0] / qn, rx = q[1] / qn, ry = q[2] / qn, rz = q[3] / qn;
  M3 Rq = quat_rot(rw, rx, ry, rz);
  double e2[3];
  for (int k = 0; k < 3; ++k) { double e = std::exp((double)P.lsc[k * n + i]); e2[k] = e * e; }
  for (int k = 0; k < 3; ++k) {
    double s = 0;
    for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) s += Rq.m[r][k] * G3.m[r][c] * Rq.m[c][k];
    g3[3 + k] += 2.0 * e2[k] * s;
  }
  double GR[3][3];  // dL/dRq = 2 G3 Rq D
  for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) {
    double s = 0; for (int k = 0; k < 3; ++k) s += G3.m[r][k] * Rq.m[k][c];
    GR[r][c] = 2.0 * s * e2[c];
  }
  double gr[4];
  gr[0] = 2 * (-rz * GR[0][1] + ry * GR[0][2] + rz * GR[1][0] - rx * GR[1][2] - ry * GR[2][0] + rx * GR[2][1]);
  gr[1] = 2 * (ry * GR[0][1] + rz * GR[0][2] + ry * GR[1][0] - 2 * rx * GR[1][1] - rw * GR[1][2] + rz * GR[2][0] + rw * GR[2][1] - 2 * rx * GR[2][2]);
  gr[2] = 2 * (-2 * ry * GR[0][0] + rx * GR[0][1] + rw * GR[0][2] + rx * GR[1][0] + rz * GR[1][2] - rw * GR[2][0] + rz * GR[2][1] - 2 * ry * GR[2][2]);
  gr[3] = 2 * (-2 * rz * GR[0][0] - rw * GR[0][1] + rx * GR[0][2] + rw * GR[1][0] - 2 * rz * GR[1][1] + ry * GR[1][2] + rx * GR[2][0] + ry * GR[2][1]);
  const double rho[4] = {rw, rx, ry, rz};
  const double dot = rho[0] * gr[0] + rho[1] * gr[1] + rho[2] * gr[2] + rho[3] * gr[3];
  for (int k = 0; k < 4; ++k) g3[6 + k] += (gr[k] - rho[k] * dot) / qn;
}

// Builds the visible set of one view in depth order and the per-row lists.
void build_view(const Params& P, const Cam& cam, ViewData& vd, int row0, int row1) {
  vd.cam = &cam;
  const int64_t n = P.n;
  std::vector<Proj> all(n);
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) project_one(P, i, cam, all[i]);
  std::vector<int64_t> vis;
  for (int64_t i = 0; i < n; ++i) if (all[i].visible) vis.push_back(i);
  // order by (FP32 depth bits, Gaussian index)
  std::sort(vis.begin(), vis.end(), [&](int64_t x, int64_t y) {
    if (all[x].zbits != all[y].zbits) return all[x].zbits < all[y].zbits;
    return x < y;
  });
  vd.ids = vis;
  vd.pr.resize(vis.size());
  for (size_t e = 0; e < vis.size(); ++e) vd.pr[e] = all[vis[e]];
  vd.rows.assign(cam.height, {});
  for (size_t e = 0; e < vis.size(); ++e) {
    const Proj& g = vd.pr[e];
    for (int y = std::max(g.py0, row0); y <= std::min(g.py1, row1 - 1); ++y) vd.rows[y].push_back((int32_t)e);
  }
}

Params make_params(const float* mean, const float* lsc, const float* quat, const float* opac, const float* sh,
                   int64_t n, int deg) {
  Params P;
  P.mean = mean; P.lsc = lsc; P.quat = quat; P.opac = opac; P.sh = sh; P.n = n; P.deg = deg;
  return P;
}

}  // namespace

extern "C" {

int or_version() { return 1; }

// Evaluate the SH basis (and its gradient) at unit direction d.
void or_sh_basis(int deg, const double* d, double* Y, double* dY) {
  sh_eval(deg, d[0], d[1], d[2], Y);
  if (dY) {
    double g[16][3];
    sh_grad(deg, d[0], d[1], d[2], g);
    for (int k = 0; k < nk_of(deg); ++k) for (int a = 0; a < 3; ++a) dY[k * 3 + a] = g[k][a];
  }
}

// Stage "project/cull" for all views.  Per (v, i):
//  out_vis[v*n+i]            1 if visible
//  out_zbits                 FP32 depth key bits
//  out_rec[(v*n+i)*16 + k]   u, w, A, B, C, a, b, c, o, r, g, b, pre_r, pre_g, pre_b, x_z
//  out_rect[(v*n+i)*4 + k]   px0, py0, px1, py1 (inclusive pixel rectangle)
void or_project(const float* mean, const float* lsc, const float* quat, const float* opac, const float* sh,
                int64_t n, int deg, const void* cams_v, int nv,
                uint8_t* out_vis, uint32_t* out_zbits, double* out_rec, int32_t* out_rect) {
  const Cam* cams = (const Cam*)cams_v;
  Params P = make_params(mean, lsc, quat, opac, sh, n, deg);
  for (int v = 0; v < nv; ++v) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      Proj pr;
      project_one(P, i, cams[v], pr);
      const int64_t o = (int64_t)v * n + i;
      out_vis[o] = (uint8_t)pr.visible;
      out_zbits[o] = pr.visible ? pr.zbits : 0u;
      double* r = out_rec + o * 16;
      const double vals[16] = {pr.u, pr.w, pr.A, pr.B, pr.C, pr.a, pr.b, pr.c, pr.o,
                               pr.col[0], pr.col[1], pr.col[2], pr.pre[0], pr.pre[1], pr.pre[2], pr.x[2]};
      for (int k = 0; k < 16; ++k) r[k] = pr.visible ? vals[k] : 0.0;
      int32_t* rc = out_rect + o * 4;
      rc[0] = pr.visible ? pr.px0 : -1; rc[1] = pr.visible ? pr.py0 : -1;
      rc[2] = pr.visible ? pr.px1 : -1; rc[3] = pr.visible ? pr.py1 : -1;
    }
  }
}

// Per-(view, tile) lists in the order (tile, depth bits, Gaussian index).
// Global tile id = tile_base[v] + ty * tiles_x(v) + tx, views in order.
// Returns K; writes up to `cap` values (v*n + i) and [start, end) per tile.
int64_t or_tile_lists(const float* mean, const float* lsc, const float* quat, const float* opac, const float* sh,
                      int64_t n, int deg, const void* cams_v, int nv, int tile_w, int tile_h,
                      uint32_t* out_vals, int64_t cap, uint32_t* out_ranges /* [tiles][2] */) {
  const Cam* cams = (const Cam*)cams_v;
  Params P = make_params(mean, lsc, quat, opac, sh, n, deg);
  struct Key { uint32_t tile, z; uint32_t val; };
  std::vector<Key> keys;
  std::vector<int64_t> tile_base(nv + 1, 0);
  for (int v = 0; v < nv; ++v) {
    const int tx = (cams[v].width + tile_w - 1) / tile_w, ty = (cams[v].height + tile_h - 1) / tile_h;
    tile_base[v + 1] = tile_base[v] + (int64_t)tx * ty;
  }
  for (int v = 0; v < nv; ++v) {
    std::vector<Proj> pr(n);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) project_one(P, i, cams[v], pr[i]);
    const int tiles_x = (cams[v].width + tile_w - 1) / tile_w;
    for (int64_t i = 0; i < n; ++i) {
      if (!pr[i].visible) continue;
      for (int ty = pr[i].py0 / tile_h; ty <= pr[i].py1 / tile_h; ++ty)
        for (int tx = pr[i].px0 / tile_w; tx <= pr[i].px1 / tile_w; ++tx)
          keys.push_back({(uint32_t)(tile_base[v] + (int64_t)ty * tiles_x + tx), pr[i].zbits,
                          (uint32_t)((int64_t)v * n + i)});
    }
  }
  std::sort(keys.begin(), keys.end(), [](const Key& x, const Key& y) {
    if (x.tile != y.tile) return x.tile < y.tile;
    if (x.z != y.z) return x.z < y.z;
    return x.val < y.val;
  });
  const int64_t K = (int64_t)keys.size();
  for (int64_t k = 0; k < K && k < cap; ++k) out_vals[k] = keys[k].val;
  for (int64_t t = 0; t < tile_base[nv]; ++t) { out_ranges[2 * t] = 0; out_ranges[2 * t + 1] = 0; }
  for (int64_t k = 0; k < K; ++k) {
    const uint32_t t = keys[k].tile;
    if (k == 0 || keys[k - 1].tile != t) out_ranges[2 * t] = (uint32_t)k;
    if (k == K - 1 || keys[k + 1].tile != t) out_ranges[2 * t + 1] = (uint32_t)(k + 1);
  }
  return K;
}

// Forward render of all views (rows [row0,row1) of each view, or all rows if
// row1 <= row0).  Images are planar CHW per view, views packed in order.
// Writes the primary result, T_final, n_contrib and the number of
// near-threshold decisions met per pixel.
void or_render(const float* mean, const float* lsc, const float* quat, const float* opac, const float* sh,
               int64_t n, int deg, const void* cams_v, int nv, const double* bg,
               int row0, int row1, double* out_img, double* out_T, int32_t* out_n, int32_t* out_flags) {
  const Cam* cams = (const Cam*)cams_v;
  Params P = make_params(mean, lsc, quat, opac, sh, n, deg);
  int64_t pix_off = 0;
  for (int v = 0; v < nv; ++v) {
    const int W = cams[v].width, H = cams[v].height;
    const int r0 = (row1 > row0) ? std::max(0, row0) : 0;
    const int r1 = (row1 > row0) ? std::min(H, row1) : H;
    ViewData vd;
    build_view(P, cams[v], vd, r0, r1);
    const int64_t HW = (int64_t)H * W;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int y = r0; y < r1; ++y) {
      for (int x = 0; x < W; ++x) {
        PixResult res;
        composite_pixel(vd, x, y, bg, 0u, res, nullptr);
        const int64_t p = (int64_t)y * W + x;
        for (int ch = 0; ch < 3; ++ch) out_img[3 * pix_off + ch * HW + p] = res.C[ch];
        out_T[pix_off + p] = res.T;
        out_n[pix_off + p] = res.n;
        out_flags[pix_off + p] = res.flags;
      }
    }
    pix_off += HW;
  }
}

// All outcomes of one pixel's near-threshold decisions (at most 16).
// out_count[q] = number of distinct paths; each path writes (r, g, b, T, n).
void or_render_alternatives(const float* mean, const float* lsc, const float* quat, const float* opac, const float* sh,
                           int64_t n, int deg, const void* cams_v, int view, const double* bg,
                           const int32_t* pix_xy, int npix, double* out /* [npix][16][5] */, int32_t* out_count) {
  const Cam* cams = (const Cam*)cams_v;
  Params P = make_params(mean, lsc, quat, opac, sh, n, deg);
  ViewData vd;
  build_view(P, cams[view], vd, 0, cams[view].height);
  #pragma omp parallel for schedule(dynamic, 16)
  for (int q = 0; q < npix; ++q) {
    const int x = pix_xy[2 * q], y = pix_xy[2 * q + 1];
    int cnt = 0;
    for (unsigned mask = 0; mask < (1u << MAX_FLAGS); ++mask) {
      PixResult res;
      composite_pixel(vd, x, y, bg, mask, res, nullptr);
      // a mask whose highest set bit lies beyond the flags met repeats a path
      const int used = std::min(res.flags, MAX_FLAGS);
      if (mask >> used) continue;
      double* o = out + ((int64_t)q * 16 + cnt) * 5;
      o[0] = res.C[0]; o[1] = res.C[1]; o[2] = res.C[2]; o[3] = res.T; o[4] = res.n;
      ++cnt;
    }
    out_count[q] = cnt;
  }
}

// Forward + backward of all views.
//  mode 0: upstream dL/dimage given in `up` (layout of the images).
//  mode 1: L1 loss against the target in `up`, per-view weight w_v
//          (loss_mode 0: w_v = 1, sum; loss_mode 1: w_v = 1/(3 H W), mean).
// Outputs (per Gaussian, layout of the parameters [nparam][n]):
//  g3     gradient summed over views
//  s3     magnitude scale: sum over views of |J|^T (sum over pixels of |2D terms|)
//  k3     slack: |J|^T (largest change of the 2D terms over the alternative
//         outcomes of near-threshold decisions and L1 sign ambiguities)
//  t3     depth-weighted scale: |J|^T (sum over pixels of |2D terms| times
//         E_p = sum over the pixel's composited splats of 1/(1 - alpha)),
//         the condition number of the pixel's transmittance product: an
//         evaluation whose alphas carry relative error u has transmittances
//         off by at most about u * E_p relative.
//  loss   (mode 1) the loss value; also images/T/n of the primary path.
// `kink` is the |img - target| margin below which an L1 sign is ambiguous.
void or_backward(const float* mean, const float* lsc, const float* quat, const float* opac, const float* sh,
                 int64_t n, int deg, const void* cams_v, int nv, const double* bg,
                 const float* up, int mode, int loss_mode, double kink,
                 double* g3, double* s3, double* k3, double* t3, double* loss_out, double* out_img) {
  const Cam* cams = (const Cam*)cams_v;
  Params P = make_params(mean, lsc, quat, opac, sh, n, deg);
  const int np = nparam_of(deg);
  std::memset(g3, 0, sizeof(double) * np * n);
  std::memset(s3, 0, sizeof(double) * np * n);
  std::memset(k3, 0, sizeof(double) * np * n);
  std::memset(t3, 0, sizeof(double) * np * n);
  double loss = 0.0;
  int64_t pix_off = 0;
  using Acc = std::vector<std::pair<int32_t, std::array<double, 9>>>;
  for (int v = 0; v < nv; ++v) {
    const Cam& cam = cams[v];
    const int W = cam.width, H = cam.height;
    const int64_t HW = (int64_t)H * W;
    const double wv = (mode == 1 && loss_mode == 1) ? 1.0 / (3.0 * (double)HW) : 1.0;
    ViewData vd;
    build_view(P, cam, vd, 0, H);
    const size_t nvis = vd.ids.size();
    const int nth = omp_get_max_threads();
    std::vector<std::vector<double>> accG(nth), accS(nth), accK(nth), accT(nth);
    std::vector<double> lossT(nth, 0.0);
    #pragma omp parallel
    {
      const int tid = omp_get_thread_num();
      accG[tid].assign(nvis * 9, 0.0); accS[tid].assign(nvis * 9, 0.0); accK[tid].assign(nvis * 9, 0.0);
      accT[tid].assign(nvis * 9, 0.0);
      std::vector<Contrib> cs, cs_alt;
      Acc d0, db, dk;
      std::vector<std::array<double, 9>> dmax;
      std::vector<int32_t> touched;
      #pragma omp for schedule(dynamic, 1)
      for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
          const int64_t p = (int64_t)y * W + x;
          PixResult res;
          composite_pixel(vd, x, y, bg, 0u, res, &cs);
          if (out_img) for (int ch = 0; ch < 3; ++ch) out_img[3 * pix_off + ch * HW + p] = res.C[ch];
          double Gup[3];
          auto upstream = [&](const PixResult& r, double* Gv) {
            for (int ch = 0; ch < 3; ++ch) {
              const double u = up[3 * pix_off + ch * HW + p];
              if (mode == 0) Gv[ch] = u;
              else { const double df = r.C[ch] - u; Gv[ch] = wv * (double)((df > 0) - (df < 0)); }
            }
          };
          upstream(res, Gup);
          if (mode == 1)
            for (int ch = 0; ch < 3; ++ch) lossT[tid] += wv * std::fabs(res.C[ch] - (double)up[3 * pix_off + ch * HW + p]);
          pixel_backward(vd, cs, res.T, bg, Gup, &d0);
          double Ep = 0.0;
          for (const Contrib& c : cs) Ep += 1.0 / (1.0 - c.alpha);
          for (auto& e : d0)
            for (int f = 0; f < 9; ++f) {
              accG[tid][e.first * 9 + f] += e.second[f];
              accS[tid][e.first * 9 + f] += std::fabs(e.second[f]);
              accT[tid][e.first * 9 + f] += std::fabs(e.second[f]) * Ep;
            }
          // L1 sign ambiguity on the primary path: the channel's upstream may
          // be -w, 0 or +w, so the terms may move by up to 2 w |d/dG_ch|.
          if (mode == 1) {
            for (int ch = 0; ch < 3; ++ch) {
              const double df = res.C[ch] - up[3 * pix_off + ch * HW + p];
              if (std::fabs(df) >= kink) continue;
              double Gc[3] = {0, 0, 0}; Gc[ch] = wv;
              pixel_backward(vd, cs, res.T, bg, Gc, &dk);
              for (auto& e : dk) for (int f = 0; f < 9; ++f) accK[tid][e.first * 9 + f] += 2.0 * std::fabs(e.second[f]);
            }
          }
          if (res.flags == 0) continue;
          // alternative outcomes of near-threshold decisions
          touched.clear(); dmax.clear();
          auto slot = [&](int32_t j) -> std::array<double, 9>& {
            for (size_t s = 0; s < touched.size(); ++s) if (touched[s] == j) return dmax[s];
            touched.push_back(j); dmax.push_back({}); return dmax.back();
          };
          for (unsigned mask = 1; mask < (1u << MAX_FLAGS); ++mask) {
            PixResult rb;
            composite_pixel(vd, x, y, bg, mask, rb, &cs_alt);
            if (mask >> std::min(rb.flags, MAX_FLAGS)) continue;
            double Gb[3];
            upstream(rb, Gb);
            pixel_backward(vd, cs_alt, rb.T, bg, Gb, &db);
            // difference of the 2D terms against the primary path
            std::vector<std::pair<int32_t, std::array<double, 9>>> diff;
            for (auto& e : db) diff.push_back(e);
            for (auto& e : d0) {
              bool found = false;
              for (auto& f : diff) if (f.first == e.first) {
                for (int k = 0; k < 9; ++k) f.second[k] -= e.second[k];
                found = true; break;
              }
              if (!found) { auto m = e; for (int k = 0; k < 9; ++k) m.second[k] = -m.second[k]; diff.push_back(m); }
            }
            for (auto& f : diff) {
              auto& s = slot(f.first);
              for (int k = 0; k < 9; ++k) s[k] = std::max(s[k], std::fabs(f.second[k]));
            }
            if (mode == 1) {  // sign ambiguity on the alternative path as well
              for (int ch = 0; ch < 3; ++ch) {
                const double df = rb.C[ch] - up[3 * pix_off + ch * HW + p];
                if (std::fabs(df) >= kink) continue;
                double Gc[3] = {0, 0, 0}; Gc[ch] = wv;
                pixel_backward(vd, cs_alt, rb.T, bg, Gc, &dk);
                for (auto& e : dk) { auto& s = slot(e.first); for (int k = 0; k < 9; ++k) s[k] += 2.0 * std::fabs(e.second[k]); }
              }
            }
          }
          for (size_t s = 0; s < touched.size(); ++s)
            for (int k = 0; k < 9; ++k) accK[tid][touched[s] * 9 + k] += dmax[s][k];
        }
      }
    }
    for (int t = 0; t < nth; ++t) loss += lossT[t];
    // reduce thread accumulators
    std::vector<double> G2(nvis * 9, 0.0), S2(nvis * 9, 0.0), K2(nvis * 9, 0.0), T2(nvis * 9, 0.0);
    for (int t = 0; t < nth; ++t)
      for (size_t k = 0; k < nvis * 9; ++k) {
        G2[k] += accG[t][k]; S2[k] += accS[t][k]; K2[k] += accK[t][k]; T2[k] += accT[t][k];
      }
    // chain rule per visible Gaussian; |J| from unit 2D vectors
    #pragma omp parallel
    {
      std::vector<double> gl(np), col(np);
      #pragma omp for schedule(dynamic, 64)
      for (size_t e = 0; e < nvis; ++e) {
        const int64_t i = vd.ids[e];
        std::fill(gl.begin(), gl.end(), 0.0);
        chain_rule(P, i, cam, vd.pr[e], &G2[e * 9], gl.data());
        std::vector<double> sl(np, 0.0), kl(np, 0.0), tl(np, 0.0);
        for (int f = 0; f < 9; ++f) {
          if (S2[e * 9 + f] == 0.0 && K2[e * 9 + f] == 0.0) continue;
          double unit[9] = {0}; unit[f] = 1.0;
          std::fill(col.begin(), col.end(), 0.0);
          chain_rule(P, i, cam, vd.pr[e], unit, col.data());
          for (int k = 0; k < np; ++k) {
            sl[k] += std::fabs(col[k]) * S2[e * 9 + f];
            kl[k] += std::fabs(col[k]) * K2[e * 9 + f];
            tl[k] += std::fabs(col[k]) * T2[e * 9 + f];
          }
        }
        // each Gaussian appears once per view: no write conflicts within a view
        for (int k = 0; k < np; ++k) {
          g3[k * n + i] += gl[k];
          s3[k * n + i] += sl[k];
          k3[k * n + i] += kl[k];
          t3[k * n + i] += tl[k];
        }
      }
    }
    pix_off += HW;
  }
  if (loss_out) *loss_out = loss;
}

// Adam (torch.optim.Adam semantics: no weight decay, no amsgrad) on one
// tensor; FP32 inputs promoted, FP64 outputs.  `step` is 1-based.
void or_adam(const float* theta, const float* g, const float* m, const float* v, int64_t count,
             float lr, float beta1, float beta2, float eps, int step,
             double* theta_out, double* m_out, double* v_out) {
  const double b1 = beta1, b2 = beta2;
  const double bc1 = 1.0 - std::pow(b1, step), bc2 = 1.0 - std::pow(b2, step);
  for (int64_t k = 0; k < count; ++k) {
    const double gk = g[k];
    const double mk = b1 * (double)m[k] + (1.0 - b1) * gk;
    const double vk = b2 * (double)v[k] + (1.0 - b2) * gk * gk;
    m_out[k] = mk; v_out[k] = vk;
    theta_out[k] = (double)theta[k] - (double)lr * (mk / bc1) / (std::sqrt(vk / bc2) + (double)eps);
  }
}

// Changed-Gaussian delta for the six attribute groups, in this order:
//  0 opacity (1), 1 SH DC (3), 2 SH rest (3((D+1)^2-1)), 3 mean (3),
//  4 log-scale (3), 5 quaternion (4).
// Row i of a group is flagged when some element k has
//   fl32(|p_k - b_k|) > fl32(tau * |b_k|),  evaluated in FP32.
// Output words: [6 counts] then, per group in order, count indices (ascending)
// followed by count*width values (row-major).  Baseline rows of flagged
// Gaussians are overwritten with the current values.  Returns words written.
int64_t or_delta(const float* const* cur, float* const* base, const int32_t* widths, int64_t n,
                 uint32_t group_mask, float tau, uint32_t* out) {
  int64_t pos = 6;
  for (int g = 0; g < 6; ++g) {
    out[g] = 0;
    if (!((group_mask >> g) & 1u) || widths[g] == 0) continue;
    std::vector<int64_t> rows;
    for (int64_t i = 0; i < n; ++i) {
      bool flag = false;
      for (int k = 0; k < widths[g]; ++k) {
        const float p = cur[g][k * n + i], b = base[g][k * n + i];
        const float diff = std::fabs(p - b);
        const float thr = tau * std::fabs(b);
        if (diff > thr) { flag = true; break; }
      }
      if (flag) rows.push_back(i);
    }
    out[g] = (uint32_t)rows.size();
    for (int64_t i : rows) out[pos++] = (uint32_t)i;
    for (int64_t i : rows)
      for (int k = 0; k < widths[g]; ++k) {
        const float p = cur[g][k * n + i];
        std::memcpy(&out[pos++], &p, 4);
        base[g][k * n + i] = p;
      }
  }
  return pos;
}

// ---- delta codecs and client replay (Sec. 3.5) -----------------------------
// The paper codes means and scales as residuals against the previously
// transmitted state and the other attributes as quantized updates, without
// giving bit counts, ranges or rounding.  The reading implemented here, per
// group g with step s_g (inv_g = fl32(1 / s_g)), code width B_g (8 or 16):
//  mode 0 (raw):      the rule of or_delta; the value is sent as FP32 bits and
//                     becomes the baseline.
//  mode 1 (residual): c = clamp(rint(fl32(fl32(p - b) * inv)), -(2^(B-1)-1),
//                     2^(B-1)-1) (NaN -> 0); the row is sent when some c != 0;
//                     the baseline (and the receiver) become fl32(b + fl32(c s)),
//                     so sender and receiver stay bit-identical (closed loop).
//  mode 2 (quantized): q(x) = clamp(rint(fl32(fl32(x - lo) * inv)), 0, 2^B - 1)
//                     (NaN -> 0); the row is sent when some q(p) != q(b); the
//                     baseline and the receiver become fl32(lo + fl32(q(p) s)).
// rint rounds half to even.  A sent row carries all of its elements; codes
// of a row are packed little-endian, 32/B per word, a row starting on a word
// boundary.  Packet words: [0] epoch, [1] group mask, [2..7] row counts,
// [8] total words, then per masked group in order the ascending indices and
// the rows' words.
namespace {
const int kCodecHeader = 9;

int64_t codec_row_words(int mode, int bits, int width) {
  if (mode == 0) return width;
  const int per = 32 / bits;
  return (width + per - 1) / per;
}

long codec_code(int mode, int bits, float step, float lo, float p, float b, bool of_base) {
  const float inv = 1.0f / step;
  if (mode == 1) {
    const float r = p - b;
    const float x = r * inv;
    double q = std::nearbyint((double)x);
    if (std::isnan(x)) q = 0.0;
    const double m = (double)((1L << (bits - 1)) - 1);
    return (long)std::min(std::max(q, -m), m);
  }
  const float v = of_base ? b : p;
  const float d = v - lo;
  const float x = d * inv;
  double q = std::nearbyint((double)x);
  if (std::isnan(x)) q = 0.0;
  const double m = (double)((1L << bits) - 1);
  return (long)std::min(std::max(q, 0.0), m);
}
}  // namespace

// Encodes the masked groups of `cur` against `base` (updated in place) into
// out (capacity checked by the caller); returns the words written.
int64_t or_codec_encode(const float* const* cur, float* const* base, const int32_t* widths, int64_t n,
                        uint32_t group_mask, const int32_t* modes, const int32_t* bits, const float* steps,
                        const float* los, const float* taus, uint32_t epoch, uint32_t* out) {
  int64_t pos = kCodecHeader;
  out[0] = epoch;
  out[1] = group_mask;
  for (int g = 0; g < 6; ++g) {
    out[2 + g] = 0;
    if (!((group_mask >> g) & 1u) || widths[g] == 0) continue;
    const int W = widths[g], md = modes[g], B = md == 0 ? 32 : bits[g];
    std::vector<int64_t> rows;
    for (int64_t i = 0; i < n; ++i) {
      bool send = false;
      for (int k = 0; k < W && !send; ++k) {
        const float p = cur[g][k * n + i], b = base[g][k * n + i];
        if (md == 0) {
          const float diff = std::fabs(p - b);
          const float thr = taus[g] * std::fabs(b);
          send = diff > thr;
        } else if (md == 1) {
          send = codec_code(1, B, steps[g], los[g], p, b, false) != 0;
        } else {
          send = codec_code(2, B, steps[g], los[g], p, b, false) != codec_code(2, B, steps[g], los[g], p, b, true);
        }
      }
      if (send) rows.push_back(i);
    }
    out[2 + g] = (uint32_t)rows.size();
    for (int64_t i : rows) out[pos++] = (uint32_t)i;
    const int64_t wpr = codec_row_words(md, B, W);
    for (int64_t i : rows) {
      for (int64_t w = 0; w < wpr; ++w) out[pos + w] = 0u;
      for (int k = 0; k < W; ++k) {
        const float p = cur[g][k * n + i];
        float& b = base[g][k * n + i];
        if (md == 0) {
          std::memcpy(&out[pos + k], &p, 4);
          b = p;
          continue;
        }
        const long c = codec_code(md, B, steps[g], los[g], p, b, false);
        const float t = (float)c * steps[g];
        b = md == 1 ? b + t : los[g] + t;
        const int per = 32 / B;
        const uint32_t field = (uint32_t)((uint64_t)(int64_t)c & ((1ull << B) - 1));
        out[pos + k / per] |= field << ((k % per) * B);
      }
      pos += wpr;
    }
  }
  out[8] = (uint32_t)pos;
  return pos;
}

// Client replay: applies a packet to the receiver's model.  Returns the
// status bits: 1 epoch differs from `epoch`, 2 malformed (too short, mask bits
// above 5, rows in unmasked groups, counts above n, a total that disagrees
// with the header or exceeds packet_words, an index >= n, indices not
// strictly ascending).  The model is changed only when the status is 0.
uint32_t or_codec_apply(float* const* model, const int32_t* widths, int64_t n, const uint32_t* pk,
                        int64_t packet_words, const int32_t* modes, const int32_t* bits, const float* steps,
                        const float* los, uint32_t epoch) {
  if (packet_words < kCodecHeader) return 2u;
  uint32_t status = pk[0] != epoch ? 1u : 0u;
  const uint32_t mask = pk[1];
  if (mask & ~0x3Fu) return status | 2u;
  int64_t total = kCodecHeader;
  for (int g = 0; g < 6; ++g) {
    const int64_t c = pk[2 + g];
    if ((!((mask >> g) & 1u) && c != 0) || c > n) return status | 2u;
    const int md = modes[g], B = md == 0 ? 32 : bits[g];
    total += c * (1 + codec_row_words(md, B, widths[g]));
  }
  if (total != (int64_t)pk[8] || total > packet_words) return status | 2u;
  int64_t pos = kCodecHeader;
  for (int g = 0; g < 6; ++g) {
    const int64_t c = pk[2 + g];
    for (int64_t r = 0; r < c; ++r) {
      const int64_t i = pk[pos + r];
      if (i >= n || (r > 0 && (int64_t)pk[pos + r - 1] >= i)) return status | 2u;
    }
    pos += c * (1 + codec_row_words(modes[g], modes[g] == 0 ? 32 : bits[g], widths[g]));
  }
  if (status) return status;
  pos = kCodecHeader;
  for (int g = 0; g < 6; ++g) {
    const int64_t c = pk[2 + g];
    const int W = widths[g], md = modes[g], B = md == 0 ? 32 : bits[g];
    const int64_t wpr = codec_row_words(md, B, W);
    const uint32_t* vals = pk + pos + c;
    for (int64_t r = 0; r < c; ++r) {
      const int64_t i = pk[pos + r];
      for (int k = 0; k < W; ++k) {
        float& x = model[g][k * n + i];
        if (md == 0) {
          std::memcpy(&x, &vals[r * wpr + k], 4);
          continue;
        }
        const int per = 32 / B;
        const uint32_t field = (vals[r * wpr + k / per] >> ((k % per) * B)) & (uint32_t)((1ull << B) - 1);
        long code = (long)field;
        if (md == 1 && (field >> (B - 1)) & 1u) code -= 1L << B;   // two's complement
        const float t = (float)code * steps[g];
        x = md == 1 ? x + t : los[g] + t;
      }
    }
    pos += c * (1 + wpr);
  }
  return 0u;
}

}  // extern "C"
