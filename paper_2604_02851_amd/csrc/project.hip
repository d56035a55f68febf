// Project/cull (forward) and the projection chain rule (backward).
//
// A workgroup takes 64 Gaussians (one per lane) and its kViewWaves
// wavefronts split the views of the call between them (view v goes to
// wavefront v mod kViewWaves), so the parameters are read from HBM once per
// call however many views it covers; the backward sums a Gaussian's views
// over the wavefronts through LDS.  One wavefront measured fastest: the
// FP64 per-Gaussian set-up is then not repeated.
//
// The screen-space gradients are nine field-major planes (field f of pair o
// at f * VN + o), all zero between steps: the workspace is cleared once
// (gs_workspace_init), the compositing adjoint adds into the fields of
// visible pairs only, and each part of the projection adjoint clears the
// fields it has read (the geometric part fields 0-5, the colour part 6-8),
// so every field is read once and written back once.  Geometry (camera-space mean,
// covariance, screen-space conic, projected mean, tile rectangle) is
// evaluated in FP64: the projected mean feeds every pixel test at up to
// 1920 px, where FP32 leaves ~1e-4 px of error; FP64 costs little here
// because this stage is a small part of the step.  Colour (SH) is FP32.
#include "internal.h"

namespace gs {
namespace {

// Real SH basis (orthonormal, (-1)^m sign), k = l*l + l + m, and its
// gradient with respect to the direction (as polynomials in x, y, z).
constexpr float Y00 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float Y1 = 0.48860251190291992f;    // sqrt(3)/(2 sqrt(pi))
constexpr float Y2a = 1.0925484305920792f;    // sqrt(15)/(2 sqrt(pi))
constexpr float Y2b = 0.31539156525252005f;   // sqrt(5)/(4 sqrt(pi))
constexpr float Y2c = 0.54627421529603959f;   // sqrt(15)/(4 sqrt(pi))
constexpr float Y3a = 0.59004358992664352f;   // sqrt(35/2)/(4 sqrt(pi))
constexpr float Y3b = 2.8906114426405538f;    // sqrt(105)/(2 sqrt(pi))
constexpr float Y3c = 0.45704579946446572f;   // sqrt(21/2)/(4 sqrt(pi))
constexpr float Y3d = 0.3731763325901154f;    // sqrt(7)/(4 sqrt(pi))
constexpr float Y3e = 1.4453057213202769f;    // sqrt(105)/(4 sqrt(pi))

__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y) {
  Y[0] = Y00;
  if (deg >= 1) { Y[1] = -Y1 * y; Y[2] = Y1 * z; Y[3] = -Y1 * x; }
  if (deg >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = Y2a * x * y;
    Y[5] = -Y2a * y * z;
    Y[6] = Y2b * (2.f * zz - xx - yy);
    Y[7] = -Y2a * x * z;
    Y[8] = Y2c * (xx - yy);
    if (deg >= 3) {
      Y[9] = -Y3a * y * (3.f * xx - yy);
      Y[10] = Y3b * x * y * z;
      Y[11] = -Y3c * y * (4.f * zz - xx - yy);
      Y[12] = Y3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
      Y[13] = -Y3c * x * (4.f * zz - xx - yy);
      Y[14] = Y3e * z * (xx - yy);
      Y[15] = -Y3a * x * (xx - 3.f * yy);
    }
  }
}

// g += sum_k w[k] * grad Y_k(x, y, z)
__device__ __forceinline__ void sh_grad_accum(int deg, float x, float y, float z, const float* w, float* g) {
  if (deg < 1) return;
  g[1] += -Y1 * w[1];
  g[2] += Y1 * w[2];
  g[0] += -Y1 * w[3];
  if (deg < 2) return;
  g[0] += Y2a * y * w[4];            g[1] += Y2a * x * w[4];
  g[1] += -Y2a * z * w[5];           g[2] += -Y2a * y * w[5];
  g[0] += -2.f * Y2b * x * w[6];     g[1] += -2.f * Y2b * y * w[6];  g[2] += 4.f * Y2b * z * w[6];
  g[0] += -Y2a * z * w[7];           g[2] += -Y2a * x * w[7];
  g[0] += 2.f * Y2c * x * w[8];      g[1] += -2.f * Y2c * y * w[8];
  if (deg < 3) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  g[0] += -6.f * Y3a * x * y * w[9];           g[1] += -3.f * Y3a * (xx - yy) * w[9];
  g[0] += Y3b * y * z * w[10];                 g[1] += Y3b * x * z * w[10];       g[2] += Y3b * x * y * w[10];
  g[0] += 2.f * Y3c * x * y * w[11];           g[1] += -Y3c * (4.f * zz - xx - 3.f * yy) * w[11];
  g[2] += -8.f * Y3c * y * z * w[11];
  g[0] += -6.f * Y3d * x * z * w[12];          g[1] += -6.f * Y3d * y * z * w[12];
  g[2] += Y3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
  g[0] += -Y3c * (4.f * zz - 3.f * xx - yy) * w[13];  g[1] += 2.f * Y3c * x * y * w[13];
  g[2] += -8.f * Y3c * x * z * w[13];
  g[0] += 2.f * Y3e * x * z * w[14];           g[1] += -2.f * Y3e * y * z * w[14]; g[2] += Y3e * (xx - yy) * w[14];
  g[0] += -3.f * Y3a * (xx - yy) * w[15];      g[1] += 6.f * Y3a * x * y * w[15];
}

// FP32 camera depth evaluated in a fixed order with every operation rounded
// on its own (no fused multiply-add), so that it equals the same expression
// evaluated anywhere else in IEEE single precision.
__device__ __forceinline__ float depth_key(float r20, float r21, float r22, float t2, float mx, float my, float mz) {
#pragma clang fp contract(off)
  float a = r20 * mx;
  float b = r21 * my;
  float s = a + b;
  float d = r22 * mz;
  s = s + d;
  return s + t2;
}

struct Gauss {
  float mu[3];
  double Sig[6];   // world covariance (00, 01, 02, 11, 12, 22)
  double Rq[9];    // rotation of the normalised quaternion
  double rho[4], qn;
  double e2[3];    // exp(2 s)
  float o;
  bool ok;
};

// sh_finite: whether the Gaussian's SH coefficients are all finite (the
// caller checks them where it loads them, or passes true where only pairs
// already found visible are visited).
__device__ __forceinline__ void load_gauss(const ParamPtrs& p, int64_t i, Gauss& g, bool sh_finite) {
  const int64_t n = p.n;
  bool fin = true;
  for (int k = 0; k < 3; ++k) {
    g.mu[k] = __builtin_nontemporal_load(p.mean + k * n + i);
    fin &= isfinite(g.mu[k]);
  }
  float ls[3], q[4];
  for (int k = 0; k < 3; ++k) { ls[k] = __builtin_nontemporal_load(p.lsc + k * n + i); fin &= isfinite(ls[k]); }
  for (int k = 0; k < 4; ++k) { q[k] = __builtin_nontemporal_load(p.quat + k * n + i); fin &= isfinite(q[k]); }
  const float w = __builtin_nontemporal_load(p.opac + i);
  fin &= isfinite(w) && sh_finite;
  const double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
  g.qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  g.ok = fin && g.qn > 0.0;
  if (!g.ok) return;
  const double iqn = 1.0 / g.qn;
  const double a = qw * iqn, b = qx * iqn, c = qy * iqn, d = qz * iqn;
  g.rho[0] = a; g.rho[1] = b; g.rho[2] = c; g.rho[3] = d;
  double* R = g.Rq;
  R[0] = 1 - 2 * (c * c + d * d); R[1] = 2 * (b * c - a * d);     R[2] = 2 * (b * d + a * c);
  R[3] = 2 * (b * c + a * d);     R[4] = 1 - 2 * (b * b + d * d); R[5] = 2 * (c * d - a * b);
  R[6] = 2 * (b * d - a * c);     R[7] = 2 * (c * d + a * b);     R[8] = 1 - 2 * (b * b + c * c);
  for (int k = 0; k < 3; ++k) g.e2[k] = exp(2.0 * (double)ls[k]);
  // Sigma = Rq diag(e2) Rq^T
  const int idx[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  for (int t = 0; t < 6; ++t) {
    const int r = idx[t][0], c2 = idx[t][1];
    g.Sig[t] = R[r * 3 + 0] * g.e2[0] * R[c2 * 3 + 0] + R[r * 3 + 1] * g.e2[1] * R[c2 * 3 + 1] +
               R[r * 3 + 2] * g.e2[2] * R[c2 * 3 + 2];
  }
  g.o = 1.f / (1.f + expf(-w));
}

// Per-view geometry of one Gaussian.
struct ViewGeom {
  double x[3];
  double M[6];            // W Sigma W^T (00, 01, 02, 11, 12, 22)
  double j00, j02, j11, j12;
  bool clx, cly;
  double A, B, C, det;
  double u, w;
};

__device__ __forceinline__ bool view_geom(const Gauss& g, const ViewD& cam, ViewGeom& vg) {
  const double* W = cam.W;
  for (int r = 0; r < 3; ++r)
    vg.x[r] = W[r * 3] * (double)g.mu[0] + W[r * 3 + 1] * (double)g.mu[1] + W[r * 3 + 2] * (double)g.mu[2] +
              cam.t[r];
  // T = W Sigma
  const double S[9] = {g.Sig[0], g.Sig[1], g.Sig[2], g.Sig[1], g.Sig[3], g.Sig[4], g.Sig[2], g.Sig[4], g.Sig[5]};
  double T[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) T[r * 3 + c] = W[r * 3] * S[c] + W[r * 3 + 1] * S[3 + c] + W[r * 3 + 2] * S[6 + c];
  const int idx[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  for (int t = 0; t < 6; ++t) {
    const int r = idx[t][0], c = idx[t][1];
    vg.M[t] = T[r * 3] * W[c * 3] + T[r * 3 + 1] * W[c * 3 + 1] + T[r * 3 + 2] * W[c * 3 + 2];
  }
  const double fx = cam.fx, fy = cam.fy, z = vg.x[2];
  const double limx = cam.limx, limy = cam.limy;
  const double iz = 1.0 / z;   // one FP64 division per view; the rest multiply by it
  double tx = vg.x[0] * iz, ty = vg.x[1] * iz;
  vg.clx = tx < -limx || tx > limx;
  vg.cly = ty < -limy || ty > limy;
  tx = fmin(limx, fmax(-limx, tx));
  ty = fmin(limy, fmax(-limy, ty));
  vg.j00 = fx * iz;
  vg.j02 = -fx * tx * iz;
  vg.j11 = fy * iz;
  vg.j12 = -fy * ty * iz;
  const double M00 = vg.M[0], M01 = vg.M[1], M02 = vg.M[2], M11 = vg.M[3], M12 = vg.M[4], M22 = vg.M[5];
  const double s00 = vg.j00 * vg.j00 * M00 + 2.0 * vg.j00 * vg.j02 * M02 + vg.j02 * vg.j02 * M22;
  const double s01 = vg.j00 * vg.j11 * M01 + vg.j00 * vg.j12 * M02 + vg.j02 * vg.j11 * M12 + vg.j02 * vg.j12 * M22;
  const double s11 = vg.j11 * vg.j11 * M11 + 2.0 * vg.j11 * vg.j12 * M12 + vg.j12 * vg.j12 * M22;
  vg.A = s00 + (double)kDilation;
  vg.B = s01;
  vg.C = s11 + (double)kDilation;
  vg.det = vg.A * vg.C - vg.B * vg.B;
  vg.u = fx * vg.x[0] * iz + cam.cx;
  vg.w = fy * vg.x[1] * iz + cam.cy;
  return vg.det > 0.0 && isfinite(vg.det) && isfinite(vg.u) && isfinite(vg.w);
}

__device__ __forceinline__ void view_dir(const gs_camera& cam, const float* mu, float* d, float* len) {
  const float vx = mu[0] - cam.campos[0], vy = mu[1] - cam.campos[1], vz = mu[2] - cam.campos[2];
  const float l = sqrtf(vx * vx + vy * vy + vz * vz);
  *len = l;
  const float il = 1.f / l;
  d[0] = vx * il; d[1] = vy * il; d[2] = vz * il;
}

// The cameras are not written while a projection kernel runs: read through
// the constant address space, a wavefront-uniform view index makes them
// scalar loads (the scalar cache, no vector registers, no wait at the top of
// every view).
typedef const uint32_t __attribute__((address_space(4))) ConstWord;
static_assert(sizeof(gs_camera) == 21 * sizeof(uint32_t), "camera words");
__device__ __forceinline__ gs_camera read_camera(const gs_camera* cams, int v) {
  ConstWord* src = (ConstWord*)(cams + v);
  gs_camera c;
  uint32_t* dst = reinterpret_cast<uint32_t*>(&c);
#pragma unroll
  for (int k = 0; k < 21; ++k) dst[k] = src[k];
  return c;
}

typedef const double __attribute__((address_space(4))) ConstDouble;
static_assert(sizeof(ViewD) == 18 * sizeof(double), "view constant words");
__device__ __forceinline__ ViewD read_view_d(const ViewD* vds, int v) {
  ConstDouble* src = (ConstDouble*)(vds + v);
  ViewD d;
  double* dst = reinterpret_cast<double*>(&d);
#pragma unroll
  for (int k = 0; k < 18; ++k) dst[k] = src[k];
  return d;
}

// One thread per view of the launch: the camera in double precision and the
// guard-band limits kGuard (width / 2) / fx, kGuard (height / 2) / fy.
__global__ void k_view_consts(const gs_camera* cams, int v0, int nv, ViewD* out) {
  const int v = v0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (v >= v0 + nv) return;
  const gs_camera cam = cams[v];
  ViewD d;
  for (int k = 0; k < 9; ++k) d.W[k] = cam.R[k];
  for (int k = 0; k < 3; ++k) d.t[k] = cam.t[k];
  d.fx = cam.fx;
  d.fy = cam.fy;
  d.cx = cam.cx;
  d.cy = cam.cy;
  d.limx = (double)kGuard * (0.5 * (double)cam.width) / d.fx;
  d.limy = (double)kGuard * (0.5 * (double)cam.height) / d.fy;
  out[v] = d;
}

struct ProjArgs {
  ParamPtrs p;
  const gs_camera* cams;
  const ViewD* vd;           // per-view constants of the same cameras
  const ViewInfo* views;
  int v0, nv;
  int tile_sw, tile_sh;      // log2 of the tile width and height
  uint32_t* depth;
  uint32_t* count;
  ushort4* rect;
  float4* rec;
  uint64_t* vmask;           // per Gaussian: the views of this call that see it
  const uint32_t* cell_of;   // preculling (null = off)
  const uint8_t* cell_mask;
  int32_t cell_row;
};

constexpr int kViewWaves = 1;   // (the per-Gaussian view mask assumes a single wavefront per Gaussian)
static_assert(kViewWaves == 1, "one wavefront writes a Gaussian's view mask");

template <int DEG>
__global__ __launch_bounds__(64 * kViewWaves) void k_project(ProjArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  // uniform, so that the per-view camera is read with scalar loads
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t n = a.p.n;
  if (i >= n || wave >= a.nv) return;
  constexpr int nk = (DEG + 1) * (DEG + 1);
  const uint32_t cell = a.cell_mask ? a.cell_of[i] : 0u;
  if (a.cell_mask) {
    // a Gaussian whose cell no view of the call can see is culled everywhere
    // without touching its parameters
    bool any = false;
    for (int v = a.v0 + wave; v < a.v0 + a.nv; v += kViewWaves) any |= a.cell_mask[(int64_t)v * a.cell_row + cell] != 0;
    if (!any) {
      for (int v = a.v0 + wave; v < a.v0 + a.nv; v += kViewWaves) a.count[(int64_t)v * n + i] = 0u;
      a.vmask[i] = 0ull;
      return;
    }
  }
  // SH coefficients parked in this wavefront's own LDS columns (each lane
  // reads back only what it wrote, so no barrier is needed)
  __shared__ float s_sh[kViewWaves][3 * nk][64];
  const int lane = threadIdx.x & 63;
  bool sh_ok = true;
#pragma unroll
  for (int k = 0; k < 3 * nk; ++k) {
    const float c = __builtin_nontemporal_load(a.p.sh + (int64_t)k * n + i);
    sh_ok &= isfinite(c);
    s_sh[wave][k][lane] = c;
  }
  Gauss g;
  load_gauss(a.p, i, g, sh_ok);
  uint64_t vm = 0ull;
#pragma unroll 1
  for (int v = a.v0 + wave; v < a.v0 + a.nv; v += kViewWaves) {
    const int64_t o = (int64_t)v * n + i;
    const gs_camera cam = read_camera(a.cams, v);
    uint32_t cnt = 0;
    if (g.ok && (!a.cell_mask || a.cell_mask[(int64_t)v * a.cell_row + cell])) {
      const float z32 = depth_key(cam.R[6], cam.R[7], cam.R[8], cam.t[2], g.mu[0], g.mu[1], g.mu[2]);
      ViewGeom vg;
      if (z32 >= kNear && view_geom(g, read_view_d(a.vd, v), vg)) {
        const double slack = 1.0 + 0x1p-10;
        const double hx = 3.0 * sqrt(vg.A) * slack, hy = 3.0 * sqrt(vg.C) * slack;
        double lx = ceil(vg.u - hx - 0.5), ux = floor(vg.u + hx - 0.5);
        double ly = ceil(vg.w - hy - 0.5), uy = floor(vg.w + hy - 0.5);
        lx = fmax(lx, 0.0); ly = fmax(ly, 0.0);
        ux = fmin(ux, (double)(cam.width - 1)); uy = fmin(uy, (double)(cam.height - 1));
        if (lx <= ux && ly <= uy) {
          // the bounds are clamped to >= 0, so the shifts are floor divisions
          const int tx0 = (int)lx >> a.tile_sw, tx1 = (int)ux >> a.tile_sw;
          const int ty0 = (int)ly >> a.tile_sh, ty1 = (int)uy >> a.tile_sh;
          cnt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
          a.rect[o] = make_ushort4((unsigned short)tx0, (unsigned short)ty0, (unsigned short)tx1, (unsigned short)ty1);
          a.depth[o] = __float_as_uint(z32);
          // splat record
          const float uh = (float)vg.u, wh = (float)vg.w;
          const float ul = (float)(vg.u - (double)uh), wl = (float)(vg.w - (double)wh);
          const double iC = 1.0 / vg.C;
          const float qa = (float)(vg.C / vg.det);
          const float qr = (float)(-vg.B * iC);
          const float qs = (float)iC;
          float d[3], len;
          view_dir(cam, g.mu, d, &len);
          float Y[16];
          sh_basis(DEG, d[0], d[1], d[2], Y);
          float col[3];
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            float s = 0.5f;
#pragma unroll
            for (int k = 0; k < nk; ++k) s = fmaf(s_sh[wave][k * 3 + ch][lane], Y[k], s);
            col[ch] = fmaxf(s, 0.f);
          }
          a.rec[o * 3 + 0] = make_float4(uh, wh, ul, wl);
          a.rec[o * 3 + 1] = make_float4(qa, qr, qs, g.o);
          a.rec[o * 3 + 2] = make_float4(col[0], col[1], col[2], 0.f);
        }
      }
    }
    a.count[o] = cnt;
    if (cnt != 0u) vm |= a.nv <= 64 ? 1ull << (v - a.v0) : ~0ull;
  }
  a.vmask[i] = vm;
}

// OR of a 64-bit value over the wavefront's lanes (every lane receives it).
__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo |= (uint32_t)__shfl_xor((int)lo, off, 64);
    hi |= (uint32_t)__shfl_xor((int)hi, off, 64);
  }
  return ((uint64_t)hi << 32) | lo;
}

// Runs body(v, o) for the views v of the call that see this lane's Gaussian
// (vm from the projection).  With at most 64 views the wavefront walks the
// union of its lanes' masks (uniform) and a lane takes the views of its own
// mask, with no per-view memory traffic; with more views every view's count
// is read as the mask cannot hold them.
template <class F>
__device__ __forceinline__ void for_seen_views(int v0, int nv, int64_t n, int64_t i, uint64_t vm, const uint32_t* count,
                                               F&& body) {
  if (nv <= 64) {
    const uint64_t any = wave_or_u64(vm);
    const uint64_t wm = (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)any) |
                        ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(any >> 32)) << 32);
#pragma unroll 1
    for (uint64_t m = wm; m != 0ull; m &= m - 1ull) {
      const int vi = __builtin_ctzll(m);
      if (!((vm >> vi) & 1ull)) continue;
      const int v = v0 + vi;
      body(v, (int64_t)v * n + i);
    }
  } else {
#pragma unroll 1
    for (int v = v0; v < v0 + nv; ++v) {
      const int64_t o = (int64_t)v * n + i;
      if (vm == 0ull || count[o] == 0u) continue;
      body(v, o);
    }
  }
}

struct ProjBwdArgs {
  ParamPtrs p;
  const gs_camera* cams;
  const ViewD* vd;    // per-view constants of the same cameras
  int v0, nv;
  const uint32_t* count;
  const uint64_t* vmask;
  float* g2;          // field f of pair o at g2[f * g2_plane + o]
  size_t g2_plane;
  float* gmean; float* glsc; float* gquat; float* gopac; float* gsh;
  int64_t n_active;   // gradients for Gaussians i < n_active, rows strided by n_active
  int accumulate;
};

// Geometric part of the projection adjoint (mean, log-scale, quaternion,
// opacity); the SH coefficients and the view-direction term of the mean
// gradient come from k_color_bwd, which runs after it.
template <int DEG>
__global__ __launch_bounds__(64 * kViewWaves) void k_project_bwd(ProjBwdArgs a) {
  constexpr int kOut = 11;   // mean 3, log-scale 3, quaternion 4, opacity 1
  __shared__ float s_part[kViewWaves > 1 ? kViewWaves - 1 : 1][kOut][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const int64_t n = a.p.n, na = a.n_active;
  Gauss g;
  g.ok = false;
  // Gaussians visible in no view of the last projection need no set-up
  const uint64_t vm = (i < na && wave < a.nv) ? a.vmask[i] : 0ull;
  if (vm != 0ull) load_gauss(a.p, i, g, true);
  const double iqn = g.ok ? 1.0 / g.qn : 0.0;
  double gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0;
  for_seen_views(a.v0, a.nv, n, i, g.ok ? vm : 0ull, a.count, [&](int v, int64_t o) {
    float* gp = a.g2 + o;
    const size_t P = a.g2_plane;
    const double gu = gp[0], gw = gp[P], ga = gp[2 * P], gb = gp[3 * P], gc = gp[4 * P], gop = gp[5 * P];
#pragma unroll
    for (int f = 0; f < 6; ++f) gp[f * P] = 0.f;
    const ViewD cam = read_view_d(a.vd, v);
    ViewGeom vg;
    view_geom(g, cam, vg);
    // opacity
    go += gop * (double)g.o * (1.0 - (double)g.o);
    // conic -> screen covariance: dL/dSigma2 = -Q G_Q Q
    const double idet = 1.0 / vg.det;
    const double qa = vg.C * idet, qb = -vg.B * idet, qc = vg.A * idet;
    const double S00 = -(qa * qa * ga + qa * qb * gb + qb * qb * gc);
    const double S01 = -(qa * qb * ga + 0.5 * (qb * qb + qa * qc) * gb + qb * qc * gc);
    const double S11 = -(qb * qb * ga + qb * qc * gb + qc * qc * gc);
    // Sigma2 = J M J^T + eps I
    const double j00 = vg.j00, j02 = vg.j02, j11 = vg.j11, j12 = vg.j12;
    double GM[6];
    GM[0] = j00 * j00 * S00;
    GM[1] = j00 * j11 * S01;
    GM[2] = j00 * (S00 * j02 + S01 * j12);
    GM[3] = j11 * j11 * S11;
    GM[4] = j11 * (S01 * j02 + S11 * j12);
    GM[5] = j02 * j02 * S00 + 2.0 * j02 * j12 * S01 + j12 * j12 * S11;
    const double M00 = vg.M[0], M01 = vg.M[1], M02 = vg.M[2], M11 = vg.M[3], M12 = vg.M[4], M22 = vg.M[5];
    const double JM0[3] = {j00 * M00 + j02 * M02, j00 * M01 + j02 * M12, j00 * M02 + j02 * M22};
    const double JM1[3] = {j11 * M01 + j12 * M02, j11 * M11 + j12 * M12, j11 * M12 + j12 * M22};
    const double GJ00 = 2.0 * (S00 * JM0[0] + S01 * JM1[0]);
    const double GJ02 = 2.0 * (S00 * JM0[2] + S01 * JM1[2]);
    const double GJ11 = 2.0 * (S01 * JM0[1] + S11 * JM1[1]);
    const double GJ12 = 2.0 * (S01 * JM0[2] + S11 * JM1[2]);
    const double fx = cam.fx, fy = cam.fy, z = vg.x[2];
    double gx[3];
    const double iz = 1.0 / z, iz2 = iz * iz, iz3 = iz2 * iz;
    gx[0] = gu * fx * iz;
    gx[1] = gw * fy * iz;
    gx[2] = -(gu * fx * vg.x[0] + gw * fy * vg.x[1] + GJ00 * fx + GJ11 * fy) * iz2;
    if (!vg.clx) { gx[0] += -GJ02 * fx * iz2; gx[2] += GJ02 * 2.0 * fx * vg.x[0] * iz3; }
    else { gx[2] += -GJ02 * j02 * iz; }          // j02 = -fx c / z, c fixed
    if (!vg.cly) { gx[1] += -GJ12 * fy * iz2; gx[2] += GJ12 * 2.0 * fy * vg.x[1] * iz3; }
    else { gx[2] += -GJ12 * j12 * iz; }
    // x = W mu + t ;  M = W Sigma W^T
    double W[9];
    for (int k = 0; k < 9; ++k) W[k] = cam.W[k];
    for (int c = 0; c < 3; ++c) gm[c] += W[c] * gx[0] + W[3 + c] * gx[1] + W[6 + c] * gx[2];
    const double G[9] = {GM[0], GM[1], GM[2], GM[1], GM[3], GM[4], GM[2], GM[4], GM[5]};
    double T[9], G3[9];   // G3 = W^T G W
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) T[r * 3 + c] = W[r] * G[c] + W[3 + r] * G[3 + c] + W[6 + r] * G[6 + c];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) G3[r * 3 + c] = T[r * 3] * W[c] + T[r * 3 + 1] * W[3 + c] + T[r * 3 + 2] * W[6 + c];
    // Sigma = Rq diag(e2) Rq^T
    const double* R = g.Rq;
    double GR[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        GR[r * 3 + c] = 2.0 * (G3[r * 3] * R[c] + G3[r * 3 + 1] * R[3 + c] + G3[r * 3 + 2] * R[6 + c]) * g.e2[c];
    for (int k = 0; k < 3; ++k) {
      // (Rq^T G3 Rq)_kk = sum_rc R[r][k] G3[r][c] R[c][k]
      double s = 0;
      for (int r = 0; r < 3; ++r)
        s += R[r * 3 + k] * (G3[r * 3] * R[k] + G3[r * 3 + 1] * R[3 + k] + G3[r * 3 + 2] * R[6 + k]);
      gs[k] += 2.0 * g.e2[k] * s;
    }
    const double w_ = g.rho[0], x_ = g.rho[1], y_ = g.rho[2], z_ = g.rho[3];
    double gr[4];
    gr[0] = 2 * (-z_ * GR[1] + y_ * GR[2] + z_ * GR[3] - x_ * GR[5] - y_ * GR[6] + x_ * GR[7]);
    gr[1] = 2 * (y_ * GR[1] + z_ * GR[2] + y_ * GR[3] - 2 * x_ * GR[4] - w_ * GR[5] + z_ * GR[6] + w_ * GR[7] -
                 2 * x_ * GR[8]);
    gr[2] = 2 * (-2 * y_ * GR[0] + x_ * GR[1] + w_ * GR[2] + x_ * GR[3] + z_ * GR[5] - w_ * GR[6] + z_ * GR[7] -
                 2 * y_ * GR[8]);
    gr[3] = 2 * (-2 * z_ * GR[0] - w_ * GR[1] + x_ * GR[2] + w_ * GR[3] - 2 * z_ * GR[4] + y_ * GR[5] +
                 x_ * GR[6] + y_ * GR[7]);
    const double dot = w_ * gr[0] + x_ * gr[1] + y_ * gr[2] + z_ * gr[3];
    for (int k = 0; k < 4; ++k) gq[k] += (gr[k] - g.rho[k] * dot) * iqn;
  });
  // sum over the wavefronts: waves 1.. park their partial sums in LDS
  float part[kOut];
#pragma unroll
  for (int k = 0; k < 3; ++k) part[k] = (float)gm[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) part[3 + k] = (float)gs[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) part[6 + k] = (float)gq[k];
  part[10] = (float)go;
  if (wave > 0) {
#pragma unroll
    for (int k = 0; k < kOut; ++k) s_part[wave - 1][k][lane] = part[k];
  }
  __syncthreads();
  if (wave > 0 || i >= na) return;
#pragma unroll
  for (int w = 0; w < kViewWaves - 1; ++w)
#pragma unroll
    for (int k = 0; k < kOut; ++k) part[k] += s_part[w][k][lane];
  auto put = [&](float* dst, float val) {
    if (a.accumulate) *dst += val; else *dst = val;
  };
  for (int k = 0; k < 3; ++k) put(&a.gmean[k * na + i], part[k]);
  for (int k = 0; k < 3; ++k) put(&a.glsc[k * na + i], part[3 + k]);
  for (int k = 0; k < 4; ++k) put(&a.gquat[k * na + i], part[6 + k]);
  put(&a.gopac[i], part[10]);
}

// Colour part of the projection adjoint: SH coefficients, and the term of
// the mean gradient that comes through the view direction (added to the mean
// gradient written by k_project_bwd).
template <int DEG>
__global__ __launch_bounds__(64 * kViewWaves) void k_color_bwd(ProjBwdArgs a) {
  constexpr int nk = (DEG + 1) * (DEG + 1);
  constexpr int kOut = 3 + 3 * nk;   // mean (direction term) 3, SH
  __shared__ float s_part[kViewWaves > 1 ? kViewWaves - 1 : 1][kOut][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const int64_t n = a.p.n, na = a.n_active;
  float part[kOut];
#pragma unroll
  for (int k = 0; k < kOut; ++k) part[k] = 0.f;
  __shared__ float s_sh[kViewWaves][3 * nk][64];   // per-lane columns: no barrier needed
  const uint64_t vm = (i < na && wave < a.nv) ? a.vmask[i] : 0ull;
  {
    float* sh_col = &s_sh[wave][0][lane];
    float mu[3] = {0.f, 0.f, 0.f};
    if (vm != 0ull) {
#pragma unroll
      for (int k = 0; k < 3 * nk; ++k) sh_col[k * 64] = a.p.sh[(int64_t)k * n + i];
      mu[0] = a.p.mean[i], mu[1] = a.p.mean[n + i], mu[2] = a.p.mean[2 * n + i];
    }
#define SH(k) sh_col[(k) * 64]
    for_seen_views(a.v0, a.nv, n, i, vm, a.count, [&](int v, int64_t o) {
      float* gp = a.g2 + o;
      const size_t P = a.g2_plane;
      const float gcol[3] = {gp[6 * P], gp[7 * P], gp[8 * P]};
      gp[6 * P] = gp[7 * P] = gp[8 * P] = 0.f;
      float d[3], len;
      const gs_camera cam = read_camera(a.cams, v);
      view_dir(cam, mu, d, &len);
      float Y[16];
      sh_basis(DEG, d[0], d[1], d[2], Y);
      float wk[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) wk[k] = 0.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float s = 0.5f;
#pragma unroll
        for (int k = 0; k < nk; ++k) s = fmaf(SH(k * 3 + ch), Y[k], s);
        const float gcc = s > 0.f ? gcol[ch] : 0.f;
#pragma unroll
        for (int k = 0; k < nk; ++k) {
          part[3 + k * 3 + ch] += Y[k] * gcc;
          wk[k] += gcc * SH(k * 3 + ch);
        }
      }
      float gd[3] = {0.f, 0.f, 0.f};
      sh_grad_accum(DEG, d[0], d[1], d[2], wk, gd);
      const float dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
      for (int k = 0; k < 3; ++k) part[k] += (gd[k] - d[k] * dd) / len;
    });
#undef SH
  }
  if (wave > 0) {
#pragma unroll
    for (int k = 0; k < kOut; ++k) s_part[wave - 1][k][lane] = part[k];
  }
  __syncthreads();
  if (wave > 0 || i >= na) return;
#pragma unroll
  for (int w = 0; w < kViewWaves - 1; ++w)
#pragma unroll
    for (int k = 0; k < kOut; ++k) part[k] += s_part[w][k][lane];
  for (int k = 0; k < 3; ++k) a.gmean[k * na + i] += part[k];
#pragma unroll
  for (int k = 0; k < nk * 3; ++k) {
    float* dst = &a.gsh[(int64_t)k * na + i];
    *dst = a.accumulate ? *dst + part[3 + k] : part[3 + k];
  }
}

}  // namespace

hipError_t launch_project(const Plan& pl, const ParamPtrs& p, const gs_camera* cams, int v0, int nv, void* ws,
                          hipStream_t st) {
  ProjArgs a;
  a.p = p;
  a.cams = cams;
  a.vd = seg<ViewD>(ws, pl.ws.vconst);
  a.views = pl.d_views;
  a.v0 = v0;
  a.nv = nv;
  a.tile_sw = __builtin_ctz((unsigned)pl.tile_w);
  a.tile_sh = __builtin_ctz((unsigned)pl.tile_h);
  a.depth = seg<uint32_t>(ws, pl.ws.depth);
  a.count = seg<uint32_t>(ws, pl.ws.count);
  a.rect = seg<ushort4>(ws, pl.ws.rect);
  a.rec = seg<float4>(ws, pl.ws.rec);
  a.vmask = seg<uint64_t>(ws, pl.ws.vmask);
  a.cell_of = pl.cell_of;
  a.cell_mask = pl.cell_mask;
  a.cell_row = pl.cell_row;
  const int blocks = (p.n + 63) / 64;
  if (blocks == 0) return hipSuccess;
  if (nv < 1 || v0 < 0 || v0 + nv > kMaxViews) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_view_consts, dim3(1), dim3(kMaxViews), 0, st, cams, v0, nv, seg<ViewD>(ws, pl.ws.vconst));
  const dim3 block(64 * kViewWaves);
  switch (p.deg) {
    case 0: hipLaunchKernelGGL(k_project<0>, dim3(blocks), block, 0, st, a); break;
    case 1: hipLaunchKernelGGL(k_project<1>, dim3(blocks), block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_project<2>, dim3(blocks), block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(k_project<3>, dim3(blocks), block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_project_bwd(const Plan& pl, const ParamPtrs& p, const gs_camera* cams, int v0, int nv, void* ws,
                              const gs_params& grads, int accumulate, hipStream_t st) {
  ProjBwdArgs a;
  a.p = p;
  a.cams = cams;
  a.vd = seg<ViewD>(ws, pl.ws.vconst);
  a.v0 = v0;
  a.nv = nv;
  a.count = seg<uint32_t>(ws, pl.ws.count);
  a.vmask = seg<uint64_t>(ws, pl.ws.vmask);
  a.g2 = seg<float>(ws, pl.ws.g2);
  a.g2_plane = (size_t)pl.ws.vn;
  a.gmean = grads.mean;
  a.glsc = grads.log_scale;
  a.gquat = grads.quat;
  a.gopac = grads.opacity_logit;
  a.gsh = grads.sh;
  a.n_active = grads.n;
  a.accumulate = accumulate;
  const int blocks = (grads.n + 63) / 64;
  if (blocks == 0) return hipSuccess;
  if (nv < 1 || v0 < 0 || v0 + nv > kMaxViews) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_view_consts, dim3(1), dim3(kMaxViews), 0, st, cams, v0, nv, seg<ViewD>(ws, pl.ws.vconst));
  const dim3 block(64 * kViewWaves);
  switch (p.deg) {
    case 0: hipLaunchKernelGGL(k_project_bwd<0>, dim3(blocks), block, 0, st, a); break;
    case 1: hipLaunchKernelGGL(k_project_bwd<1>, dim3(blocks), block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_project_bwd<2>, dim3(blocks), block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(k_project_bwd<3>, dim3(blocks), block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  switch (p.deg) {
    case 0: hipLaunchKernelGGL(k_color_bwd<0>, dim3(blocks), block, 0, st, a); break;
    case 1: hipLaunchKernelGGL(k_color_bwd<1>, dim3(blocks), block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_color_bwd<2>, dim3(blocks), block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(k_color_bwd<3>, dim3(blocks), block, 0, st, a); break;
  }
  return hipGetLastError();
}

}  // namespace gs
