// Preculling by grid cells (Sec. 3.3): Gaussians are assigned to the cells of
// a regular world grid, each view decides which cells it can see, and the
// projection skips the Gaussians of cells a view cannot see.
//
// The visibility test here is conservative by construction, so preculling
// never changes a result: a cell is dropped for a view only when no Gaussian
// whose mean lies in the cell can pass the projection's own visibility rule
// (depth at least the near plane and a pixel rectangle that meets the
// image).  The rectangle's half-width is 3 (1 + 2^-10) sqrt(A) with
// A = J M J^T + 0.3, and with M's eigenvalues at most sigma^2 (sigma = the
// largest scale of the cell's Gaussians) and the guard-band clamp on J,
//   z * hx <= 3 (1 + 2^-10) (fx kx sigma + sqrt(0.3) z),  kx = sqrt(1 + gx^2),
// gx = 1.3 (W/2)/fx.  "u + hx >= -1 and u - hx <= W + 1" then becomes, for
// camera-space (x, z) with z > 0, two inequalities linear in (x, z); each is
// checked at the eight corners of the cell box (a linear function takes its
// extremes at corners).  The same holds for y.  Callers that have a better
// visibility source (the engine's depth test in the paper) pass their own
// per-view cell mask instead.
#include "internal.h"

namespace gs {
namespace {

__device__ __forceinline__ uint32_t cell_of_point(const gs_grid& g, float x, float y, float z) {
  const float p[3] = {x, y, z};
  uint32_t idx = 0, stride = 1;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float t = (p[k] - g.origin[k]) / g.cell_size;
    if (!(t >= 0.f) || !(t < (float)g.dims[k])) return 0xffffffffu;   // outside (or NaN)
    idx += (uint32_t)t * stride;
    stride *= (uint32_t)g.dims[k];
  }
  return idx;
}

// cell_of[i] = cell index, or n_cells (the "outside" cell, never culled);
// cell_sigma[c] = largest exp(log-scale) over the cell's Gaussians (as float
// bits: positive floats order like their bit patterns).
__global__ __launch_bounds__(256) void k_assign_cells(ParamPtrs p, gs_grid g, uint32_t n_cells, uint32_t* cell_of,
                                                       uint32_t* cell_sigma) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const int64_t n = p.n;
  uint32_t c = cell_of_point(g, p.mean[i], p.mean[n + i], p.mean[2 * n + i]);
  if (c == 0xffffffffu) c = n_cells;
  cell_of[i] = c;
  const float s = fmaxf(fmaxf(p.lsc[i], p.lsc[n + i]), p.lsc[2 * n + i]);
  const float sig = expf(s);
  if (sig >= 0.f) atomicMax(&cell_sigma[c], __float_as_uint(sig));
  else atomicMax(&cell_sigma[c], 0x7f800000u);   // NaN scale: never cull its cell
}

// The same with the per-cell maxima first taken in LDS over a chunk of
// kCellChunk Gaussians (for grids of at most kLdsCells cells), so that each
// workgroup sends one global atomic per cell it touched.
constexpr int kLdsCells = 8192;
constexpr int kCellChunk = 8192;

__global__ __launch_bounds__(256) void k_assign_cells_lds(ParamPtrs p, gs_grid g, uint32_t n_cells,
                                                           uint32_t* cell_of, uint32_t* cell_sigma) {
  __shared__ uint32_t s_max[kLdsCells];
  for (uint32_t c = threadIdx.x; c <= n_cells; c += blockDim.x) s_max[c] = 0u;
  __syncthreads();
  const int64_t n = p.n;
  const int64_t i0 = (int64_t)blockIdx.x * kCellChunk;
  const int64_t i1 = i0 + kCellChunk < n ? i0 + kCellChunk : n;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    uint32_t c = cell_of_point(g, p.mean[i], p.mean[n + i], p.mean[2 * n + i]);
    if (c == 0xffffffffu) c = n_cells;
    cell_of[i] = c;
    const float sig = expf(fmaxf(fmaxf(p.lsc[i], p.lsc[n + i]), p.lsc[2 * n + i]));
    atomicMax(&s_max[c], sig >= 0.f ? __float_as_uint(sig) : 0x7f800000u);
  }
  __syncthreads();
  for (uint32_t c = threadIdx.x; c <= n_cells; c += blockDim.x)
    if (s_max[c] != 0u) atomicMax(&cell_sigma[c], s_max[c]);
}

__global__ void k_zero_words(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// mask[v][c] for the views of the call (row stride n_cells + 1; the last
// column, the outside cell, is always 1).
__global__ __launch_bounds__(256) void k_visible_cells(gs_grid g, const gs_camera* cams, int v0, int nv,
                                                        uint32_t n_cells, const uint32_t* cell_sigma, uint8_t* mask) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = (int64_t)n_cells + 1;
  if (t >= (int64_t)nv * row) return;
  const int v = v0 + (int)(t / row);
  const uint32_t c = (uint32_t)(t % row);
  uint8_t vis = 1;
  if (c < n_cells) {
    const gs_camera cam = cams[v];
    const uint32_t cx_ = c % (uint32_t)g.dims[0], rest = c / (uint32_t)g.dims[0];
    const uint32_t cy_ = rest % (uint32_t)g.dims[1], cz_ = rest / (uint32_t)g.dims[1];
    const double lo[3] = {(double)g.origin[0] + (double)g.cell_size * cx_,
                          (double)g.origin[1] + (double)g.cell_size * cy_,
                          (double)g.origin[2] + (double)g.cell_size * cz_};
    const double sigma = (double)__uint_as_float(cell_sigma[c]);
    const double fx = cam.fx, fy = cam.fy, W = cam.width, H = cam.height;
    const double gxr = (double)kGuard * 0.5 * W / fx, gyr = (double)kGuard * 0.5 * H / fy;
    const double slack = 3.0 * (1.0 + 0x1p-10) * 1.001;
    const double bx = slack * fx * sqrt(1.0 + gxr * gxr) * sigma, by = slack * fy * sqrt(1.0 + gyr * gyr) * sigma;
    const double ez = slack * sqrt((double)kDilation) + 1.0;   // per-unit-depth margin (px)
    // constraints a.(x, y, z) + b >= 0 that every visible Gaussian's mean meets
    double amin[5] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};
    for (int k = 0; k < 8; ++k) {
      const double w[3] = {lo[0] + ((k & 1) ? g.cell_size : 0.0), lo[1] + ((k & 2) ? g.cell_size : 0.0),
                           lo[2] + ((k & 4) ? g.cell_size : 0.0)};
      double x[3];
      for (int r = 0; r < 3; ++r)
        x[r] = (double)cam.R[r * 3] * w[0] + (double)cam.R[r * 3 + 1] * w[1] + (double)cam.R[r * 3 + 2] * w[2] +
               (double)cam.t[r];
      const double z = x[2];
      const double f[5] = {
          z - ((double)kNear - 1e-3),                                    // in front of the near plane
          fx * x[0] + ((double)cam.cx + ez) * z + bx,                    // u + hx >= -1
          -fx * x[0] + (W - (double)cam.cx + ez) * z + bx,               // u - hx <= W + 1
          fy * x[1] + ((double)cam.cy + ez) * z + by,
          -fy * x[1] + (H - (double)cam.cy + ez) * z + by};
      for (int q = 0; q < 5; ++q) amin[q] = fmin(amin[q], -f[q]);   // min of -f = -(max f)
    }
    // culled when one constraint fails at every corner (max f < 0, i.e. -max f > 0)
    for (int q = 0; q < 5; ++q)
      if (amin[q] > 0.0 && isfinite(sigma)) vis = 0;
  }
  mask[(int64_t)(t / row) * row + c] = vis;
}

}  // namespace

hipError_t launch_assign_cells(const ParamPtrs& p, const gs_grid& g, uint32_t* cell_of, uint32_t* cell_sigma,
                               hipStream_t st) {
  const int64_t nc = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((nc + 1 + 255) / 256)), dim3(256), 0, st, cell_sigma, nc + 1);
  if (p.n > 0 && nc + 1 <= kLdsCells)
    hipLaunchKernelGGL(k_assign_cells_lds, dim3((unsigned)((p.n + kCellChunk - 1) / kCellChunk)), dim3(256), 0, st,
                       p, g, (uint32_t)nc, cell_of, cell_sigma);
  else if (p.n > 0)
    hipLaunchKernelGGL(k_assign_cells, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, st, p, g, (uint32_t)nc,
                       cell_of, cell_sigma);
  return hipGetLastError();
}

hipError_t launch_visible_cells(const gs_grid& g, const gs_camera* cams, int v0, int nv, const uint32_t* cell_sigma,
                                uint8_t* mask, hipStream_t st) {
  const int64_t nc = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
  const int64_t total = (int64_t)nv * (nc + 1);
  if (total > 0)
    hipLaunchKernelGGL(k_visible_cells, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g, cams, v0, nv,
                       (uint32_t)nc, cell_sigma, mask);
  return hipGetLastError();
}

}  // namespace gs
