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
constexpr int kCellChunk = 2048;

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

// ---- spatial order: the model kept grouped by cell ---------------------------
// With Gaussians stored in index order independent of position, every
// wavefront of the projection holds Gaussians from all over the scene, so
// per-view culling (by the frustum or by cells) almost never removes a whole
// wavefront.  Stored grouped by cell, a wavefront's Gaussians share a cell,
// and a culled cell costs the projection and its adjoints almost nothing.

// sort key: pool (active 0, frozen 1) above the cell index (out-of-range
// values count as the outside cell n_cells); the value is the position
__global__ void k_cell_keys(const uint32_t* cell_of, int64_t n, int64_t n_active, uint32_t n_cells, int cell_bits,
                            uint32_t* key, uint32_t* val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = cell_of[i] < n_cells ? cell_of[i] : n_cells;
  key[i] = ((i >= n_active ? 1u : 0u) << cell_bits) | c;
  val[i] = (uint32_t)i;
}

__global__ void k_copy_row(const uint32_t* src, uint32_t* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// row[k] = old[from[k]], k < n (old parked in scratch)
__global__ void k_gather_row(const uint32_t* scratch, const uint32_t* from, int64_t n, uint32_t* row) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) row[k] = scratch[from[k]];
}

}  // namespace

hipError_t launch_sort_cells(const Plan& pl, const gs_params& p, const gs_params* m, const gs_params* v,
                             uint32_t* cell_of, int32_t n_cells, int64_t n_active, uint32_t* ids, const gs_params* base,
                             void* ws, hipStream_t st) {
  const int64_t n = p.n;
  if (n == 0) return hipSuccess;
  int cell_bits = 1;
  while (((int64_t)1 << cell_bits) <= (int64_t)n_cells) ++cell_bits;
  const int bits = (cell_bits + 1 + 7) / 8 * 8;
  uint32_t* ka = seg<uint32_t>(ws, pl.ws.vkey_a);
  uint32_t* kb = seg<uint32_t>(ws, pl.ws.vkey_b);
  uint32_t* va = seg<uint32_t>(ws, pl.ws.vis_a);
  uint32_t* vb = seg<uint32_t>(ws, pl.ws.vis_b);
  uint32_t* scratch = seg<uint32_t>(ws, pl.ws.depth);
  const unsigned gb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_cell_keys, dim3(gb), dim3(256), 0, st, cell_of, n, n_active, (uint32_t)n_cells, cell_bits, ka,
                     va);
  bool in_b = false;
  hipError_t e = launch_sort_pairs(pl, ws, ka, va, kb, vb, n, bits, &in_b, st);
  if (e != hipSuccess) return e;
  const uint32_t* from = in_b ? vb : va;   // from[k] = old position of the Gaussian that lands at k
  auto permute = [&](uint32_t* row, int64_t len) {
    if (len == 0) return;
    const unsigned g = (unsigned)((len + 255) / 256);
    hipLaunchKernelGGL(k_copy_row, dim3(g), dim3(256), 0, st, row, scratch, len);
    hipLaunchKernelGGL(k_gather_row, dim3(g), dim3(256), 0, st, scratch, from, len, row);
  };
  const int nk = (p.sh_degree + 1) * (p.sh_degree + 1);
  auto permute_tensor = [&](const gs_params& t, int64_t len) {
    float* rows_of[5] = {t.mean, t.log_scale, t.quat, t.opacity_logit, t.sh};
    const int count[5] = {3, 3, 4, 1, 3 * nk};
    for (int g = 0; g < 5; ++g)
      for (int r = 0; r < count[g]; ++r) permute(reinterpret_cast<uint32_t*>(rows_of[g] + (int64_t)r * len), len);
  };
  permute_tensor(p, n);
  if (base) permute_tensor(*base, n);
  if (ids) permute(ids, n);
  permute(cell_of, n);
  // the active prefix maps onto itself (pool bit above the cell), so the
  // moments take the permutation's first n_active entries
  if (m) permute_tensor(*m, n_active);
  if (v) permute_tensor(*v, n_active);
  return hipGetLastError();
}

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
