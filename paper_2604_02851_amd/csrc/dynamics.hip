// Scene dynamics (Sec. 3.4) and model expansion (Sec. 3.3) on the device.
//
//  * Rigid objects: Gaussians carry an object index; before an optimization
//    step the engine's object motion x -> R (x - p) + p + t (R the rotation of
//    the unit quaternion q / |q|) is applied to the means of the object's
//    Gaussians, and q / |q| is composed onto their orientation quaternions.
//    FP64 arithmetic, one rounding to FP32 per stored value.
//  * Relighting of the diffuse DC term: the DC colour C0 dc + 1/2 of each
//    channel is scaled by a per-Gaussian gain (one for all channels or one
//    per channel); a gain of exactly 1 leaves the coefficient untouched.
//  * Appending: new Gaussians join the end of the active pool (the frozen
//    pool moves up by their count); optimizer moments are extended with
//    zeros.  Written out of place into caller-sized tensors, row by row.
#include "internal.h"

namespace gs {
namespace {

__global__ __launch_bounds__(256) void k_object_transform(float* mean, float* quat, int64_t n,
                                                           const int32_t* object_of, const gs_transform* tf,
                                                           int32_t n_objects) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t o = object_of[i];
  if (o < 0 || o >= n_objects) return;
  const gs_transform T = tf[o];
  const double qn = sqrt((double)T.q[0] * T.q[0] + (double)T.q[1] * T.q[1] + (double)T.q[2] * T.q[2] +
                         (double)T.q[3] * T.q[3]);
  const double w = T.q[0] / qn, x = T.q[1] / qn, y = T.q[2] / qn, z = T.q[3] / qn;
  const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                       2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                       2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = (double)mean[k * n + i] - (double)T.pivot[k];
  for (int r = 0; r < 3; ++r)
    mean[r * n + i] = (float)(R[r * 3] * d[0] + R[r * 3 + 1] * d[1] + R[r * 3 + 2] * d[2] + (double)T.pivot[r] +
                              (double)T.t[r]);
  const double bw = quat[i], bx = quat[n + i], by = quat[2 * n + i], bz = quat[3 * n + i];
  quat[i] = (float)(w * bw - x * bx - y * by - z * bz);
  quat[n + i] = (float)(w * bx + x * bw + y * bz - z * by);
  quat[2 * n + i] = (float)(w * by - x * bz + y * bw + z * bx);
  quat[3 * n + i] = (float)(w * bz + x * by - y * bx + z * bw);
}

__global__ __launch_bounds__(256) void k_relight_dc(float* sh, int64_t n, const float* gain, int channels) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double c0 = 0.28209479177387814;   // 1 / (2 sqrt(pi)), the degree-0 basis function
  for (int c = 0; c < 3; ++c) {
    const float g = gain[(channels == 3 ? c : 0) * n + i];
    if (g == 1.0f) continue;
    const double dc = sh[c * n + i];
    sh[c * n + i] = (float)(((c0 * dc + 0.5) * (double)g - 0.5) / c0);
  }
}

// dst row r (stride dst_n): old[0, na) | add[0, k) (zeros when add is null) | old[na, n_old)
__global__ __launch_bounds__(256) void k_append_rows(const uint32_t* old, int64_t n_old, int64_t na,
                                                      const uint32_t* add, int64_t k, uint32_t* dst) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  const int64_t dst_n = n_old + k;
  if (j >= dst_n) return;
  uint32_t v;
  if (j < na) v = old[r * n_old + j];
  else if (j < na + k) v = add ? add[r * k + (j - na)] : 0u;
  else v = old[r * n_old + (j - k)];
  dst[r * dst_n + j] = v;
}

}  // namespace

hipError_t launch_object_transform(const gs_params& p, const int32_t* object_of, const gs_transform* tf,
                                   int32_t n_objects, hipStream_t st) {
  if (p.n > 0 && n_objects > 0)
    hipLaunchKernelGGL(k_object_transform, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, st, p.mean, p.quat,
                       (int64_t)p.n, object_of, tf, n_objects);
  return hipGetLastError();
}

hipError_t launch_relight_dc(const gs_params& p, const float* gain, int channels, hipStream_t st) {
  if (p.n > 0)
    hipLaunchKernelGGL(k_relight_dc, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, st, p.sh, (int64_t)p.n,
                       gain, channels);
  return hipGetLastError();
}

hipError_t launch_append(const gs_params& old_p, const gs_params* old_m, const gs_params* old_v, int64_t na,
                         const gs_params& add, const gs_params& new_p, const gs_params* new_m,
                         const gs_params* new_v, const uint32_t* const* old_cols, const uint32_t* const* add_cols,
                         uint32_t* const* new_cols, int n_cols, hipStream_t st) {
  const int nk = (old_p.sh_degree + 1) * (old_p.sh_degree + 1);
  const int rows[5] = {3, 3, 4, 1, 3 * nk};
  const int64_t k = add.n;
  auto rows_of = [](const gs_params& t, int g) -> float* {
    float* r[5] = {t.mean, t.log_scale, t.quat, t.opacity_logit, t.sh};
    return r[g];
  };
  auto copy = [&](const void* old, int64_t n_old, int64_t keep, const void* add_rows, void* dst, int nrows) {
    const int64_t dn = n_old + k;
    if (dn == 0 || nrows == 0) return;
    hipLaunchKernelGGL(k_append_rows, dim3((unsigned)((dn + 255) / 256), (unsigned)nrows), dim3(256), 0, st,
                       static_cast<const uint32_t*>(old), n_old, keep, static_cast<const uint32_t*>(add_rows), k,
                       static_cast<uint32_t*>(dst));
  };
  for (int g = 0; g < 5; ++g) {
    copy(rows_of(old_p, g), old_p.n, na, rows_of(add, g), rows_of(new_p, g), rows[g]);
    if (old_m) copy(rows_of(*old_m, g), na, na, nullptr, rows_of(*new_m, g), rows[g]);
    if (old_v) copy(rows_of(*old_v, g), na, na, nullptr, rows_of(*new_v, g), rows[g]);
  }
  for (int c = 0; c < n_cols; ++c) copy(old_cols[c], old_p.n, na, add_cols[c], new_cols[c], 1);
  return hipGetLastError();
}

}  // namespace gs
