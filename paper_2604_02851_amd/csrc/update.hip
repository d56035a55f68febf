// Parameter update (fused Adam over every tensor) and changed-Gaussian delta
// extraction with stable compaction.  Both are streaming, HBM-bound kernels:
// one pass over the parameters and their state, coalesced planar accesses.
#include "internal.h"

namespace gs {
namespace {

struct AdamSeg {
  float* theta;      // row r of the group at theta + r * n_total
  const float* g;    // gradient and moments: row r at + r * n_active
  float* m;
  float* v;
  int32_t rows;
  float lr;
};

struct AdamArgs {
  AdamSeg seg[6];
  int64_t chunk0[7];   // first chunk of each group (exclusive prefix), chunk0[6] = total
  int64_t n_total;     // parameter row stride
  int64_t n_active;    // trainable Gaussians (a prefix): elements per row and moment row stride
  int64_t row_chunks;  // chunks per row
  const int32_t* step;
  float beta1, beta2, eps;
};

constexpr int kAdamVec = 4;                    // elements per thread
constexpr int kAdamChunk = 256 * kAdamVec;     // elements per workgroup

__device__ __forceinline__ void adam_one(float& th, float g, float& m, float& v, float b1, float b2, float c1,
                                         float c2, float step, float rbc2, float eps) {
  m = fmaf(b1, m, c1 * g);
  v = fmaf(b2, v, c2 * g * g);
  th -= step * m / (sqrtf(v) * rbc2 + eps);
}

// One workgroup per chunk of kAdamChunk elements of one row of one group;
// thread t updates 4 consecutive elements (one 16-byte access per array when
// aligned, scalar otherwise and in the row's tail).  Only the first n_active
// Gaussians of each row are trainable; frozen ones are left untouched.  The
// bias corrections are computed once per workgroup in FP64.
__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
  __shared__ float s_corr[2];
  int si = 0;
#pragma unroll
  for (int q = 1; q < 6; ++q) si += (int64_t)blockIdx.x >= a.chunk0[q] ? 1 : 0;
  const AdamSeg s = a.seg[si];
  if (threadIdx.x == 0) {
    const int t = *a.step + 1;
    const double bc1 = 1.0 - pow((double)a.beta1, (double)t);
    s_corr[0] = (float)bc1;
    s_corr[1] = (float)(1.0 / sqrt(1.0 - pow((double)a.beta2, (double)t)));
  }
  __syncthreads();
  const float step = s.lr / s_corr[0], rbc2 = s_corr[1];
  const float b1 = a.beta1, b2 = a.beta2, c1 = 1.f - a.beta1, c2 = 1.f - a.beta2, eps = a.eps;
  const int64_t local = (int64_t)blockIdx.x - a.chunk0[si];
  const int64_t row = local / a.row_chunks, chunk = local - row * a.row_chunks;
  const int64_t k0 = chunk * kAdamChunk + (int64_t)threadIdx.x * kAdamVec;
  if (k0 >= a.n_active) return;
  float* th_p = s.theta + row * a.n_total + k0;
  const float* g_p = s.g + row * a.n_active + k0;
  float* m_p = s.m + row * a.n_active + k0;
  float* v_p = s.v + row * a.n_active + k0;
  const bool vec = k0 + kAdamVec <= a.n_active &&
                   ((reinterpret_cast<uintptr_t>(th_p) | reinterpret_cast<uintptr_t>(g_p) |
                     reinterpret_cast<uintptr_t>(m_p) | reinterpret_cast<uintptr_t>(v_p)) & 15u) == 0;
  if (vec) {
    float4 th = *reinterpret_cast<const float4*>(th_p);
    const float4 g = *reinterpret_cast<const float4*>(g_p);
    float4 m = *reinterpret_cast<const float4*>(m_p);
    float4 v = *reinterpret_cast<const float4*>(v_p);
    adam_one(th.x, g.x, m.x, v.x, b1, b2, c1, c2, step, rbc2, eps);
    adam_one(th.y, g.y, m.y, v.y, b1, b2, c1, c2, step, rbc2, eps);
    adam_one(th.z, g.z, m.z, v.z, b1, b2, c1, c2, step, rbc2, eps);
    adam_one(th.w, g.w, m.w, v.w, b1, b2, c1, c2, step, rbc2, eps);
    *reinterpret_cast<float4*>(m_p) = m;
    *reinterpret_cast<float4*>(v_p) = v;
    *reinterpret_cast<float4*>(th_p) = th;
  } else {
    for (int c = 0; c < kAdamVec && k0 + c < a.n_active; ++c) {
      float th = th_p[c], m = m_p[c], v = v_p[c];
      adam_one(th, g_p[c], m, v, b1, b2, c1, c2, step, rbc2, eps);
      m_p[c] = m;
      v_p[c] = v;
      th_p[c] = th;
    }
  }
}

__global__ void k_bump(int32_t* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

__global__ void k_bump_u32(uint32_t* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += 1u;
}

// ---- delta extraction -------------------------------------------------------
struct DeltaGroups {
  const float* cur[6];
  float* base[6];
  int32_t width[6];
};

struct DeltaArgs {
  DeltaGroups g;
  int64_t n;
  uint32_t mask;
  float tau;
  uint8_t* flags;
  uint32_t* bcount;   // [6][nb], scanned in place
  uint32_t* dbase;    // [0..5] section base, [6..11] count, [15] total
  int32_t nb;
  uint32_t* out;
};

__global__ __launch_bounds__(256) void k_delta_flags(DeltaArgs a) {
  __shared__ uint32_t s_w[6][4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  uint32_t f = 0;
  if (i < a.n) {
    for (int g = 0; g < 6; ++g) {
      if (!((a.mask >> g) & 1u)) continue;
      bool hit = false;
      for (int k = 0; k < a.g.width[g] && !hit; ++k) {
        const float p = a.g.cur[g][(int64_t)k * a.n + i];
        const float b = a.g.base[g][(int64_t)k * a.n + i];
        const float diff = fabsf(p - b);
        const float thr = a.tau * fabsf(b);
        hit = diff > thr;
      }
      f |= hit ? (1u << g) : 0u;
    }
    a.flags[i] = (uint8_t)f;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int g = 0; g < 6; ++g) {
    const uint64_t bal = __ballot((f >> g) & 1u);
    if (lane == 0) s_w[g][w] = (uint32_t)__popcll(bal);
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int g = threadIdx.x;
    a.bcount[(int64_t)g * a.nb + blockIdx.x] = s_w[g][0] + s_w[g][1] + s_w[g][2] + s_w[g][3];
  }
}

__global__ void k_delta_header(DeltaArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t run = 6;
  for (int g = 0; g < 6; ++g) {
    const uint32_t lo = a.bcount[(int64_t)g * a.nb];
    const uint32_t hi = g < 5 ? a.bcount[(int64_t)(g + 1) * a.nb] : a.dbase[15];
    const uint32_t c = hi - lo;
    a.dbase[g] = run;
    a.dbase[6 + g] = c;
    a.out[g] = c;
    run += c * (1u + (uint32_t)a.g.width[g]);
  }
}

__global__ __launch_bounds__(256) void k_delta_write(DeltaArgs a) {
  __shared__ uint32_t s_w[6][4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t f = i < a.n ? a.flags[i] : 0u;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint32_t wrank[6];
  for (int g = 0; g < 6; ++g) {
    const uint64_t bal = __ballot((f >> g) & 1u);
    wrank[g] = (uint32_t)__popcll(bal & lt);
    if (lane == 0) s_w[g][w] = (uint32_t)__popcll(bal);
  }
  __syncthreads();
  if (f == 0) return;
  for (int g = 0; g < 6; ++g) {
    if (!((f >> g) & 1u)) continue;
    uint32_t r = wrank[g];
    for (int q = 0; q < w; ++q) r += s_w[g][q];
    r += a.bcount[(int64_t)g * a.nb + blockIdx.x] - a.bcount[(int64_t)g * a.nb];
    const uint32_t base = a.dbase[g], cnt = a.dbase[6 + g];
    const int wd = a.g.width[g];
    a.out[base + r] = (uint32_t)i;
    uint32_t* vals = a.out + base + cnt + (size_t)r * wd;
    for (int k = 0; k < wd; ++k) {
      const float p = a.g.cur[g][(int64_t)k * a.n + i];
      vals[k] = __float_as_uint(p);
      a.g.base[g][(int64_t)k * a.n + i] = p;
    }
  }
}

// ---- freezing: stable partition of the active pool ----------------------------
// Active Gaussians flagged for freezing move behind the ones that stay
// active (both in their old order), ahead of the Gaussians frozen before;
// the moments of the Gaussians that stay active are compacted to the new
// active count.  Rows are moved one at a time through a scratch copy.
__global__ void k_fill_i32_zero(int32_t* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__global__ void k_keep_flags(const uint8_t* flags, int64_t n_active, uint32_t* keep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_active) keep[i] = flags[i] ? 0u : 1u;
}

__global__ void k_freeze_dst(const uint32_t* pos, const uint32_t* kept, const uint8_t* flags, int64_t n_active,
                             uint32_t* dst, int32_t* new_active) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nk = *kept;
  if (i == 0) *new_active = (int32_t)nk;
  if (i < n_active) dst[i] = flags[i] ? nk + (uint32_t)i - pos[i] : pos[i];
}

__global__ void k_copy_words(const uint32_t* src, uint32_t* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// row[dst[i]] = scratch[i] for i < n_active (a permutation of the prefix)
__global__ void k_scatter_words(const uint32_t* scratch, const uint32_t* dst, int64_t n_active, uint32_t* row) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_active) row[dst[i]] = scratch[i];
}

// moment row r, compacted: (base + r * kept)[pos[i]] = scratch[i] for kept i
__global__ void k_compact_words(const uint32_t* scratch, const uint32_t* pos, const uint8_t* flags, int64_t n_active,
                                const uint32_t* kept, uint32_t* base, int64_t r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_active && !flags[i]) base[r * (int64_t)*kept + pos[i]] = scratch[i];
}

}  // namespace

hipError_t launch_adam(const gs_params& p, const gs_params& g, const gs_params& m, const gs_params& v, int32_t* step,
                       const gs_adam_hparams& hp, hipStream_t st) {
  const int64_t n = p.n, na = g.n;
  const int nk = (p.sh_degree + 1) * (p.sh_degree + 1);
  AdamArgs a;
  auto setseg = [&](int s, float* th, const float* gr, float* mm, float* vv, int rows, int64_t row0) {
    a.seg[s] = AdamSeg{th + row0 * n, gr + row0 * na, mm + row0 * na, vv + row0 * na, rows, hp.lr[s]};
  };
  setseg(0, p.mean, g.mean, m.mean, v.mean, 3, 0);
  setseg(1, p.log_scale, g.log_scale, m.log_scale, v.log_scale, 3, 0);
  setseg(2, p.quat, g.quat, m.quat, v.quat, 4, 0);
  setseg(3, p.opacity_logit, g.opacity_logit, m.opacity_logit, v.opacity_logit, 1, 0);
  setseg(4, p.sh, g.sh, m.sh, v.sh, 3, 0);
  setseg(5, p.sh, g.sh, m.sh, v.sh, 3 * (nk - 1), 3);
  a.n_total = n;
  a.n_active = na;
  a.row_chunks = (na + kAdamChunk - 1) / kAdamChunk;
  a.step = step;
  a.beta1 = hp.beta1;
  a.beta2 = hp.beta2;
  a.eps = hp.eps;
  a.chunk0[0] = 0;
  for (int q = 0; q < 6; ++q) a.chunk0[q + 1] = a.chunk0[q] + (int64_t)a.seg[q].rows * a.row_chunks;
  if (a.chunk0[6] > 0x7fffffffll) return hipErrorInvalidValue;
  if (a.chunk0[6] > 0) hipLaunchKernelGGL(k_adam, dim3((unsigned)a.chunk0[6]), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, st, step);
  return hipGetLastError();
}

static inline unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_freeze(const Plan& pl, const gs_params& p, const gs_params& m, const gs_params& v,
                         const uint8_t* flags, uint32_t* ids, const gs_params* base, void* ws, int32_t* new_active,
                         hipStream_t st) {
  const int64_t n = p.n, na = m.n;
  if (na == 0) {
    hipLaunchKernelGGL(k_fill_i32_zero, dim3(1), dim3(64), 0, st, new_active);
    return hipGetLastError();
  }
  uint32_t* keep = seg<uint32_t>(ws, pl.ws.depth);
  uint32_t* pos = seg<uint32_t>(ws, pl.ws.koff);
  uint32_t* dst = seg<uint32_t>(ws, pl.ws.vkey_a);
  uint32_t* scratch = seg<uint32_t>(ws, pl.ws.vkey_b);
  uint32_t* kept = &seg<Counters>(ws, pl.ws.counters)->pad[0];
  hipLaunchKernelGGL(k_keep_flags, dim3(blocks256(na)), dim3(256), 0, st, flags, na, keep);
  hipError_t e = launch_scan(keep, pos, na, nullptr, seg<uint32_t>(ws, pl.ws.partial), pl.ws.partial_len, kept, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_freeze_dst, dim3(blocks256(na)), dim3(256), 0, st, pos, kept, flags, na, dst, new_active);
  const int nk = (p.sh_degree + 1) * (p.sh_degree + 1);
  auto permute_rows = [&](const gs_params& t) {
    float* rows_of[5] = {t.mean, t.log_scale, t.quat, t.opacity_logit, t.sh};
    const int count[5] = {3, 3, 4, 1, 3 * nk};
    for (int g = 0; g < 5; ++g)
      for (int r = 0; r < count[g]; ++r) {
        uint32_t* row = reinterpret_cast<uint32_t*>(rows_of[g] + (int64_t)r * n);
        hipLaunchKernelGGL(k_copy_words, dim3(blocks256(na)), dim3(256), 0, st, row, scratch, na);
        hipLaunchKernelGGL(k_scatter_words, dim3(blocks256(na)), dim3(256), 0, st, scratch, dst, na, row);
      }
  };
  auto compact_rows = [&](const gs_params& t) {
    float* rows_of[5] = {t.mean, t.log_scale, t.quat, t.opacity_logit, t.sh};
    const int count[5] = {3, 3, 4, 1, 3 * nk};
    for (int g = 0; g < 5; ++g)
      for (int r = 0; r < count[g]; ++r) {
        uint32_t* base = reinterpret_cast<uint32_t*>(rows_of[g]);
        hipLaunchKernelGGL(k_copy_words, dim3(blocks256(na)), dim3(256), 0, st, base + (int64_t)r * na, scratch, na);
        hipLaunchKernelGGL(k_compact_words, dim3(blocks256(na)), dim3(256), 0, st, scratch, pos, flags, na, kept,
                           base, (int64_t)r);
      }
  };
  permute_rows(p);
  if (base) permute_rows(*base);
  if (ids) {
    hipLaunchKernelGGL(k_copy_words, dim3(blocks256(na)), dim3(256), 0, st, ids, scratch, na);
    hipLaunchKernelGGL(k_scatter_words, dim3(blocks256(na)), dim3(256), 0, st, scratch, dst, na, ids);
  }
  compact_rows(m);
  compact_rows(v);
  return hipGetLastError();
}

hipError_t launch_epoch_bump(uint32_t* epoch, hipStream_t st) {
  hipLaunchKernelGGL(k_bump_u32, dim3(1), dim3(64), 0, st, epoch);
  return hipGetLastError();
}

hipError_t launch_delta(const Plan& pl, const gs_params& cur, const gs_params& base, uint32_t mask, float tau,
                        uint32_t* out, void* ws, hipStream_t st) {
  DeltaArgs a;
  const int64_t n = cur.n;
  const int nk = (cur.sh_degree + 1) * (cur.sh_degree + 1);
  a.g.cur[0] = cur.opacity_logit;  a.g.base[0] = base.opacity_logit;  a.g.width[0] = 1;
  a.g.cur[1] = cur.sh;             a.g.base[1] = base.sh;             a.g.width[1] = 3;
  a.g.cur[2] = cur.sh + 3 * n;     a.g.base[2] = base.sh + 3 * n;     a.g.width[2] = 3 * (nk - 1);
  a.g.cur[3] = cur.mean;           a.g.base[3] = base.mean;           a.g.width[3] = 3;
  a.g.cur[4] = cur.log_scale;      a.g.base[4] = base.log_scale;      a.g.width[4] = 3;
  a.g.cur[5] = cur.quat;           a.g.base[5] = base.quat;           a.g.width[5] = 4;
  a.n = n;
  a.mask = mask;
  a.tau = tau;
  a.flags = seg<uint8_t>(ws, pl.ws.dflags);
  a.bcount = seg<uint32_t>(ws, pl.ws.dcount);
  a.dbase = seg<uint32_t>(ws, pl.ws.dbase);
  a.nb = (int32_t)((n + 255) / 256);
  a.out = out;
  if (a.nb > pl.ws.dblocks) return hipErrorInvalidValue;
  if (a.nb > 0) hipLaunchKernelGGL(k_delta_flags, dim3(a.nb), dim3(256), 0, st, a);
  hipError_t e = launch_scan(a.bcount, a.bcount, 6ll * a.nb, nullptr, seg<uint32_t>(ws, pl.ws.partial),
                             pl.ws.partial_len, a.dbase + 15, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_delta_header, dim3(1), dim3(64), 0, st, a);
  if (a.nb > 0) hipLaunchKernelGGL(k_delta_write, dim3(a.nb), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
