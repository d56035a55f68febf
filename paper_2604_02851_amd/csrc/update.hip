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
  const gs_adam_hparams* dev_hp;   // when set: hyper-parameters read here at run time instead
};

typedef float V4 __attribute__((ext_vector_type(4)));
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
  __shared__ float s_hp[4];   // this group's lr, beta1, beta2, eps
  int si = 0;
#pragma unroll
  for (int q = 1; q < 6; ++q) si += (int64_t)blockIdx.x >= a.chunk0[q] ? 1 : 0;
  const AdamSeg s = a.seg[si];
  if (threadIdx.x == 0) {
    const gs_adam_hparams* h = a.dev_hp;
    const float lr = h ? h->lr[si] : s.lr, b1 = h ? h->beta1 : a.beta1, b2 = h ? h->beta2 : a.beta2;
    s_hp[0] = lr, s_hp[1] = b1, s_hp[2] = b2, s_hp[3] = h ? h->eps : a.eps;
    const int t = *a.step + 1;
    const double bc1 = 1.0 - pow((double)b1, (double)t);
    s_corr[0] = (float)bc1;
    s_corr[1] = (float)(1.0 / sqrt(1.0 - pow((double)b2, (double)t)));
  }
  __syncthreads();
  const float step = s_hp[0] / s_corr[0], rbc2 = s_corr[1];
  const float b1 = s_hp[1], b2 = s_hp[2], c1 = 1.f - b1, c2 = 1.f - b2, eps = s_hp[3];
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
    // every value is touched once per step: streaming (non-temporal) accesses
    // keep the update from evicting what the other stages reuse
    V4 th = __builtin_nontemporal_load(reinterpret_cast<const V4*>(th_p));
    const V4 g = __builtin_nontemporal_load(reinterpret_cast<const V4*>(g_p));
    V4 m = __builtin_nontemporal_load(reinterpret_cast<const V4*>(m_p));
    V4 v = __builtin_nontemporal_load(reinterpret_cast<const V4*>(v_p));
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      float t = th[c], mc = m[c], vc = v[c];
      adam_one(t, g[c], mc, vc, b1, b2, c1, c2, step, rbc2, eps);
      th[c] = t, m[c] = mc, v[c] = vc;
    }
    __builtin_nontemporal_store(m, reinterpret_cast<V4*>(m_p));
    __builtin_nontemporal_store(v, reinterpret_cast<V4*>(v_p));
    __builtin_nontemporal_store(th, reinterpret_cast<V4*>(th_p));
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

// ---- delta extraction and delta codecs ---------------------------------------
// One set of kernels serves the plain extraction (every group raw, 6-word
// header) and the coded packets (9-word header: epoch, mask, counts, total).
// Per group the codec decides which rows are sent and what their words hold:
//   raw       rows with fl32(|p - b|) > fl32(tau |b|); FP32 values
//   residual  c = clamp(rint((p - b) * inv), +-(2^(B-1) - 1)); rows with some
//             c != 0; baseline b + c step (what the receiver rebuilds)
//   quantized q(x) = clamp(rint((x - lo) * inv), 0, 2^B - 1); rows with some
//             q(p) != q(b); baseline lo + q(p) step
// Every operation is a separately rounded FP32 operation (contraction is off
// in these functions, written with plain operators: the header's rounding
// intrinsics would be fused under the default contraction of their own
// definitions),
// so that sender and receiver reconstruct bit-identical values.  Codes are
// packed little-endian, 32/B per word, each row starting on a word.
struct DeltaGroups {
  const float* cur[6];
  float* base[6];
  int32_t width[6];
};

struct CodecDev {
  int32_t mode[6], bits[6], wpr[6];
  float step[6], inv[6], lo[6], tau[6];
};

struct DeltaArgs {
  DeltaGroups g;
  CodecDev c;
  int64_t n;
  uint32_t mask;
  int32_t hdr;              // 6 (plain extraction) or 9 (coded packet)
  const uint32_t* epoch;    // coded packets: the transmission epoch
  uint8_t* flags;
  uint32_t* bcount;   // [6][nb], scanned in place
  uint32_t* dbase;    // [0..5] section base, [6..11] count, [15] total
  int32_t nb;
  uint32_t* out;
};

__device__ __forceinline__ float q_index(float x) {   // rint, NaN -> 0
  const float q = rintf(x);
  return q == q ? q : 0.f;
}

__device__ __forceinline__ int32_t residual_code(float p, float b, float inv, int bits) {
#pragma clang fp contract(off)
  const float m = (float)((1 << (bits - 1)) - 1);
  const float q = q_index((p - b) * inv);
  return (int32_t)fminf(fmaxf(q, -m), m);
}

__device__ __forceinline__ int32_t quant_code(float x, float lo, float inv, int bits) {
#pragma clang fp contract(off)
  const float m = (float)((1 << bits) - 1);
  const float q = q_index((x - lo) * inv);
  return (int32_t)fminf(fmaxf(q, 0.f), m);
}

__device__ __forceinline__ bool row_sent(const DeltaArgs& a, int g, int64_t i) {
#pragma clang fp contract(off)
  const int md = a.c.mode[g];
  for (int k = 0; k < a.g.width[g]; ++k) {
    const float p = a.g.cur[g][(int64_t)k * a.n + i];
    const float b = a.g.base[g][(int64_t)k * a.n + i];
    bool hit;
    if (md == 0) hit = fabsf(p - b) > a.c.tau[g] * fabsf(b);
    else if (md == 1) hit = residual_code(p, b, a.c.inv[g], a.c.bits[g]) != 0;
    else hit = quant_code(p, a.c.lo[g], a.c.inv[g], a.c.bits[g]) != quant_code(b, a.c.lo[g], a.c.inv[g], a.c.bits[g]);
    if (hit) return true;
  }
  return false;
}

__global__ __launch_bounds__(256) void k_delta_flags(DeltaArgs a) {
  __shared__ uint32_t s_w[6][4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  uint32_t f = 0;
  if (i < a.n) {
    for (int g = 0; g < 6; ++g)
      if (((a.mask >> g) & 1u) && row_sent(a, g, i)) f |= 1u << g;
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
  uint32_t run = (uint32_t)a.hdr;
  for (int g = 0; g < 6; ++g) {
    // (no Gaussians: no block counts were written, every group is empty)
    const uint32_t lo = a.nb > 0 ? a.bcount[(int64_t)g * a.nb] : 0u;
    const uint32_t hi = a.nb > 0 ? (g < 5 ? a.bcount[(int64_t)(g + 1) * a.nb] : a.dbase[15]) : 0u;
    const uint32_t c = hi - lo;
    a.dbase[g] = run;
    a.dbase[6 + g] = c;
    a.out[a.hdr == 6 ? g : 2 + g] = c;
    run += c * (1u + (uint32_t)a.c.wpr[g]);
  }
  if (a.hdr == 9) {
    a.out[0] = *a.epoch;
    a.out[1] = a.mask;
    a.out[8] = run;
  }
}

__global__ __launch_bounds__(256) void k_delta_write(DeltaArgs a) {
#pragma clang fp contract(off)
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
    const int wd = a.g.width[g], md = a.c.mode[g];
    const int64_t wpr = a.c.wpr[g];
    a.out[base + r] = (uint32_t)i;
    uint32_t* vals = a.out + base + cnt + (size_t)r * wpr;
    if (md == 0) {
      for (int k = 0; k < wd; ++k) {
        const float p = a.g.cur[g][(int64_t)k * a.n + i];
        vals[k] = __float_as_uint(p);
        a.g.base[g][(int64_t)k * a.n + i] = p;
      }
      continue;
    }
    const int B = a.c.bits[g], per = 32 / B;
    const uint32_t fmask = (1u << B) - 1u;
    const float step = a.c.step[g], inv = a.c.inv[g], lo = a.c.lo[g];
    uint32_t word = 0u;
    for (int k = 0; k < wd; ++k) {
      const float p = a.g.cur[g][(int64_t)k * a.n + i];
      float& b = a.g.base[g][(int64_t)k * a.n + i];
      const int32_t c = md == 1 ? residual_code(p, b, inv, B) : quant_code(p, lo, inv, B);
      const float t = (float)c * step;
      b = md == 1 ? (b + t) : (lo + t);
      word |= ((uint32_t)c & fmask) << ((k % per) * B);
      if (k % per == per - 1 || k == wd - 1) {
        vals[k / per] = word;
        word = 0u;
      }
    }
  }
}

// ---- client replay: apply a coded packet to the receiver's model -------------
struct ApplyArgs {
  float* grp[6];
  int32_t width[6];
  CodecDev c;
  int64_t n;
  const uint32_t* pk;
  int64_t pk_words;
  const uint32_t* epoch;
  uint32_t* status;
};

// header sanity (every thread derives the same answer); false if malformed
__device__ bool packet_layout(const ApplyArgs& a, int64_t* sec) {
  if (a.pk_words < 9) return false;
  const uint32_t mask = a.pk[1];
  if (mask & ~0x3Fu) return false;
  int64_t total = 9;
  for (int g = 0; g < 6; ++g) {
    const int64_t c = a.pk[2 + g];
    if ((!((mask >> g) & 1u) && c != 0) || c > a.n) return false;
    sec[g] = total;
    total += c * (1 + (int64_t)a.c.wpr[g]);
  }
  return total == (int64_t)a.pk[8] && total <= a.pk_words;
}

__global__ __launch_bounds__(256) void k_apply_check(ApplyArgs a) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t sec[6];
  if (!packet_layout(a, sec)) {
    if (t0 == 0) atomicOr(a.status, 2u);
    return;
  }
  if (t0 == 0 && a.pk[0] != *a.epoch) atomicOr(a.status, 1u);
  uint32_t bad = 0u;
  for (int g = 0; g < 6; ++g) {
    const int64_t c = a.pk[2 + g];
    const uint32_t* idx = a.pk + sec[g];
    for (int64_t r = t0; r < c; r += stride) {
      const uint32_t i = idx[r];
      if ((int64_t)i >= a.n || (r > 0 && idx[r - 1] >= i)) bad = 2u;
    }
  }
  if (bad) atomicOr(a.status, bad);
}

__global__ __launch_bounds__(256) void k_apply(ApplyArgs a) {
#pragma clang fp contract(off)
  if (*a.status != 0u) return;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t sec[6];
  if (!packet_layout(a, sec)) return;   // (the check already reported it)
  for (int g = 0; g < 6; ++g) {
    const int64_t c = a.pk[2 + g];
    const uint32_t* idx = a.pk + sec[g];
    const int64_t wpr = a.c.wpr[g];
    const uint32_t* vals = idx + c;
    const int wd = a.width[g], md = a.c.mode[g];
    for (int64_t r = t0; r < c; r += stride) {
      const int64_t i = idx[r];
      const uint32_t* row = vals + r * wpr;
      if (md == 0) {
        for (int k = 0; k < wd; ++k) a.grp[g][(int64_t)k * a.n + i] = __uint_as_float(row[k]);
        continue;
      }
      const int B = a.c.bits[g], per = 32 / B;
      const uint32_t fmask = (1u << B) - 1u;
      for (int k = 0; k < wd; ++k) {
        const uint32_t field = (row[k / per] >> ((k % per) * B)) & fmask;
        const int32_t code = (md == 1 && ((field >> (B - 1)) & 1u)) ? (int32_t)field - (1 << B) : (int32_t)field;
        float& x = a.grp[g][(int64_t)k * a.n + i];
        const float t = (float)code * a.c.step[g];
        x = md == 1 ? (x + t) : (a.c.lo[g] + t);
      }
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
                       const gs_adam_hparams& hp, const gs_adam_hparams* dev_hp, hipStream_t st) {
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
  a.dev_hp = dev_hp;
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
  uint32_t* kept = &seg<Counters>(ws, pl.ws.counters)->kept;
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

static void set_groups(const gs_params& cur, float* const* base_rows, DeltaGroups& g) {
  const int64_t n = cur.n;
  const int nk = (cur.sh_degree + 1) * (cur.sh_degree + 1);
  const float* c[6] = {cur.opacity_logit, cur.sh, cur.sh + 3 * n, cur.mean, cur.log_scale, cur.quat};
  const int32_t w[6] = {1, 3, 3 * (nk - 1), 3, 3, 4};
  for (int q = 0; q < 6; ++q) {
    g.cur[q] = c[q];
    g.base[q] = base_rows[q];
    g.width[q] = w[q];
  }
}

static void group_rows(const gs_params& t, float** rows) {
  const int64_t n = t.n;
  float* r[6] = {t.opacity_logit, t.sh, t.sh + 3 * n, t.mean, t.log_scale, t.quat};
  for (int q = 0; q < 6; ++q) rows[q] = r[q];
}

static CodecDev codec_dev(const gs_codec* codecs, const int32_t* width) {
  CodecDev d;
  for (int g = 0; g < 6; ++g) {
    const gs_codec& k = codecs[g];
    d.mode[g] = k.mode;
    d.bits[g] = k.mode == GS_CODEC_RAW ? 32 : k.bits;
    d.wpr[g] = (int32_t)codec_row_words(k, width[g]);
    d.step[g] = k.step;
    d.inv[g] = 1.0f / k.step;
    d.lo[g] = k.lo;
    d.tau[g] = k.rel_tau;
  }
  return d;
}

// The delta kernels' scratch: a flag byte per Gaussian, six block-count rows
// (scanned in place), the scan's partials and the section bases.  Nothing in
// it needs to start at zero: every call writes each word it reads.
struct DeltaScratch {
  uint8_t* flags;
  uint32_t* bcount;
  uint32_t* partial;
  int64_t partial_len;
  uint32_t* dbase;
  int32_t max_blocks;
};

static hipError_t run_delta(DeltaArgs& a, const DeltaScratch& s, hipStream_t st) {
  a.flags = s.flags;
  a.bcount = s.bcount;
  a.dbase = s.dbase;
  a.nb = (int32_t)((a.n + 255) / 256);
  if (a.nb > s.max_blocks) return hipErrorInvalidValue;
  if (a.nb > 0) hipLaunchKernelGGL(k_delta_flags, dim3(a.nb), dim3(256), 0, st, a);
  hipError_t e = launch_scan(a.bcount, a.bcount, 6ll * a.nb, nullptr, s.partial, s.partial_len, a.dbase + 15, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_delta_header, dim3(1), dim3(64), 0, st, a);
  if (a.nb > 0) hipLaunchKernelGGL(k_delta_write, dim3(a.nb), dim3(256), 0, st, a);
  return hipGetLastError();
}

static hipError_t run_delta(const Plan& pl, DeltaArgs& a, void* ws, hipStream_t st) {
  const DeltaScratch s{seg<uint8_t>(ws, pl.ws.dflags), seg<uint32_t>(ws, pl.ws.dcount),
                       seg<uint32_t>(ws, pl.ws.partial), pl.ws.partial_len, seg<uint32_t>(ws, pl.ws.dbase),
                       pl.ws.dblocks};
  return run_delta(a, s, st);
}

hipError_t launch_delta(const Plan& pl, const gs_params& cur, const gs_params& base, uint32_t mask, float tau,
                        uint32_t* out, void* ws, hipStream_t st) {
  DeltaArgs a;
  float* rows[6];
  group_rows(base, rows);
  set_groups(cur, rows, a.g);
  gs_codec raw[6];
  for (int g = 0; g < 6; ++g) raw[g] = gs_codec{GS_CODEC_RAW, 32, 1.0f, 0.0f, tau};
  a.c = codec_dev(raw, a.g.width);
  a.n = cur.n;
  a.mask = mask;
  a.hdr = 6;
  a.epoch = nullptr;
  a.out = out;
  return run_delta(pl, a, ws, st);
}

hipError_t launch_delta_encode(const Plan& pl, const gs_params& cur, const gs_params& base, const gs_codec* codecs,
                               uint32_t mask, const uint32_t* epoch, uint32_t* out, void* ws, hipStream_t st) {
  DeltaArgs a;
  float* rows[6];
  group_rows(base, rows);
  set_groups(cur, rows, a.g);
  a.c = codec_dev(codecs, a.g.width);
  a.n = cur.n;
  a.mask = mask;
  a.hdr = 9;
  a.epoch = epoch;
  a.out = out;
  return run_delta(pl, a, ws, st);
}

// ---- the delta encoder without a workspace ----------------------------------
// Scratch of gs_delta_encode_noalloc in a file-scope device array: each GPU
// that the library runs on holds its own copy until the process ends.  Its
// address is looked up once per device (noalloc_scratch_init, called by
// gs_create with the device current); host code uses only that address,
// never the array's name, which on the host is a stand-in and not a device
// address.
namespace {
constexpr int64_t kNaBlocks = kNoAllocMaxN / 256;
constexpr int64_t kNaPartial = (6 * kNaBlocks + kSortChunk - 1) / kSortChunk + 2;
constexpr size_t na_round(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kNaFlagsAt = 0;
constexpr size_t kNaCountAt = na_round(kNaFlagsAt + (size_t)kNoAllocMaxN);
constexpr size_t kNaPartialAt = na_round(kNaCountAt + (size_t)(6 * kNaBlocks) * 4);
constexpr size_t kNaBaseAt = na_round(kNaPartialAt + (size_t)kNaPartial * 4);
constexpr size_t kNaBytes = kNaBaseAt + 16 * 4;
static_assert(kNaCountAt % 256 == 0 && kNaPartialAt % 256 == 0 && kNaBaseAt % 256 == 0, "scratch alignment");
constexpr int kNaMaxDevices = 64;

void* g_scratch_ptr[kNaMaxDevices] = {};
}  // namespace

static __device__ __align__(256) uint8_t scratch[kNaBytes];

size_t noalloc_scratch_bytes() { return kNaBytes; }

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kNaMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

hipError_t launch_delta_encode_noalloc(int device, const gs_params& cur, const gs_params& base, const gs_codec* codecs,
                                       uint32_t mask, const uint32_t* epoch, uint32_t* out, hipStream_t st) {
  if (device < 0 || device >= kNaMaxDevices || !g_scratch_ptr[device]) return hipErrorNotInitialized;
  if (cur.n > kNoAllocMaxN) return hipErrorInvalidValue;
  char* p = static_cast<char*>(g_scratch_ptr[device]);
  const DeltaScratch s{reinterpret_cast<uint8_t*>(p + kNaFlagsAt), reinterpret_cast<uint32_t*>(p + kNaCountAt),
                       reinterpret_cast<uint32_t*>(p + kNaPartialAt), kNaPartial,
                       reinterpret_cast<uint32_t*>(p + kNaBaseAt), (int32_t)kNaBlocks};
  DeltaArgs a;
  float* rows[6];
  group_rows(base, rows);
  set_groups(cur, rows, a.g);
  a.c = codec_dev(codecs, a.g.width);
  a.n = cur.n;
  a.mask = mask;
  a.hdr = 9;
  a.epoch = epoch;
  a.out = out;
  return run_delta(a, s, st);
}

hipError_t launch_delta_apply(const gs_params& model, const gs_codec* codecs, const uint32_t* packet,
                              int64_t packet_words, const uint32_t* epoch, uint32_t* status, hipStream_t st) {
  ApplyArgs a;
  group_rows(model, a.grp);
  DeltaGroups g;
  set_groups(model, a.grp, g);
  for (int q = 0; q < 6; ++q) a.width[q] = g.width[q];
  a.c = codec_dev(codecs, a.width);
  a.n = model.n;
  a.pk = packet;
  a.pk_words = packet_words;
  a.epoch = epoch;
  a.status = status;
  hipError_t e = launch_fill_u32(status, 0u, 1, st);
  if (e != hipSuccess) return e;
  // rows of all groups together are at most 6 n; a grid-stride loop covers them
  const int64_t want = (model.n + 255) / 256;
  const unsigned blocks = (unsigned)(want < 1 ? 1 : (want > 2048 ? 2048 : want));
  hipLaunchKernelGGL(k_apply_check, dim3(blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_apply, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
