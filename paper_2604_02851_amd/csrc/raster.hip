// Front-to-back compositing per tile and its adjoint.
//
// One workgroup per tile, one thread per pixel.  The tile's list is consumed
// in batches of BATCH splat records staged in LDS (every pixel of the tile
// reads every record, so a record is fetched from HBM once per tile).  The
// forward pass stops a pixel once its transmittance would fall below 1e-4 and
// the whole workgroup once every pixel has stopped; it saves T_final, the
// contributor count and the last list position.  The backward pass walks the
// same list back to front from each pixel's last position, rebuilding the
// transmittance by division, and reduces each splat's screen-space gradient
// over the 64 pixels of a wavefront before one LDS atomic per wavefront and
// one global atomic per (tile, splat, field).
#include "internal.h"

namespace gs {
namespace {

struct CompArgs {
  const ViewInfo* views;
  const int32_t* tile_view;
  int32_t tile_begin;
  const uint2* ranges;
  const uint32_t* vals;
  const float4* rec;
  float* img;
  float* T;
  uint32_t* ncontrib;
  uint32_t* last;
  uint32_t cap;
  float bg0, bg1, bg2;
};

// Ranges are clamped to the key capacity so that a workspace whose lists were
// never built cannot send a read past the key buffers.
__device__ __forceinline__ uint2 clamp_range(uint2 rg, uint32_t cap) {
  rg.y = min(rg.y, cap);
  rg.x = min(rg.x, rg.y);
  return rg;
}

template <int TW, int TH, int BATCH>
__global__ __launch_bounds__(TW* TH) void k_composite(CompArgs a) {
  constexpr int NT = TW * TH;
  __shared__ float4 s_rec[BATCH * 3];
  const int t = a.tile_begin + blockIdx.x;
  const ViewInfo view = a.views[a.tile_view[t]];
  const int local = t - view.tile_base;
  const int ty = local / view.tiles_x, tx = local - ty * view.tiles_x;
  const int px = tx * TW + (int)(threadIdx.x % TW), py = ty * TH + (int)(threadIdx.x / TW);
  const bool inside = px < view.width && py < view.height;
  const uint2 rg = clamp_range(a.ranges[t], a.cap);
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  float T = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
  uint32_t n = 0, last = rg.x;
  bool done = !inside;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += BATCH) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t cnt = min((uint32_t)BATCH, rg.y - b0);
    for (uint32_t j = threadIdx.x; j < cnt; j += NT) {
      const uint32_t id = a.vals[b0 + j];
      s_rec[j * 3 + 0] = a.rec[(size_t)id * 3 + 0];
      s_rec[j * 3 + 1] = a.rec[(size_t)id * 3 + 1];
      s_rec[j * 3 + 2] = a.rec[(size_t)id * 3 + 2];
    }
    __syncthreads();
    if (!done) {
      for (uint32_t j = 0; j < cnt; ++j) {
        const SplatEval s = eval_splat(pxc, pyc, s_rec[j * 3], s_rec[j * 3 + 1]);
        if (!s.inside) continue;
        const float Tn = T * (1.f - s.alpha);
        if (Tn < kTMin) {
          done = true;
          break;
        }
        const float4 r2 = s_rec[j * 3 + 2];
        const float w = s.alpha * T;
        c0 = fmaf(r2.x, w, c0);
        c1 = fmaf(r2.y, w, c1);
        c2 = fmaf(r2.z, w, c2);
        T = Tn;
        ++n;
        last = b0 + j + 1;
      }
    }
  }
  if (inside) {
    const int64_t HW = (int64_t)view.width * view.height;
    const int64_t p = (int64_t)py * view.width + px;
    float* im = a.img + 3 * view.pix_off;
    im[p] = fmaf(T, a.bg0, c0);
    im[HW + p] = fmaf(T, a.bg1, c1);
    im[2 * HW + p] = fmaf(T, a.bg2, c2);
    a.T[view.pix_off + p] = T;
    a.ncontrib[view.pix_off + p] = n;
    a.last[view.pix_off + p] = last;
  }
}

struct BwdArgs {
  const ViewInfo* views;
  const int32_t* tile_view;
  int32_t tile_begin;
  const uint2* ranges;
  const uint32_t* vals;
  const float4* rec;
  const float* img;
  const float* T;
  const uint32_t* last;
  const float* up;
  int mode;
  int loss_mode;
  float* g2;
  float* loss;
  uint32_t cap;
  float bg0, bg1, bg2;
};

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <int TW, int TH, int BATCH>
__global__ __launch_bounds__(TW* TH) void k_composite_bwd(BwdArgs a) {
  constexpr int NT = TW * TH;
  __shared__ float4 s_rec[BATCH * 3];
  __shared__ uint32_t s_id[BATCH];
  __shared__ float s_g[BATCH * 9];
  __shared__ uint32_t s_max;
  const int t = a.tile_begin + blockIdx.x;
  const ViewInfo view = a.views[a.tile_view[t]];
  const int local = t - view.tile_base;
  const int ty = local / view.tiles_x, tx = local - ty * view.tiles_x;
  const int px = tx * TW + (int)(threadIdx.x % TW), py = ty * TH + (int)(threadIdx.x / TW);
  const bool inside = px < view.width && py < view.height;
  const uint2 rg = clamp_range(a.ranges[t], a.cap);
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) s_max = rg.x;
  __syncthreads();
  float G0 = 0.f, G1 = 0.f, G2 = 0.f, lossv = 0.f, T = 1.f;
  uint32_t my_last = rg.x;
  if (inside) {
    const int64_t HW = (int64_t)view.width * view.height;
    const int64_t p = (int64_t)py * view.width + px;
    const int64_t ib = 3 * view.pix_off + p;
    if (a.mode == 0) {
      G0 = a.up[ib];
      G1 = a.up[ib + HW];
      G2 = a.up[ib + 2 * HW];
    } else {
      const float wv = a.loss_mode == 1 ? 1.f / (3.f * (float)HW) : 1.f;
      const float d0 = a.img[ib] - a.up[ib];
      const float d1 = a.img[ib + HW] - a.up[ib + HW];
      const float d2 = a.img[ib + 2 * HW] - a.up[ib + 2 * HW];
      G0 = wv * (float)((d0 > 0.f) - (d0 < 0.f));
      G1 = wv * (float)((d1 > 0.f) - (d1 < 0.f));
      G2 = wv * (float)((d2 > 0.f) - (d2 < 0.f));
      lossv = wv * (fabsf(d0) + fabsf(d1) + fabsf(d2));
    }
    T = a.T[view.pix_off + p];
    my_last = min(max(a.last[view.pix_off + p], rg.x), rg.y);
    atomicMax(&s_max, my_last);
  }
  float S0 = a.bg0, S1 = a.bg1, S2 = a.bg2;
  __syncthreads();
  const uint32_t end_all = s_max;
  for (uint32_t b_end = end_all; b_end > rg.x;) {
    const uint32_t b_begin = (b_end - rg.x > (uint32_t)BATCH) ? b_end - BATCH : rg.x;
    const uint32_t cnt = b_end - b_begin;
    for (uint32_t j = threadIdx.x; j < cnt; j += NT) {
      const uint32_t id = a.vals[b_begin + j];
      s_id[j] = id;
      s_rec[j * 3 + 0] = a.rec[(size_t)id * 3 + 0];
      s_rec[j * 3 + 1] = a.rec[(size_t)id * 3 + 1];
      s_rec[j * 3 + 2] = a.rec[(size_t)id * 3 + 2];
    }
    for (uint32_t q = threadIdx.x; q < cnt * 9; q += NT) s_g[q] = 0.f;
    __syncthreads();
    for (int j = (int)cnt - 1; j >= 0; --j) {
      float g[9];
#pragma unroll
      for (int f = 0; f < 9; ++f) g[f] = 0.f;
      bool contrib = false;
      if (inside && b_begin + (uint32_t)j < my_last) {
        const float4 r0 = s_rec[j * 3], r1 = s_rec[j * 3 + 1];
        const SplatEval s = eval_splat(pxc, pyc, r0, r1);
        if (s.inside) {
          contrib = true;
          const float4 r2 = s_rec[j * 3 + 2];
          const float al = s.alpha;
          const float Tj = T / (1.f - al);
          const float at = al * Tj;
          g[6] = at * G0;
          g[7] = at * G1;
          g[8] = at * G2;
          const float dLda = Tj * ((r2.x - S0) * G0 + (r2.y - S1) * G1 + (r2.z - S2) * G2);
          S0 = fmaf(al, r2.x - S0, S0);
          S1 = fmaf(al, r2.y - S1, S1);
          S2 = fmaf(al, r2.z - S2, S2);
          T = Tj;
          if (!s.clamped) {
            const float dLdP = dLda * al;
            g[5] = dLda * s.G;
            const float ae = r1.x * s.e;
            g[0] = dLdP * ae;
            g[1] = dLdP * fmaf(ae, r1.y, r1.z * s.dy);
            g[2] = -0.5f * dLdP * s.dx * s.dx;
            g[3] = -dLdP * s.dx * s.dy;
            g[4] = -0.5f * dLdP * s.dy * s.dy;
          }
        }
      }
      if (__ballot(contrib) != 0ull) {
#pragma unroll
        for (int f = 0; f < 9; ++f) g[f] = wave_sum(g[f]);
        if (lane == 0) {
#pragma unroll
          for (int f = 0; f < 9; ++f) atomicAdd(&s_g[j * 9 + f], g[f]);
        }
      }
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < cnt * 9; q += NT) {
      const float v = s_g[q];
      if (v != 0.f) atomicAdd(&a.g2[(size_t)s_id[q / 9] * kG2Stride + (q % 9)], v);
    }
    __syncthreads();
    b_end = b_begin;
  }
  if (a.mode == 1) {
    lossv = wave_sum(lossv);
    if (lane == 0 && lossv != 0.f) atomicAdd(a.loss, lossv);
  }
}

template <int TW, int TH>
hipError_t comp_batch(int batch, dim3 grid, hipStream_t st, const CompArgs& a) {
  switch (batch) {
    case 32: hipLaunchKernelGGL((k_composite<TW, TH, 32>), grid, dim3(TW * TH), 0, st, a); break;
    case 64: hipLaunchKernelGGL((k_composite<TW, TH, 64>), grid, dim3(TW * TH), 0, st, a); break;
    case 128: hipLaunchKernelGGL((k_composite<TW, TH, 128>), grid, dim3(TW * TH), 0, st, a); break;
    case 256: hipLaunchKernelGGL((k_composite<TW, TH, 256>), grid, dim3(TW * TH), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TW, int TH>
hipError_t bwd_batch(int batch, dim3 grid, hipStream_t st, const BwdArgs& a) {
  switch (batch) {
    case 32: hipLaunchKernelGGL((k_composite_bwd<TW, TH, 32>), grid, dim3(TW * TH), 0, st, a); break;
    case 64: hipLaunchKernelGGL((k_composite_bwd<TW, TH, 64>), grid, dim3(TW * TH), 0, st, a); break;
    case 128: hipLaunchKernelGGL((k_composite_bwd<TW, TH, 128>), grid, dim3(TW * TH), 0, st, a); break;
    case 256: hipLaunchKernelGGL((k_composite_bwd<TW, TH, 256>), grid, dim3(TW * TH), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

void tile_span(const Plan& pl, int v0, int nv, int32_t* tb, int32_t* ntiles) {
  *tb = pl.views[v0].tile_base;
  const int32_t te = (v0 + nv < pl.n_views) ? pl.views[v0 + nv].tile_base : pl.total_tiles;
  *ntiles = te - *tb;
}

}  // namespace

bool sorted_values_in_b(const Plan& pl, int v0, int nv) {
  const int32_t tb = pl.views[v0].tile_base;
  const int32_t te = (v0 + nv < pl.n_views) ? pl.views[v0 + nv].tile_base : pl.total_tiles;
  int bits = 0;
  while ((1ll << bits) < (int64_t)(te - tb)) ++bits;
  const int passes = bits == 0 ? 1 : (bits + 7) / 8;
  return (passes & 1) != 0;
}

hipError_t launch_composite(const Plan& pl, int v0, int nv, void* ws, float* img, float* T, uint32_t* nc,
                            hipStream_t st) {
  CompArgs a;
  a.views = pl.d_views;
  a.tile_view = pl.d_tile_view;
  int32_t ntiles;
  tile_span(pl, v0, nv, &a.tile_begin, &ntiles);
  a.ranges = seg<uint2>(ws, pl.ws.ranges);
  a.vals = seg<uint32_t>(ws, sorted_values_in_b(pl, v0, nv) ? pl.ws.vals_b : pl.ws.vals_a);
  a.rec = seg<float4>(ws, pl.ws.rec);
  a.img = img;
  a.T = T;
  a.ncontrib = nc;
  a.last = seg<uint32_t>(ws, pl.ws.last);
  a.cap = (uint32_t)pl.cap;
  a.bg0 = pl.bg[0];
  a.bg1 = pl.bg[1];
  a.bg2 = pl.bg[2];
  if (ntiles <= 0) return hipSuccess;
  const dim3 grid(ntiles);
  const int tw = pl.tile_w, th = pl.tile_h, b = pl.batch_depth;
  if (tw == 8 && th == 8) return comp_batch<8, 8>(b, grid, st, a);
  if (tw == 16 && th == 8) return comp_batch<16, 8>(b, grid, st, a);
  if (tw == 16 && th == 16) return comp_batch<16, 16>(b, grid, st, a);
  if (tw == 32 && th == 16) return comp_batch<32, 16>(b, grid, st, a);
  if (tw == 32 && th == 32) return comp_batch<32, 32>(b, grid, st, a);
  return hipErrorInvalidValue;
}

hipError_t launch_composite_bwd(const Plan& pl, int v0, int nv, void* ws, const float* img, const float* T,
                                const float* up, int mode, float* loss, hipStream_t st) {
  BwdArgs a;
  a.views = pl.d_views;
  a.tile_view = pl.d_tile_view;
  int32_t ntiles;
  tile_span(pl, v0, nv, &a.tile_begin, &ntiles);
  a.ranges = seg<uint2>(ws, pl.ws.ranges);
  a.vals = seg<uint32_t>(ws, sorted_values_in_b(pl, v0, nv) ? pl.ws.vals_b : pl.ws.vals_a);
  a.rec = seg<float4>(ws, pl.ws.rec);
  a.img = img;
  a.T = T;
  a.last = seg<uint32_t>(ws, pl.ws.last);
  a.up = up;
  a.mode = mode;
  a.loss_mode = pl.loss_mode;
  a.g2 = seg<float>(ws, pl.ws.g2);
  a.loss = loss;
  a.cap = (uint32_t)pl.cap;
  a.bg0 = pl.bg[0];
  a.bg1 = pl.bg[1];
  a.bg2 = pl.bg[2];
  if (ntiles <= 0) return hipSuccess;
  const dim3 grid(ntiles);
  const int tw = pl.tile_w, th = pl.tile_h, b = pl.batch_depth;
  if (tw == 8 && th == 8) return bwd_batch<8, 8>(b, grid, st, a);
  if (tw == 16 && th == 8) return bwd_batch<16, 8>(b, grid, st, a);
  if (tw == 16 && th == 16) return bwd_batch<16, 16>(b, grid, st, a);
  if (tw == 32 && th == 16) return bwd_batch<32, 16>(b, grid, st, a);
  if (tw == 32 && th == 32) return bwd_batch<32, 32>(b, grid, st, a);
  return hipErrorInvalidValue;
}

}  // namespace gs
