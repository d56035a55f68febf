// Front-to-back compositing per tile and its adjoint.
//
// One workgroup per tile.  Each thread owns PPT pixels of the tile; each
// wavefront owns an SW x WROWS sub-tile (a band of whole rows when SW = TW,
// squarer blocks otherwise, which a splat's box misses more often).  The
// tile's list is consumed in batches of BATCH splat records staged in LDS:
// every pixel of the tile reads every record, so a record leaves HBM once per
// tile.  Before evaluating a splat, a wavefront tests the splat's 3-sigma box
// against its own sub-tile and skips it as a whole when they do not meet; the box
// is widened so that it contains every pixel whose FP32 ellipse test can
// pass, so skipping never changes a result.
//
// Forward: stops a pixel once its transmittance would fall below 1e-4 and
// the workgroup once every pixel has stopped; saves T_final, the contributor
// count and the last composited list position.
// The forward stores each list entry's strip bits (which wavefront pixel
// slots its splat may reach), and the backward stages them with the records
// instead of testing the strips again: it only walks list positions before
// the tile's largest last position, all of which the forward has staged.
// Backward: walks the list back to front from each pixel's last position,
// rebuilding the transmittance by division (FP32 reciprocal); a splat's screen-space
// gradient is summed over the thread's pixels in registers, then over the
// wavefront with DPP row operations, then over the wavefronts of the tile in
// LDS, and finally added once per (tile, splat, field) to the global
// accumulator.
#include "internal.h"

namespace gs {
namespace {

// A wavefront owns an SW x WROWS sub-tile; lane l covers column l % SW and
// rows l / SW + q * LROWS for q < PPT.
template <int TW, int TH, int PPT, int SW>
struct Geom {
  static constexpr int NT = TW * TH / PPT;       // threads per workgroup
  static constexpr int NWAVES = NT / 64;
  static constexpr int LROWS = 64 / SW;          // sub-tile rows spanned by one pixel slot of a wave
  static constexpr int WROWS = LROWS * PPT;      // sub-tile height
  static constexpr int WPR = TW / SW;            // wavefronts per tile row
  static_assert(NT % 64 == 0 && 64 % SW == 0 && TW % SW == 0 && TH % WROWS == 0 &&
                    NWAVES == WPR * (TH / WROWS),
                "tile / pixels-per-thread / wave shape");
  static_assert(NWAVES * PPT <= 31, "one strip bit per wavefront and pixel slot, below the active bit");
  // strip bits of the first half of the wavefronts (two threads share a
  // splat's strip tests when the tile has several wavefronts)
  static constexpr int HALF_BITS = (NWAVES >= 2 ? NWAVES / 2 : NWAVES) * PPT;
  static_assert(HALF_BITS <= 16, "each half of the strip bits fits 16 bits");
};

// Workgroup -> tile.  Schedule 0: row-major tile order.  Schedule 1: each
// XCD (workgroups are dealt to the 8 XCDs round-robin) receives a contiguous
// run of tiles, so neighbouring tiles share splat records in that XCD's L2.
__device__ __forceinline__ uint32_t tile_of_block(uint32_t b, uint32_t ntiles, int schedule) {
  if (schedule == 0) return b;
  const uint32_t xcd = b & 7u, k = b >> 3;
  return xcd * (ntiles >> 3) + min(xcd, ntiles & 7u) + k;
}

// Culling of a splat against the pixel-centre rectangle [x0, x1] x [y0, y1]:
// a lower bound of q = a (dx + r dy)^2 + s dy^2 (P = -q/2) over the
// rectangle.  q is convex, so its minimum is 0 at the centre when the centre
// lies inside, else it lies on an edge: along a horizontal edge (dy fixed) at
// dx = -r dy, along a vertical edge (dx fixed) at dy = -a r dx / (a r^2 + s),
// each clamped to the edge.  A pixel of the rectangle can pass the 3-sigma
// test (q <= 9) only if this minimum is <= 9; the threshold is widened by
// 0.1% + 0.01 for FP32 rounding of both evaluations, so culling never
// changes a result.
constexpr float kCullQ = 9.0f * 1.001f + 0.01f;
constexpr uint32_t kActiveBit = 0x80000000u;   // in the per-splat strip mask (at most 31 strip bits)

__device__ __forceinline__ float rect_qmin(float a, float r, float s, float inv, float cu, float cw, float x0,
                                           float x1, float y0, float y1) {
  if (cu >= x0 && cu <= x1 && cw >= y0 && cw <= y1) return 0.f;
  float best = INFINITY;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float dy = (k ? y1 : y0) - cw;
    const float xs = fminf(fmaxf(cu - r * dy, x0), x1);
    const float e = (xs - cu) + r * dy;
    best = fminf(best, a * e * e + s * dy * dy);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float dx = (k ? x1 : x0) - cu;
    const float dys = fminf(fmaxf(-a * r * dx * inv, y0 - cw), y1 - cw);
    const float e = dx + r * dys;
    best = fminf(best, a * e * e + s * dys * dys);
  }
  return best;
}

// Bit (w * PPT + q) set when the splat may reach a pixel of pixel slot q of
// wavefront w (a strip of SW x LROWS pixels of the tile whose top-left pixel
// is (tx0, ty0)), for the wavefronts w in [w0, w1).
template <class G, int SW, int PPT>
__device__ __forceinline__ uint32_t splat_strip_mask(const float4& r0, const float4& r1, int tx0, int ty0, int w0,
                                                     int w1) {
  const float cu = r0.x + r0.z, cw = r0.y + r0.w;
  const float a = r1.x, r = r1.y, s = r1.z;
  const float inv = 1.f / fmaf(a * r, r, s);
  uint32_t m = 0;
  // not unrolled: the compositing kernels' register budget is set by their
  // main loops, and unrolled strip tests would raise it
#pragma unroll 1
  for (int w = w0; w < w1; ++w) {
    const float x0 = (float)(tx0 + (w % G::WPR) * SW) + 0.5f, x1 = x0 + (float)(SW - 1);
#pragma unroll 1
    for (int q = 0; q < PPT; ++q) {
      const float y0 = (float)(ty0 + (w / G::WPR) * G::WROWS + q * G::LROWS) + 0.5f;
      const float y1 = y0 + (float)(G::LROWS - 1);
      if (!(rect_qmin(a, r, s, inv, cu, cw, x0, x1, y0, y1) > kCullQ)) m |= 1u << (w * PPT + q);
    }
  }
  return m;
}

// Largest value over the wavefront's 64 lanes (every lane receives it).
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
  return v;
}

// The strip bits of staged splat j (the halves' words combined).
template <uint32_t H>
__device__ __forceinline__ uint32_t strip_word(const uint32_t* m, uint32_t j) {
  return H == 2 ? (m[2 * j] | m[2 * j + 1]) : m[j];
}

// Ranges are clamped to the key capacity so that a workspace whose lists were
// never built cannot send a read past the key buffers.
__device__ __forceinline__ uint2 clamp_range(uint2 rg, uint32_t cap) {
  rg.y = min(rg.y, cap);
  rg.x = min(rg.x, rg.y);
  return rg;
}

// Sum over the 64 lanes: inclusive scan inside each row of 16 lanes, then the
// row totals are carried across rows; lane 63 ends with the total.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
  const int o = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, false);
  return v + __builtin_bit_cast(float, o);
}

__device__ __forceinline__ float wave_total_lane63(float v) {
  v = dpp_add<0x111, 0xf>(v);   // row_shr:1
  v = dpp_add<0x112, 0xf>(v);   // row_shr:2
  v = dpp_add<0x114, 0xf>(v);   // row_shr:4
  v = dpp_add<0x118, 0xf>(v);   // row_shr:8
  v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

template <int CTRL>
__device__ __forceinline__ float dpp_get(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

// a + b after exchanging the upper 32 lanes of a with the lower 32 lanes of b
// (resp. the odd 16-lane rows of a with the even rows of b): each result lane
// holds a partial sum of one of the two inputs.  Written as inline assembly
// because the compiler's builtin for these gfx950 swaps loses one of its two
// results here; the s_nop gives the two wait states a cross-lane read needs
// after a VALU write of its operands.
__device__ __forceinline__ float swap32_sum(float a, float b) {
  asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
  return a + b;
}
__device__ __forceinline__ float swap16_sum(float a, float b) {
  asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(a), "+v"(b));
  return a + b;
}

// Transposed reduction of eight per-lane values over the wavefront: two
// levels of lane-group swaps halve the values per lane while folding lanes,
// then a row mirror merges the last pair and three DPP steps finish the
// 8-lane groups.  Afterwards every lane of 8-lane group k holds the wave
// total of one field; which field is fixed by the lane position and found
// once per kernel by reducing one-hot tags (reduce8_field).
__device__ __forceinline__ float reduce8(const float* g, bool lo8) {
  const float w0 = swap32_sum(g[0], g[1]);
  const float w1 = swap32_sum(g[2], g[3]);
  const float w2 = swap32_sum(g[4], g[5]);
  const float w3 = swap32_sum(g[6], g[7]);
  const float x0 = swap16_sum(w0, w1);
  const float x1 = swap16_sum(w2, w3);
  const float s = lo8 ? x0 : x1, z = lo8 ? x1 : x0;
  float y = s + dpp_get<0x140>(z);   // row_mirror: lane i of a row reads lane 15 - i
  y += dpp_get<0x141>(y);            // row_half_mirror: lane i of 8 reads lane 7 - i
  y += dpp_get<0x4e>(y);             // quad_perm [2,3,0,1]
  y += dpp_get<0xb1>(y);             // quad_perm [1,0,3,2]
  return y;
}

// Field whose total reduce8 leaves in this lane (exact: sums of 0 and a
// single power of two).
__device__ __forceinline__ int reduce8_field(int lane, bool lo8) {
  float tag[8];
#pragma unroll
  for (int f = 0; f < 8; ++f) tag[f] = lane == 0 ? (float)(1 << f) : 0.f;
  const uint32_t bits = (uint32_t)reduce8(tag, lo8);
  return __builtin_ctz(bits | 256u) & 7;
}

// Work queue of the persistent compositing kernels.  head[0] counts the
// positions handed out, head[1] the workgroups that found the queue empty;
// the last of those resets both, so that the next launch starts from zero
// (they start at zero when the workspace is initialised).  Position k is
// tile order[k] of the call (longest lists first, schedule 3) or tile k.
struct TileQueue {
  uint32_t* head;
  const uint32_t* order;
};
constexpr uint32_t kQueueDone = 0xffffffffu;

__device__ __forceinline__ uint32_t queue_next(const TileQueue& q, uint32_t ntiles, uint32_t* s_next) {
  // every thread is done with the previous tile (its LDS and its position)
  __syncthreads();
  if (threadIdx.x == 0) *s_next = atomicAdd(q.head, 1u);
  __syncthreads();
  // uniform across the workgroup: kept in scalar registers, like blockIdx
  const uint32_t k = __builtin_amdgcn_readfirstlane(*s_next);
  if (k >= ntiles) return kQueueDone;
  return q.order ? __builtin_amdgcn_readfirstlane(q.order[k]) : k;
}

__device__ __forceinline__ void queue_exit(const TileQueue& q) {
  if (threadIdx.x == 0) {
    // this workgroup's last atomicAdd on head[0] has returned: once every
    // workgroup has counted itself here, nobody reads head[0] again
    if (atomicAdd(q.head + 1, 1u) == gridDim.x - 1u) {
      atomicExch(q.head, 0u);
      atomicExch(q.head + 1, 0u);
    }
  }
}

struct CompArgs {
  const ViewInfo* views;
  const int32_t* tile_view;
  int32_t tile_begin;
  int32_t ntiles;
  int32_t schedule;
  const uint2* ranges;
  const uint32_t* vals;
  const float4* rec;
  float* img;
  float* T;
  uint32_t* ncontrib;
  uint32_t* last;
  uint16_t* strips;   // per list position, two 16-bit halves: the staged splat's strip bits
  uint32_t cap;
  float bg0, bg1, bg2;
  TileQueue q;
};

// LDS of one compositing workgroup (forward).
template <int BATCH, uint32_t H>
struct FwdShared {
  float4 rec[BATCH * 3];
  uint32_t mask[BATCH * H];
};

// Forward compositing of tile `slot` of the call by the whole workgroup.
template <int TW, int TH, int PPT, int SW, int BATCH>
__device__ __forceinline__ void composite_tile(const CompArgs& a, uint32_t slot,
                                               FwdShared<BATCH, (Geom<TW, TH, PPT, SW>::NWAVES >= 2 ? 2u : 1u)>& sm) {
  using G = Geom<TW, TH, PPT, SW>;
  constexpr uint32_t kHalves = G::NWAVES >= 2 ? 2 : 1;
  float4* s_rec = sm.rec;
  uint32_t* s_mask = sm.mask;
  const int t = a.tile_begin + (int)slot;
  const ViewInfo view = a.views[a.tile_view[t]];
  const int local = t - view.tile_base;
  const int ty = local / view.tiles_x, tx = local - ty * view.tiles_x;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x0 = tx * TW + (wave % G::WPR) * SW, y0 = ty * TH + (wave / G::WPR) * G::WROWS;
  const int px = x0 + lane % SW, py0 = y0 + lane / SW;
  const uint2 rg = clamp_range(a.ranges[t], a.cap);
  const float pxc = (float)px + 0.5f;
  // T > 0 while the pixel composites; a pixel that stopped (or lies outside
  // the image) carries -T, so that one compare answers both questions
  float T[PPT], c0[PPT], c1[PPT], c2[PPT];
  uint32_t n[PPT], last[PPT];
  bool live = false;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const bool inside = px < view.width && py0 + q * G::LROWS < view.height;
    T[q] = inside ? 1.f : -1.f;
    c0[q] = c1[q] = c2[q] = 0.f;
    n[q] = 0;
    last[q] = rg.x;
    live |= inside;
  }
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += BATCH) {
    if (__syncthreads_count(live) == 0) break;
    const uint32_t cnt = min((uint32_t)BATCH, rg.y - b0);
    // two threads per splat share its strip tests (half the wavefronts each)
    for (uint32_t u = threadIdx.x; u < cnt * kHalves; u += G::NT) {
      const uint32_t j = u / kHalves, h = u % kHalves;
      const uint32_t id = a.vals[b0 + j];
      const float4 r0 = a.rec[(size_t)id * 3 + 0], r1 = a.rec[(size_t)id * 3 + 1];
      if (h == 0) {
        s_rec[j * 3 + 0] = r0;
        s_rec[j * 3 + 1] = staged_conic(r1);
        s_rec[j * 3 + 2] = a.rec[(size_t)id * 3 + 2];
      }
      const uint32_t m = splat_strip_mask<G, SW, PPT>(r0, r1, tx * TW, ty * TH, (int)h * G::NWAVES / kHalves,
                                                      ((int)h + 1) * G::NWAVES / kHalves);
      s_mask[u] = m;
      // for the adjoint: each half's bits, shifted to bit 0, in its own 16-bit slot
      a.strips[2 * (b0 + j) + h] = (uint16_t)(m >> (h * G::HALF_BITS));
      if (kHalves == 1) a.strips[2 * (b0 + j) + 1] = 0;
    }
    __syncthreads();
    // uniform: the splat walk below needs every lane (lane l reads splat
    // base + l's strip word); lanes that stopped take nothing, as their T < 0
    if (__ballot(live) != 0ull) {
      // pixel slots whose lanes have all stopped skip the batch (uniform)
      uint32_t qlive = 0u;
#pragma unroll
      for (int q = 0; q < PPT; ++q) qlive |= __ballot(T[q] > 0.f) != 0ull ? 1u << q : 0u;
      qlive = __builtin_amdgcn_readfirstlane(qlive);
      // 64 splats at a time: lane l reads the strip word of splat base + l, and
      // the wavefront then visits only the splats that touch one of its live strips
      for (uint32_t base = 0; base < cnt; base += 64) {
       const uint32_t jl = base + (uint32_t)lane;
       const uint32_t mw = jl < cnt ? strip_word<kHalves>(s_mask, jl) : 0u;
       uint64_t pend = __ballot(((mw >> (wave * PPT)) & qlive) != 0u);
       while (pend != 0ull) {
        const int l = __builtin_ctzll(pend);
        pend &= pend - 1ull;
        const uint32_t j = base + (uint32_t)l;
        const uint32_t qb = ((uint32_t)__builtin_amdgcn_readlane((int)mw, l) >> (wave * PPT)) & qlive;
        const float4 r0 = s_rec[j * 3], r1 = s_rec[j * 3 + 1], r2 = s_rec[j * 3 + 2];
        const uint32_t pos1 = b0 + j + 1;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          if (!((qb >> q) & 1u)) continue;   // uniform: the splat misses this pixel slot's strip
          const float pyc = (float)(py0 + q * G::LROWS) + 0.5f;
          const SplatGeom sg = splat_power(pxc, pyc, r0, r1);
          const bool cand = T[q] > 0.f && sg.P >= kCutoff2;
          if (__ballot(cand) == 0ull) continue;   // uniform: no lane of this row slot is near the splat
          float Gs, al;
          bool clamped;
          const bool take = splat_alpha(sg.P, r1.w, Gs, al, clamped) && cand;
          // predicated from here on: no divergent branches in the hot loop
          const float Tn = T[q] * (1.f - al);
          const bool stop = take && Tn < kTMin;
          const bool comp = take && !stop;
          const float w = comp ? al * T[q] : 0.f;
          c0[q] = fmaf(r2.x, w, c0[q]);
          c1[q] = fmaf(r2.y, w, c1[q]);
          c2[q] = fmaf(r2.z, w, c2[q]);
          T[q] = comp ? Tn : (stop ? -T[q] : T[q]);
          n[q] += comp ? 1u : 0u;
          last[q] = comp ? pos1 : last[q];
        }
       }
      }
      live = false;
#pragma unroll
      for (int q = 0; q < PPT; ++q) live |= T[q] > 0.f;
    }
  }
  const int64_t HW = (int64_t)view.width * view.height;
  float* im = a.img + 3 * view.pix_off;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int py = py0 + q * G::LROWS;
    if (px < view.width && py < view.height) {
      const int64_t p = (int64_t)py * view.width + px;
      const float Tf = fabsf(T[q]);
      im[p] = fmaf(Tf, a.bg0, c0[q]);
      im[HW + p] = fmaf(Tf, a.bg1, c1[q]);
      im[2 * HW + p] = fmaf(Tf, a.bg2, c2[q]);
      a.T[view.pix_off + p] = Tf;
      a.ncontrib[view.pix_off + p] = n[q];
      a.last[view.pix_off + p] = last[q];
    }
  }
}

// One workgroup per tile (schedules 0 and 1).  Held to seven wavefronts per
// SIMD: the stores of the strip bits would otherwise cost the compiler the
// few registers that take it to six.
template <int TW, int TH, int PPT, int SW, int BATCH>
__global__ __launch_bounds__(TW* TH / PPT) __attribute__((amdgpu_waves_per_eu(7))) void k_composite(CompArgs a) {
  __shared__ FwdShared<BATCH, (Geom<TW, TH, PPT, SW>::NWAVES >= 2 ? 2u : 1u)> sm;
  composite_tile<TW, TH, PPT, SW, BATCH>(a, tile_of_block(blockIdx.x, (uint32_t)a.ntiles, a.schedule), sm);
}

// Persistent (schedules 2 and 3): as many workgroups as fit on the chip at
// once, each taking the call's tiles from the work queue until it is empty.
// The loop around the tile body costs the compiler a few registers; held to
// the grid kernel's seven wavefronts per SIMD (a few bytes spilled) it
// measured faster than at six.
template <int TW, int TH, int PPT, int SW, int BATCH>
__global__ __launch_bounds__(TW* TH / PPT) __attribute__((amdgpu_waves_per_eu(7))) void k_composite_persistent(
    CompArgs a) {
  __shared__ FwdShared<BATCH, (Geom<TW, TH, PPT, SW>::NWAVES >= 2 ? 2u : 1u)> sm;
  __shared__ uint32_t s_next;
  for (;;) {
    const uint32_t slot = queue_next(a.q, (uint32_t)a.ntiles, &s_next);
    if (slot == kQueueDone) break;
    composite_tile<TW, TH, PPT, SW, BATCH>(a, slot, sm);
  }
  queue_exit(a.q);
}

struct BwdArgs {
  const ViewInfo* views;
  const int32_t* tile_view;
  int32_t tile_begin;
  int32_t ntiles;
  int32_t schedule;
  const uint2* ranges;
  const uint32_t* vals;
  const float4* rec;
  const float* img;
  const float* T;
  const uint32_t* last;
  const float* up;
  const uint32_t* strips;   // per list position: the forward's two 16-bit halves of the strip bits
  int mode;
  int loss_mode;
  float* g2;           // field f of pair o at g2[f * g2_plane + o]
  size_t g2_plane;
  float* loss;
  uint32_t cap;
  float bg0, bg1, bg2;
  uint32_t n_gauss;    // Gaussians per view in the value index v * n_gauss + i
  uint32_t n_active;   // Gaussians i < n_active are trainable; the rest are frozen
  TileQueue q;
};

// LDS of one compositing workgroup (adjoint).
template <int BATCH, bool MW>
struct BwdShared {
  float4 rec[BATCH * 3];
  uint32_t mask[BATCH];
  uint32_t id[BATCH];
  float g[MW ? BATCH * 9 : 1];   // the batch's splat sums over the tile's wavefronts
  uint32_t max_last;
};

// Adjoint of the compositing of one pixel, walked back to front from the
// pixel's last composited splat (Sj = colour arriving from behind splat j,
// background included; T rebuilt from T_final by division):
//   T_j = T_{j+1} / (1 - alpha_j)
//   d out / d col_j   = alpha_j T_j
//   d out / d alpha_j = T_j (col_j - S_j),   S_{j-1} = alpha_j col_j + (1 - alpha_j) S_j
// Only the projection SG_j = S_j . G of S onto the pixel's upstream gradient
// G enters the adjoint, so one scalar per pixel is carried back:
//   d L / d alpha_j = T_j (col_j . G - SG_j),   SG_{j-1} = SG_j + alpha_j (col_j . G - SG_j).
// The division chain runs in FP32 with the hardware reciprocal: each step adds
// at most about 4 units of 2^-24 to T_j's relative error (reciprocal, product,
// and 1 - alpha), which stays inside the same E_p = sum 1/(1 - alpha) bound
// as the forward product's own rounding.
template <int TW, int TH, int PPT, int SW, int BATCH>
using BwdSharedOf = BwdShared<BATCH, (Geom<TW, TH, PPT, SW>::NWAVES > 1)>;

// Adjoint of the compositing of tile `slot` of the call by the whole workgroup.
template <int TW, int TH, int PPT, int SW, int BATCH>
__device__ __forceinline__ void composite_bwd_tile(const BwdArgs& a, uint32_t slot, BwdSharedOf<TW, TH, PPT, SW, BATCH>& sm) {
  using G = Geom<TW, TH, PPT, SW>;
  constexpr bool kMultiWave = G::NWAVES > 1;
  float4* s_rec = sm.rec;
  uint32_t* s_mask = sm.mask;
  uint32_t* s_id = sm.id;
  float* s_g = sm.g;
  uint32_t& s_max = sm.max_last;
  const int t = a.tile_begin + (int)slot;
  const ViewInfo view = a.views[a.tile_view[t]];
  const int local = t - view.tile_base;
  const int ty = local / view.tiles_x, tx = local - ty * view.tiles_x;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x0 = tx * TW + (wave % G::WPR) * SW, y0 = ty * TH + (wave / G::WPR) * G::WROWS;
  const int px = x0 + lane % SW, py0 = y0 + lane / SW;
  const uint2 rg = clamp_range(a.ranges[t], a.cap);
  const float pxc = (float)px + 0.5f;
  const int64_t HW = (int64_t)view.width * view.height;
  const float wv = a.loss_mode == 1 ? 1.f / (3.f * (float)HW) : 1.f;
  const bool lo8 = (lane & 8) == 0;
  const int my_field = reduce8_field(lane, lo8);
  const bool writer = (lane & 7) == 0;
  // constant factors left out of the per-pixel sums: fields 0, 1 were summed
  // with the staged conic, which carries -log2(e)/2 (undone by -2 ln 2, one
  // rounding of the total), fields 2-4 without d P / d conic's factors -1/2,
  // -1, -1/2 (powers of two, exact)
  constexpr float kMinus2Ln2 = -1.38629436111989061f;
  const float restore = my_field < 2 ? kMinus2Ln2 : my_field == 3 ? -1.f : my_field < 5 ? -0.5f : 1.f;
  if (threadIdx.x == 0) s_max = rg.x;
  __syncthreads();
  float G0[PPT], G1[PPT], G2[PPT], SG[PPT];
  float T[PPT];
  uint32_t last[PPT];
  float lossv = 0.f;
  uint32_t my_max = rg.x;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    G0[q] = G1[q] = G2[q] = 0.f;
    T[q] = 1.f;
    last[q] = rg.x;
    const int py = py0 + q * G::LROWS;
    if (px < view.width && py < view.height) {
      const int64_t p = (int64_t)py * view.width + px;
      const int64_t ib = 3 * view.pix_off + p;
      if (a.mode == 0) {
        G0[q] = a.up[ib];
        G1[q] = a.up[ib + HW];
        G2[q] = a.up[ib + 2 * HW];
      } else {
        const float d0 = a.img[ib] - a.up[ib];
        const float d1 = a.img[ib + HW] - a.up[ib + HW];
        const float d2 = a.img[ib + 2 * HW] - a.up[ib + 2 * HW];
        G0[q] = wv * (float)((d0 > 0.f) - (d0 < 0.f));
        G1[q] = wv * (float)((d1 > 0.f) - (d1 < 0.f));
        G2[q] = wv * (float)((d2 > 0.f) - (d2 < 0.f));
        lossv += wv * (fabsf(d0) + fabsf(d1) + fabsf(d2));
      }
      T[q] = a.T[view.pix_off + p];
      last[q] = min(max(a.last[view.pix_off + p], rg.x), rg.y);
      my_max = max(my_max, last[q]);
    }
    SG[q] = fmaf(a.bg2, G2[q], fmaf(a.bg1, G1[q], a.bg0 * G0[q]));   // the background behind all splats
  }
  atomicMax(&s_max, my_max);
  // per pixel slot, the wavefront's largest last position: list entries at or
  // past it reach no lane of that slot, so the slot skips them outright
  uint32_t qlast[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) qlast[q] = __builtin_amdgcn_readfirstlane(wave_max_u32(last[q]));
  uint32_t wlast = qlast[0];
#pragma unroll
  for (int q = 1; q < PPT; ++q) wlast = max(wlast, qlast[q]);
  __syncthreads();
  const uint32_t end_all = s_max;
  for (uint32_t b_end = end_all; b_end > rg.x;) {
    const uint32_t b_begin = (b_end - rg.x > (uint32_t)BATCH) ? b_end - BATCH : rg.x;
    const uint32_t cnt = b_end - b_begin;
    // records and the forward's strip bits; bit 31: the splat's Gaussian is
    // trainable (frozen ones still shape T and S)
    for (uint32_t j = threadIdx.x; j < cnt; j += G::NT) {
      const uint32_t id = a.vals[b_begin + j];
      s_id[j] = id;
      s_rec[j * 3 + 0] = a.rec[(size_t)id * 3 + 0];
      s_rec[j * 3 + 1] = staged_conic(a.rec[(size_t)id * 3 + 1]);
      s_rec[j * 3 + 2] = a.rec[(size_t)id * 3 + 2];
      const uint32_t h2 = a.strips[b_begin + j];
      s_mask[j] = (h2 & 0xffffu) | ((h2 >> 16) << G::HALF_BITS) | (id % a.n_gauss < a.n_active ? kActiveBit : 0u);
    }
    if (kMultiWave)
      for (uint32_t q = threadIdx.x; q < cnt * 9; q += G::NT) s_g[q] = 0.f;
    __syncthreads();
    // the wavefront starts at its own last position within the batch
    const int j_hi = wlast > b_begin ? (int)min(cnt, wlast - b_begin) - 1 : -1;
    // 64 splats at a time: lane l reads the strip word of splat base - l, and
    // the wavefront then visits only the splats that touch one of its strips
    for (int base = j_hi; base >= 0; base -= 64) {
     const int jl = base - lane;
     const uint32_t mw = jl >= 0 ? s_mask[jl] : 0u;
     uint64_t pend = __ballot(((mw >> (wave * PPT)) & ((1u << PPT) - 1u)) != 0u);
     while (pend != 0ull) {
      const int l = __builtin_ctzll(pend);
      pend &= pend - 1ull;
      const int j = base - l;
      const uint32_t mword = (uint32_t)__builtin_amdgcn_readlane((int)mw, l);
      const uint32_t qb = (mword >> (wave * PPT)) & ((1u << PPT) - 1u);
      const bool act = (mword & kActiveBit) != 0u;
      const uint32_t pos = b_begin + (uint32_t)j;
      const float4 r0 = s_rec[j * 3], r1 = s_rec[j * 3 + 1];
      const float4 r2 = s_rec[j * 3 + 2];
      float g[9];
#pragma unroll
      for (int f = 0; f < 9; ++f) g[f] = 0.f;
      float contrib = 0.f;   // > 0 once the lane took the splat at one of its pixels
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        // uniform: the splat misses this pixel slot's strip, or lies behind
        // every lane's last composited splat
        if (!((qb >> q) & 1u) || pos >= qlast[q]) continue;
        const float pyc = (float)(py0 + q * G::LROWS) + 0.5f;
        const SplatGeom sg = splat_power(pxc, pyc, r0, r1);
        const bool cand = pos < last[q] && sg.P >= kCutoff2;
        if (__ballot(cand) == 0ull) continue;   // uniform
        float Gs, al;
        bool clamped;
        const bool take = splat_alpha(sg.P, r1.w, Gs, al, clamped) && cand;
        // predicated from here on: a lane that does not take the splat runs
        // with alpha 0, which leaves its S unchanged and adds zeros (staged
        // records are finite, so 0 times any product is 0).  A frozen splat
        // runs the same arithmetic (its sums are dropped below): a second,
        // gradient-free copy of this loop costs more registers than the
        // work it would save.
        const float alt = take ? al : 0.f;
        contrib += alt;
        const float Tj = T[q] * __builtin_amdgcn_rcpf(1.f - alt);
        T[q] = take ? Tj : T[q];
        const float at = alt * Tj;
        g[6] = fmaf(at, G0[q], g[6]);
        g[7] = fmaf(at, G1[q], g[7]);
        g[8] = fmaf(at, G2[q], g[8]);
        const float diff = fmaf(r2.z, G2[q], fmaf(r2.y, G1[q], r2.x * G0[q])) - SG[q];
        // the clamp cuts alpha off from opacity and power
        const float dLda = (take && !clamped) ? Tj * diff : 0.f;
        SG[q] = fmaf(alt, diff, SG[q]);
        const float dLdP = dLda * alt;
        g[5] = fmaf(dLda, Gs, g[5]);
        // with the staged conic, fields 0 and 1 collect -log2(e)/2 of their sums
        const float ae = r1.x * sg.e;
        g[0] = fmaf(dLdP, ae, g[0]);
        g[1] = fmaf(dLdP, fmaf(ae, r1.y, r1.z * sg.dy), g[1]);
        // conic fields without their constant factors -1/2, -1, -1/2 (also
        // restored exactly after the reduction)
        const float tx_ = dLdP * sg.dx, ty_ = dLdP * sg.dy;
        g[2] = fmaf(tx_, sg.dx, g[2]);
        g[3] = fmaf(tx_, sg.dy, g[3]);
        g[4] = fmaf(ty_, sg.dy, g[4]);
      }
      if (!act || __ballot(contrib > 0.f) == 0ull) continue;
      const float tot8 = reduce8(g, lo8) * restore;
      const float tot9 = wave_total_lane63(g[8]);
      if (kMultiWave) {
        // LDS float adds: one slot per (splat, field) for all wavefronts
        float* dst = s_g + j * 9;
        if (writer && tot8 != 0.f) atomicAdd(dst + my_field, tot8);
        if (lane == 63 && tot9 != 0.f) atomicAdd(dst + 8, tot9);
      } else {
        float* dst = a.g2 + s_id[j];
        if (writer && tot8 != 0.f) atomicAdd(dst + (size_t)my_field * a.g2_plane, tot8);
        if (lane == 63 && tot9 != 0.f) atomicAdd(dst + 8 * a.g2_plane, tot9);
      }
     }
    }
    __syncthreads();
    if (kMultiWave) {
      for (uint32_t q = threadIdx.x; q < cnt * 9; q += G::NT) {
        const float v = s_g[q];
        if (v != 0.f) atomicAdd(&a.g2[(size_t)(q % 9) * a.g2_plane + s_id[q / 9]], v);
      }
      __syncthreads();
    }
    b_end = b_begin;
  }
  if (a.mode == 1) {
    lossv = wave_total_lane63(lossv);
    if (lane == 63 && lossv != 0.f) atomicAdd(a.loss, lossv);
  }
}

// One workgroup per tile (schedules 0 and 1).
template <int TW, int TH, int PPT, int SW, int BATCH>
__global__ __launch_bounds__(TW* TH / PPT) void k_composite_bwd(BwdArgs a) {
  __shared__ BwdSharedOf<TW, TH, PPT, SW, BATCH> sm;
  composite_bwd_tile<TW, TH, PPT, SW, BATCH>(a, tile_of_block(blockIdx.x, (uint32_t)a.ntiles, a.schedule), sm);
}

// Persistent (schedules 2 and 3), as k_composite_persistent.
template <int TW, int TH, int PPT, int SW, int BATCH>
__global__ __launch_bounds__(TW* TH / PPT) __attribute__((amdgpu_waves_per_eu(7))) void k_composite_bwd_persistent(
    BwdArgs a) {
  __shared__ BwdSharedOf<TW, TH, PPT, SW, BATCH> sm;
  __shared__ uint32_t s_next;
  for (;;) {
    const uint32_t slot = queue_next(a.q, (uint32_t)a.ntiles, &s_next);
    if (slot == kQueueDone) break;
    composite_bwd_tile<TW, TH, PPT, SW, BATCH>(a, slot, sm);
  }
  queue_exit(a.q);
}

// ---- dispatch over the built (tile, pixels-per-thread, batch) variants ----
#define GS_RASTER_LIST(X) \
  X(8, 8, 1, 8)           \
  X(16, 8, 1, 16)         \
  X(16, 8, 2, 16)         \
  X(16, 16, 1, 16)        \
  X(16, 16, 2, 16)        \
  X(16, 16, 4, 16)        \
  X(32, 16, 1, 32)        \
  X(32, 16, 2, 32)        \
  X(32, 16, 4, 32)        \
  X(32, 16, 2, 16)        \
  X(32, 16, 4, 16)        \
  X(32, 32, 1, 32)        \
  X(32, 32, 2, 32)        \
  X(32, 32, 4, 32)        \
  X(32, 32, 2, 16)        \
  X(32, 32, 4, 16)

// Workgroups of `kernel` (NT threads) resident on the whole device at once:
// the grid of a persistent launch.  Queried once per kernel.
template <typename K>
hipError_t resident_workgroups(K kernel, int nt, int* out) {
  static int cached = 0;
  if (cached > 0) {
    *out = cached;
    return hipSuccess;
  }
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0);
  if (e != hipSuccess) return e;
  cached = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  *out = cached;
  return hipSuccess;
}

template <typename K, typename Args>
hipError_t launch_grid_or_persistent(K grid_kernel, K persistent_kernel, int nt, uint32_t ntiles, bool persistent,
                                     hipStream_t st, const Args& a) {
  if (!persistent) {
    hipLaunchKernelGGL(grid_kernel, dim3(ntiles), dim3(nt), 0, st, a);
    return hipGetLastError();
  }
  int res = 0;
  const hipError_t e = resident_workgroups(persistent_kernel, nt, &res);
  if (e != hipSuccess) return e;
  const uint32_t g = ntiles < (uint32_t)res ? ntiles : (uint32_t)res;
  hipLaunchKernelGGL(persistent_kernel, dim3(g), dim3(nt), 0, st, a);
  return hipGetLastError();
}

template <int TW, int TH, int PPT, int SW, typename Args>
hipError_t launch_fwd(int batch, uint32_t ntiles, bool persistent, hipStream_t st, const Args& a) {
  constexpr int NT = TW * TH / PPT;
  switch (batch) {
    case 32:
      return launch_grid_or_persistent(k_composite<TW, TH, PPT, SW, 32>, k_composite_persistent<TW, TH, PPT, SW, 32>,
                                       NT, ntiles, persistent, st, a);
    case 64:
      return launch_grid_or_persistent(k_composite<TW, TH, PPT, SW, 64>, k_composite_persistent<TW, TH, PPT, SW, 64>,
                                       NT, ntiles, persistent, st, a);
    case 128:
      return launch_grid_or_persistent(k_composite<TW, TH, PPT, SW, 128>,
                                       k_composite_persistent<TW, TH, PPT, SW, 128>, NT, ntiles, persistent, st, a);
    case 256:
      return launch_grid_or_persistent(k_composite<TW, TH, PPT, SW, 256>,
                                       k_composite_persistent<TW, TH, PPT, SW, 256>, NT, ntiles, persistent, st, a);
    default: return hipErrorInvalidValue;
  }
}

template <int TW, int TH, int PPT, int SW, typename Args>
hipError_t launch_bwd(int batch, uint32_t ntiles, bool persistent, hipStream_t st, const Args& a) {
  constexpr int NT = TW * TH / PPT;
  switch (batch) {
    case 32:
      return launch_grid_or_persistent(k_composite_bwd<TW, TH, PPT, SW, 32>,
                                       k_composite_bwd_persistent<TW, TH, PPT, SW, 32>, NT, ntiles, persistent, st, a);
    case 64:
      return launch_grid_or_persistent(k_composite_bwd<TW, TH, PPT, SW, 64>,
                                       k_composite_bwd_persistent<TW, TH, PPT, SW, 64>, NT, ntiles, persistent, st, a);
    case 128:
      return launch_grid_or_persistent(k_composite_bwd<TW, TH, PPT, SW, 128>,
                                       k_composite_bwd_persistent<TW, TH, PPT, SW, 128>, NT, ntiles, persistent, st,
                                       a);
    case 256:
      return launch_grid_or_persistent(k_composite_bwd<TW, TH, PPT, SW, 256>,
                                       k_composite_bwd_persistent<TW, TH, PPT, SW, 256>, NT, ntiles, persistent, st,
                                       a);
    default: return hipErrorInvalidValue;
  }
}

// The work queue of a persistent launch (schedules 2 and 3) in the workspace.
TileQueue tile_queue(const Plan& pl, void* ws) {
  TileQueue q;
  q.head = seg<Counters>(ws, pl.ws.counters)->queue;
  q.order = pl.schedule == 3 ? seg<uint32_t>(ws, pl.ws.order) : nullptr;
  return q;
}

void tile_span(const Plan& pl, int v0, int nv, int32_t* tb, int32_t* ntiles) {
  *tb = pl.views[v0].tile_base;
  const int32_t te = (v0 + nv < pl.n_views) ? pl.views[v0 + nv].tile_base : pl.total_tiles;
  *ntiles = te - *tb;
}

}  // namespace

bool raster_variant_built(int tw, int th, int ppt, int sw) {
#define GS_HAS(W, H, P, S) \
  if (tw == W && th == H && ppt == P && sw == S) return true;
  GS_RASTER_LIST(GS_HAS)
#undef GS_HAS
  return false;
}

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
  a.schedule = pl.schedule;
  int32_t ntiles;
  tile_span(pl, v0, nv, &a.tile_begin, &ntiles);
  a.ntiles = ntiles;
  a.ranges = seg<uint2>(ws, pl.ws.ranges);
  a.vals = seg<uint32_t>(ws, sorted_values_in_b(pl, v0, nv) ? pl.ws.vals_b : pl.ws.vals_a);
  a.rec = seg<float4>(ws, pl.ws.rec);
  a.img = img;
  a.T = T;
  a.ncontrib = nc;
  a.last = seg<uint32_t>(ws, pl.ws.last);
  a.strips = seg<uint16_t>(ws, pl.ws.strips);
  a.cap = (uint32_t)pl.cap;
  a.bg0 = pl.bg[0];
  a.bg1 = pl.bg[1];
  a.bg2 = pl.bg[2];
  a.q = tile_queue(pl, ws);
  if (ntiles <= 0) return hipSuccess;
  const bool persistent = pl.schedule >= 2;
  const int tw = pl.tile_w, th = pl.tile_h, ppt = pl.ppt, sw = pl.wave_w, b = pl.batch_depth;
#define GS_FWD(W, H, P, S) \
  if (tw == W && th == H && ppt == P && sw == S) return launch_fwd<W, H, P, S>(b, (uint32_t)ntiles, persistent, st, a);
  GS_RASTER_LIST(GS_FWD)
#undef GS_FWD
  return hipErrorInvalidValue;
}

hipError_t launch_composite_bwd(const Plan& pl, int v0, int nv, void* ws, const float* img, const float* T,
                                const float* up, int mode, float* loss, int32_t n_active, hipStream_t st) {
  BwdArgs a;
  a.n_gauss = (uint32_t)pl.n;
  a.n_active = (uint32_t)n_active;
  a.views = pl.d_views;
  a.tile_view = pl.d_tile_view;
  a.schedule = pl.schedule;
  int32_t ntiles;
  tile_span(pl, v0, nv, &a.tile_begin, &ntiles);
  a.ntiles = ntiles;
  a.ranges = seg<uint2>(ws, pl.ws.ranges);
  a.vals = seg<uint32_t>(ws, sorted_values_in_b(pl, v0, nv) ? pl.ws.vals_b : pl.ws.vals_a);
  a.rec = seg<float4>(ws, pl.ws.rec);
  a.img = img;
  a.T = T;
  a.last = seg<uint32_t>(ws, pl.ws.last);
  a.up = up;
  a.strips = seg<uint32_t>(ws, pl.ws.strips);
  a.mode = mode;
  a.loss_mode = pl.loss_mode;
  a.g2 = seg<float>(ws, pl.ws.g2);
  a.g2_plane = (size_t)pl.ws.vn;
  a.loss = loss;
  a.cap = (uint32_t)pl.cap;
  a.bg0 = pl.bg[0];
  a.bg1 = pl.bg[1];
  a.bg2 = pl.bg[2];
  a.q = tile_queue(pl, ws);
  if (ntiles <= 0) return hipSuccess;
  const bool persistent = pl.schedule >= 2;
  const int tw = pl.tile_w, th = pl.tile_h, ppt = pl.ppt, sw = pl.wave_w, b = pl.batch_depth;
#define GS_BWD(W, H, P, S) \
  if (tw == W && th == H && ppt == P && sw == S) return launch_bwd<W, H, P, S>(b, (uint32_t)ntiles, persistent, st, a);
  GS_RASTER_LIST(GS_BWD)
#undef GS_BWD
  return hipErrorInvalidValue;
}

}  // namespace gs
