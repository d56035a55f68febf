// Internal declarations shared by the gsopt HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/gsopt.h"

namespace gs {

constexpr int kMaxViews = 256;
constexpr int kRecFloats = 12;    // splat record: 3 x float4
constexpr int kG2Fields = 9;      // screen-space gradient fields per (view, Gaussian), one plane each
constexpr int kSortBlock = 256;   // threads of the sort / scan kernels
constexpr int kSortItems = 16;    // keys per thread per chunk
constexpr int kSortChunk = kSortBlock * kSortItems;

// Thresholds of the compositing rule, as FP32 values.
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kCutoff = -4.5f;
constexpr float kNear = 0.2f;
constexpr float kDilation = 0.3f;
constexpr float kGuard = 1.3f;

struct ViewInfo {
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  int32_t tile_base;     // first global tile of the view
  int32_t pad;
  int64_t pix_off;       // first pixel of the view in the packed frame
};

// Device counters living at the start of the workspace.
struct Counters {
  uint32_t nvis;          // visible (view, Gaussian) pairs of the last project
  uint32_t keys;          // keys needed by the last tile-list build
  uint32_t overflow;      // set when keys > capacity
  uint32_t key_cap;
  uint32_t kept;          // active count kept by the last freeze
  uint32_t overflow_any;  // set with overflow, cleared only by gs_read_counters / gs_workspace_init
  uint32_t queue[2];      // work queue of the persistent compositing kernels (zero between launches)
};

// A view's camera in double precision for the projection kernels (every
// member is the camera's float converted exactly, or the guard-band limit
// computed from them in double), written by a one-thread-per-view kernel at
// the start of each projection launch.
struct ViewD {
  double W[9];          // rotation, row-major
  double t[3];
  double fx, fy, cx, cy;
  double limx, limy;    // guard band on x/z and y/z
};

// Byte offsets of the workspace segments (computed by the host at plan time).
struct WsLayout {
  size_t counters;
  size_t depth;       // u32 [VN]   FP32 depth key bits
  size_t count;       // u32 [VN]   tiles touched (0 = culled)
  size_t rect;        // u16x4 [VN] tile rectangle (tx0, ty0, tx1, ty1)
  size_t rec;         // float4x3 [VN] splat record
  size_t g2;          // float [9][VN] screen-space gradients, field-major (one plane per field)
  size_t vis_a, vis_b, vkey_a, vkey_b;  // u32 [VN] visible ids / depth keys (sort ping-pong)
  size_t vrect_a, vrect_b;              // u16x4 [VN] tile rectangles carried through the depth sort
  size_t koff;        // u32 [VN+1] key offsets in depth order
  size_t keys_a, keys_b, vals_a, vals_b;  // u32 [cap]
  size_t strips;      // u32 [cap] strip bits of each list entry, stored by the forward compositing
  size_t hist;        // u32 [256 * max_blocks + 1]
  size_t firsts;      // u32 [max_blocks] depth-order pair owning the first key slot of each sort chunk
  size_t partial;     // u32 [scan partials]
  size_t ranges;      // u32x2 [tiles]
  size_t order;       // u32 [tiles] compositing order of the tiles (longest lists first)
  size_t obucket;     // u32 [2 * 33] list-length histogram and cursors of that order
  size_t last;        // u32 [pixels]
  size_t vconst;      // ViewD [kMaxViews] per-view camera constants of the last projection launch
  size_t vmask;       // u64 [n] views of the last projection call that see the Gaussian
                      // (bit v - v0 when the call has at most 64 views, else all ones)
  size_t dflags;      // u8 [n] delta flags
  size_t dcount;      // u32 [6 * dblocks + 1] delta block counts (scanned in place)
  size_t dbase;       // u32 [16] delta section bases
  size_t total;
  int64_t vn;
  int64_t cap;
  int64_t hist_blocks;
  int64_t partial_len;
  int32_t dblocks;
};

struct Plan {
  int32_t n = 0, sh_degree = 0, n_views = 0;
  int32_t tile_w = 16, tile_h = 16, batch_depth = 64, ppt = 1, wave_w = 16, schedule = 0;
  float bg[3] = {0, 0, 0};
  int32_t loss_mode = 0;
  int32_t total_tiles = 0;
  int64_t total_pixels = 0;
  int64_t cap = 0;
  ViewInfo views[kMaxViews];
  WsLayout ws;
  // preculling (caller-owned device arrays; null = off)
  const uint32_t* cell_of = nullptr;
  const uint8_t* cell_mask = nullptr;
  int32_t cell_row = 0;   // n_cells + 1
  // library-owned device copies
  ViewInfo* d_views = nullptr;
  int32_t* d_tile_view = nullptr;
  bool valid = false;
};

template <typename T>
__host__ __device__ inline T* seg(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

// ---------------------------------------------------------------------------
// Splat record: the projected quantities the compositing loops read.
//   r0 = (u_hi, w_hi, u_lo, w_lo)   projected mean as a float pair
//   r1 = (a, r, s, o)               conic in the form
//        P = -1/2 (a (dx + r dy)^2 + s dy^2) with a = Q00, r = Q01/Q00,
//        s = det(Q)/Q00 (= 1 / Sigma2_11); o = opacity
//   r2 = (red, green, blue, 0)
// ---------------------------------------------------------------------------
// Evaluation of one splat at one pixel centre, in two parts so that a
// wavefront can skip the second when no lane passes the first.  These are
// the one place that decides whether a pixel takes a splat; the forward and
// backward kernels call them on identical inputs, so they make identical
// decisions bit for bit.
struct SplatGeom {
  float dx, dy, e, P;
};

// The compositing kernels stage each record with the conic's a and s already
// multiplied by -log2(e)/2 (staged_conic), so that the power comes out in
// base 2, P2 = (-L a/2 e) e + (-L s/2) dy^2 = log2(e) P up to rounding, which
// the hardware exp2 takes directly.  The 3-sigma test compares P2 with
// fl(-4.5 log2(e)); it can decide differently from P >= -4.5 only where P lies
// within a few units of rounding of the cut-off.
constexpr float kLog2e = 1.44269504088896341f;
constexpr float kMinusHalfLog2e = -0.5f * kLog2e;   // exact: a power-of-two multiple
constexpr float kCutoff2 = kCutoff * kLog2e;
__device__ __forceinline__ float4 staged_conic(const float4& r1) {
  return make_float4(kMinusHalfLog2e * r1.x, r1.y, kMinusHalfLog2e * r1.z, r1.w);
}

// r1h: the record's second float4 after staged_conic; P is the base-2 power
__device__ __forceinline__ SplatGeom splat_power(float pxc, float pyc, const float4& r0, const float4& r1h) {
#pragma clang fp contract(off)
  SplatGeom g;
  g.dx = (pxc - r0.x) - r0.z;
  g.dy = (pyc - r0.y) - r0.w;
  g.e = fmaf(r1h.y, g.dy, g.dx);
  g.P = fmaf(r1h.x * g.e, g.e, r1h.z * (g.dy * g.dy));
  return g;
}

// Opacity part, for a pixel that passed the 3-sigma test (base-2 power
// P2 >= kCutoff2): returns whether alpha reaches the 1/255 skip threshold.
__device__ __forceinline__ bool splat_alpha(float P2, float opacity, float& G, float& alpha, bool& clamped) {
#pragma clang fp contract(off)
  G = __builtin_amdgcn_exp2f(P2);
  const float oG = opacity * G;
  clamped = oG >= kAlphaMax;
  alpha = clamped ? kAlphaMax : oG;
  return alpha >= kAlphaMin;
}

// ---- launchers implemented in the .hip files -------------------------------
struct ParamPtrs {
  const float* mean;
  const float* lsc;
  const float* quat;
  const float* opac;
  const float* sh;
  int32_t n, deg;
};

hipError_t launch_project(const Plan& pl, const ParamPtrs& p, const gs_camera* cams, int v0, int nv, void* ws,
                          hipStream_t st);
hipError_t launch_project_bwd(const Plan& pl, const ParamPtrs& p, const gs_camera* cams, int v0, int nv, void* ws,
                              const gs_params& grads, int accumulate, hipStream_t st);
hipError_t launch_tile_lists(const Plan& pl, int v0, int nv, void* ws, hipStream_t st);
hipError_t launch_composite(const Plan& pl, int v0, int nv, void* ws, float* img, float* T, uint32_t* nc,
                            hipStream_t st);
hipError_t launch_composite_bwd(const Plan& pl, int v0, int nv, void* ws, const float* img, const float* T,
                                const float* up, int mode, float* loss, int32_t n_active, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t st);
hipError_t launch_adam(const gs_params& p, const gs_params& g, const gs_params& m, const gs_params& v,
                       int32_t* step, const gs_adam_hparams& hp, const gs_adam_hparams* dev_hp, hipStream_t st);
hipError_t launch_assign_cells(const ParamPtrs& p, const gs_grid& g, uint32_t* cell_of, uint32_t* cell_sigma,
                               hipStream_t st);
hipError_t launch_visible_cells(const gs_grid& g, const gs_camera* cams, int v0, int nv, const uint32_t* cell_sigma,
                                uint8_t* mask, hipStream_t st);
hipError_t launch_freeze(const Plan& pl, const gs_params& p, const gs_params& m, const gs_params& v,
                         const uint8_t* flags, uint32_t* ids, const gs_params* base, void* ws, int32_t* new_active,
                         hipStream_t st);
hipError_t launch_sort_cells(const Plan& pl, const gs_params& p, const gs_params* m, const gs_params* v,
                             uint32_t* cell_of, int32_t n_cells, int64_t n_active, uint32_t* ids, const gs_params* base,
                             void* ws, hipStream_t st);
hipError_t launch_delta(const Plan& pl, const gs_params& cur, const gs_params& base, uint32_t mask, float tau,
                        uint32_t* out, void* ws, hipStream_t st);
hipError_t launch_delta_encode(const Plan& pl, const gs_params& cur, const gs_params& base, const gs_codec* codecs,
                               uint32_t mask, const uint32_t* epoch, uint32_t* out, void* ws, hipStream_t st);
// Largest model of gs_delta_encode_noalloc, whose scratch is a fixed device array.
constexpr int64_t kNoAllocMaxN = GS_NOALLOC_MAX_N;
size_t noalloc_scratch_bytes();
// Looks up this device's copy of that array (the device must be current).
hipError_t noalloc_scratch_init(int device);
hipError_t launch_delta_encode_noalloc(int device, const gs_params& cur, const gs_params& base, const gs_codec* codecs,
                                       uint32_t mask, const uint32_t* epoch, uint32_t* out, hipStream_t st);
hipError_t launch_delta_apply(const gs_params& model, const gs_codec* codecs, const uint32_t* packet,
                              int64_t packet_words, const uint32_t* epoch, uint32_t* status, hipStream_t st);
// words that one sent row of a group of `width` values occupies under a codec
inline int64_t codec_row_words(const gs_codec& k, int width) {
  if (k.mode == GS_CODEC_RAW) return width;
  const int per = 32 / k.bits;
  return (width + per - 1) / per;
}
hipError_t launch_epoch_bump(uint32_t* epoch, hipStream_t st);
hipError_t launch_object_transform(const gs_params& p, const int32_t* object_of, const gs_transform* tf,
                                   int32_t n_objects, hipStream_t st);
hipError_t launch_relight_dc(const gs_params& p, const float* gain, int channels, hipStream_t st);
hipError_t launch_append(const gs_params& old_p, const gs_params* old_m, const gs_params* old_v, int64_t na,
                         const gs_params& add, const gs_params& new_p, const gs_params* new_m,
                         const gs_params* new_v, const uint32_t* const* old_cols, const uint32_t* const* add_cols,
                         uint32_t* const* new_cols, int n_cols, hipStream_t st);
// whether the sorted tile lists of views [v0, v0+nv) end in the second buffer
bool sorted_values_in_b(const Plan& pl, int v0, int nv);
// whether compositing kernels were built for this tile shape / pixels per thread
bool raster_variant_built(int tile_w, int tile_h, int ppt, int wave_w);

// stable radix sort of `count` (key, value) pairs on key bits [0, bits) in the
// sort scratch of the workspace (histograms and partials); ping-pong buffers,
// *in_b tells whether the result landed in (kb, vb)
hipError_t launch_sort_pairs(const Plan& pl, void* ws, uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb,
                             int64_t count, int bits, bool* in_b, hipStream_t st);
// exclusive scan of `count` u32 values (count read from *dcount when non-null,
// capped at `max_count`); total written to *total when non-null.
hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t max_count, const uint32_t* dcount,
                       uint32_t* partial, int64_t partial_len, uint32_t* total, hipStream_t st);

}  // namespace gs
