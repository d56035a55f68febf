// Host side of the gsopt C ABI: validation, plan and workspace layout, stage
// sequencing (batched and plain), graph capture and replay.
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace gs;

namespace {
constexpr int kStages = 7;
const char* const kStageNames[kStages] = {"project", "tile_lists", "composite", "composite_bwd",
                                          "project_bwd", "adam", "delta"};
enum { ST_PROJECT, ST_LISTS, ST_COMPOSITE, ST_COMPOSITE_BWD, ST_PROJECT_BWD, ST_ADAM, ST_DELTA };
struct PendingTimer {
  int stage;
  hipEvent_t start, stop;
};
}  // namespace

struct gs_context {
  bool prof = false;
  bool capturing = false;
  std::vector<PendingTimer> pending;
  double stage_ms[kStages] = {0};
  int64_t stage_calls[kStages] = {0};
  int device = 0;
  std::string err;
  Plan plan;
  uint64_t plan_gen = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  gs_step_args captured{};
  uint64_t graph_gen = 0;
  // set when gs_read_counters finds that a tile-list build overflowed the key
  // capacity; the rendering calls refuse to run until the next gs_plan
  bool capacity_exceeded = false;
};

namespace {

gs_status fail(gs_ctx c, gs_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
gs_status fail(gs_ctx c, gs_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

gs_status hip_check(gs_ctx c, hipError_t e, const char* what) {
  if (e == hipSuccess) return GS_OK;
  return fail(c, GS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define GS_HIP(c, expr)                                   \
  do {                                                    \
    gs_status _s = hip_check((c), (expr), #expr);         \
    if (_s != GS_OK) return _s;                           \
  } while (0)

// Runs f() (which enqueues kernels on st), bracketed by timing events when
// the stage timers are on.
template <class F>
hipError_t timed(gs_ctx c, int stage, hipStream_t st, F&& f) {
  if (!c->prof || c->capturing) return f();
  PendingTimer t{stage, nullptr, nullptr};
  hipError_t e = hipEventCreate(&t.start);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&t.stop);
  if (e != hipSuccess) return e;
  e = hipEventRecord(t.start, st);
  if (e != hipSuccess) return e;
  e = f();
  hipError_t e2 = hipEventRecord(t.stop, st);
  c->pending.push_back(t);
  return e != hipSuccess ? e : e2;
}

hipError_t flush_timers(gs_ctx c) {
  hipError_t first = hipSuccess;
  for (auto& t : c->pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(t.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.start, t.stop);
    if (e == hipSuccess) {
      c->stage_ms[t.stage] += ms;
      c->stage_calls[t.stage] += 1;
    } else if (first == hipSuccess) {
      first = e;
    }
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  c->pending.clear();
  return first;
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool tile_ok(int w, int h) {
  return (w == 8 && h == 8) || (w == 16 && h == 8) || (w == 16 && h == 16) || (w == 32 && h == 16) ||
         (w == 32 && h == 32);
}

WsLayout make_layout(int64_t n, int64_t nviews, int64_t tiles, int64_t pixels, int64_t cap) {
  WsLayout L{};
  const int64_t vn = n * nviews;
  L.vn = vn;
  L.cap = cap;
  int64_t maxsort = vn > cap ? vn : cap;
  if (tiles > maxsort) maxsort = tiles;
  L.hist_blocks = cdiv(maxsort, kSortChunk);
  L.dblocks = (int32_t)cdiv(n, 256);
  int64_t maxscan = maxsort;
  if (256 * L.hist_blocks > maxscan) maxscan = 256 * L.hist_blocks;
  if (6ll * L.dblocks > maxscan) maxscan = 6ll * L.dblocks;
  L.partial_len = cdiv(maxscan, kSortChunk) + 2;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = al(o + (bytes ? bytes : 1)); return at; };
  L.counters = take(sizeof(Counters));
  L.depth = take(4 * vn);
  L.count = take(4 * vn);
  L.rect = take(8 * vn);
  L.rec = take(sizeof(float) * kRecFloats * vn);
  L.g2 = take(sizeof(float) * kG2Fields * vn);
  L.vis_a = take(4 * vn);
  L.vis_b = take(4 * vn);
  L.vkey_a = take(4 * vn);
  L.vkey_b = take(4 * vn);
  L.vrect_a = take(8 * vn);
  L.vrect_b = take(8 * vn);
  L.koff = take(4 * (vn + 1));
  L.keys_a = take(4 * cap);
  L.keys_b = take(4 * cap);
  L.vals_a = take(4 * cap);
  L.vals_b = take(4 * cap);
  L.strips = take(4 * (size_t)cap);
  L.hist = take(4 * (256 * L.hist_blocks + 1));
  L.firsts = take(4 * L.hist_blocks);
  L.partial = take(4 * L.partial_len);
  L.ranges = take(8 * tiles);
  L.order = take(4 * tiles);
  L.obucket = take(4 * 128);
  L.last = take(4 * pixels);
  L.vconst = take(sizeof(ViewD) * kMaxViews);
  L.vmask = take(8 * n);
  L.dflags = take(n);
  L.dcount = take(4 * (6ll * L.dblocks + 1));
  L.dbase = take(4 * 16);
  L.total = o;
  return L;
}

gs_status check_params(gs_ctx c, const gs_params* p, const char* what) {
  if (!p) return fail(c, GS_ERR_INVALID, "%s: null gs_params", what);
  if (p->n != c->plan.n || p->sh_degree != c->plan.sh_degree)
    return fail(c, GS_ERR_INVALID, "%s: n=%d sh_degree=%d differ from the plan (n=%d, sh_degree=%d)", what, p->n,
                p->sh_degree, c->plan.n, c->plan.sh_degree);
  if (p->n > 0 && (!p->mean || !p->log_scale || !p->quat || !p->opacity_logit || !p->sh))
    return fail(c, GS_ERR_INVALID, "%s: null tensor pointer", what);
  return GS_OK;
}

// Trainable tensors (gradients, Adam moments) describe the active pool: the
// first t->n Gaussians of the plan's n, rows strided by t->n.
gs_status check_trainable(gs_ctx c, const gs_params* t, const char* what) {
  if (!t) return fail(c, GS_ERR_INVALID, "%s: null gs_params", what);
  if (t->n < 0 || t->n > c->plan.n || t->sh_degree != c->plan.sh_degree)
    return fail(c, GS_ERR_INVALID, "%s: n=%d (active pool) must lie in [0, %d] with sh_degree %d", what, t->n,
                c->plan.n, c->plan.sh_degree);
  if (t->n > 0 && (!t->mean || !t->log_scale || !t->quat || !t->opacity_logit || !t->sh))
    return fail(c, GS_ERR_INVALID, "%s: null tensor pointer", what);
  return GS_OK;
}

gs_status check_range(gs_ctx c, int v0, int nv, const void* ws, const char* what) {
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "%s: no plan (call gs_plan first)", what);
  if (v0 < 0 || nv < 1 || v0 + nv > c->plan.n_views)
    return fail(c, GS_ERR_INVALID, "%s: view range [%d, %d) outside [0, %d)", what, v0, v0 + nv, c->plan.n_views);
  if (!ws) return fail(c, GS_ERR_INVALID, "%s: null workspace", what);
  return GS_OK;
}

gs_status check_capacity(gs_ctx c, const char* what) {
  if (!c->capacity_exceeded) return GS_OK;
  return fail(c, GS_ERR_CAPACITY, "%s: a tile-list build overflowed the key capacity of %lld (reported by "
              "gs_read_counters); call gs_plan with a larger key_capacity", what, (long long)c->plan.cap);
}

bool same_params(const gs_params& a, const gs_params& b) {
  return a.mean == b.mean && a.log_scale == b.log_scale && a.quat == b.quat && a.opacity_logit == b.opacity_logit &&
         a.sh == b.sh && a.n == b.n && a.sh_degree == b.sh_degree;
}

bool same_args(const gs_step_args& a, const gs_step_args& b) {
  bool same = same_params(a.params, b.params) && same_params(a.grads, b.grads) && same_params(a.adam_m, b.adam_m) &&
              same_params(a.adam_v, b.adam_v) && a.dev_cams == b.dev_cams && a.dev_target == b.dev_target &&
              a.dev_images == b.dev_images && a.dev_T_final == b.dev_T_final && a.dev_n_contrib == b.dev_n_contrib &&
              a.dev_loss == b.dev_loss && a.dev_step == b.dev_step && a.dev_workspace == b.dev_workspace &&
              a.dev_hp == b.dev_hp && (a.dev_hp || std::memcmp(&a.hp, &b.hp, sizeof(a.hp)) == 0) &&
              a.plain == b.plain && a.do_delta == b.do_delta;
  if (same && a.do_delta)
    same = same_params(a.baseline, b.baseline) && a.group_mask == b.group_mask && a.rel_tau == b.rel_tau &&
           a.dev_delta_out == b.dev_delta_out && a.delta_cap_words == b.delta_cap_words;
  return same;
}

ParamPtrs ptrs(const gs_params* p) {
  return ParamPtrs{p->mean, p->log_scale, p->quat, p->opacity_logit, p->sh, p->n, p->sh_degree};
}

}  // namespace

extern "C" {

gs_status gs_create(int32_t hip_device, gs_ctx* out) {
  if (!out) return GS_ERR_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count) return GS_ERR_INVALID;
  if (hipSetDevice(hip_device) != hipSuccess) return GS_ERR_HIP;
  // this device's copy of the allocation-free encoder's scratch
  if (noalloc_scratch_init(hip_device) != hipSuccess) return GS_ERR_HIP;
  gs_ctx c = new gs_context();
  c->device = hip_device;
  *out = c;
  return GS_OK;
}

gs_status gs_destroy(gs_ctx c) {
  if (!c) return GS_ERR_INVALID;
  (void)flush_timers(c);
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->plan.d_views) (void)hipFree(c->plan.d_views);
  if (c->plan.d_tile_view) (void)hipFree(c->plan.d_tile_view);
  delete c;
  return GS_OK;
}

const char* gs_last_error(gs_ctx c) { return c ? c->err.c_str() : "null context"; }

gs_status gs_plan(gs_ctx c, int32_t n, int32_t sh_degree, int32_t n_views, const gs_camera* cams,
                  const gs_render_opts* opts, int64_t key_capacity, size_t* ws_bytes) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (n < 0) return fail(c, GS_ERR_INVALID, "gs_plan: n=%d < 0", n);
  if (sh_degree < 0 || sh_degree > 3) return fail(c, GS_ERR_INVALID, "gs_plan: sh_degree=%d not in 0..3", sh_degree);
  if (n_views < 1 || n_views > kMaxViews)
    return fail(c, GS_ERR_INVALID, "gs_plan: n_views=%d not in 1..%d", n_views, kMaxViews);
  if (!cams || !opts || !ws_bytes) return fail(c, GS_ERR_INVALID, "gs_plan: null argument");
  if (!tile_ok(opts->tile_w, opts->tile_h))
    return fail(c, GS_ERR_UNSUPPORTED, "gs_plan: tile %dx%d not built", opts->tile_w, opts->tile_h);
  const int bd = opts->batch_depth;
  if (bd != 32 && bd != 64 && bd != 128 && bd != 256)
    return fail(c, GS_ERR_UNSUPPORTED, "gs_plan: batch_depth=%d not in {32,64,128,256}", bd);
  const int ppt = opts->pixels_per_thread == 0 ? 1 : opts->pixels_per_thread;
  const int wave_w = opts->wave_w == 0 ? opts->tile_w : opts->wave_w;
  if (!raster_variant_built(opts->tile_w, opts->tile_h, ppt, wave_w))
    return fail(c, GS_ERR_UNSUPPORTED, "gs_plan: %d pixels per thread with %d-wide wave tiles not built for %dx%d tiles",
                ppt, wave_w, opts->tile_w, opts->tile_h);
  if (opts->schedule < 0 || opts->schedule > 3)
    return fail(c, GS_ERR_INVALID, "gs_plan: schedule=%d not in {0,1,2,3}", opts->schedule);
  if (opts->loss_mode != 0 && opts->loss_mode != 1)
    return fail(c, GS_ERR_INVALID, "gs_plan: loss_mode=%d", opts->loss_mode);
  if (key_capacity < 1 || key_capacity > (int64_t)0x7fffffff)
    return fail(c, GS_ERR_INVALID, "gs_plan: key_capacity=%lld outside [1, 2^31)", (long long)key_capacity);
  if ((int64_t)n * n_views >= (int64_t)0xffffffffll)
    return fail(c, GS_ERR_INVALID, "gs_plan: n * n_views must stay below 2^32");
  Plan pl;
  pl.n = n;
  pl.sh_degree = sh_degree;
  pl.n_views = n_views;
  pl.tile_w = opts->tile_w;
  pl.tile_h = opts->tile_h;
  pl.batch_depth = bd;
  pl.ppt = ppt;
  pl.wave_w = wave_w;
  pl.schedule = opts->schedule;
  for (int k = 0; k < 3; ++k) pl.bg[k] = opts->bg[k];
  pl.loss_mode = opts->loss_mode;
  int64_t tiles = 0, pixels = 0;
  for (int v = 0; v < n_views; ++v) {
    const gs_camera& cam = cams[v];
    if (cam.width < 1 || cam.height < 1 || cam.width > 16384 || cam.height > 16384)
      return fail(c, GS_ERR_INVALID, "gs_plan: view %d size %dx%d outside 1..16384", v, cam.width, cam.height);
    if (!(cam.fx > 0.f) || !(cam.fy > 0.f) || !std::isfinite(cam.fx) || !std::isfinite(cam.fy))
      return fail(c, GS_ERR_INVALID, "gs_plan: view %d focal lengths must be finite and positive", v);
    ViewInfo& vi = pl.views[v];
    vi.width = cam.width;
    vi.height = cam.height;
    vi.tiles_x = (cam.width + pl.tile_w - 1) / pl.tile_w;
    vi.tiles_y = (cam.height + pl.tile_h - 1) / pl.tile_h;
    vi.tile_base = (int32_t)tiles;
    vi.pad = 0;
    vi.pix_off = pixels;
    tiles += (int64_t)vi.tiles_x * vi.tiles_y;
    pixels += (int64_t)cam.width * cam.height;
  }
  if (tiles > 0x7fffffff) return fail(c, GS_ERR_INVALID, "gs_plan: too many tiles");
  pl.total_tiles = (int32_t)tiles;
  pl.total_pixels = pixels;
  pl.cap = key_capacity;
  pl.ws = make_layout(n, n_views, tiles, pixels, key_capacity);
  // library-owned device tables
  std::vector<int32_t> tv(tiles);
  for (int v = 0; v < n_views; ++v) {
    const int64_t b = pl.views[v].tile_base, e = b + (int64_t)pl.views[v].tiles_x * pl.views[v].tiles_y;
    for (int64_t t = b; t < e; ++t) tv[t] = v;
  }
  GS_HIP(c, hipSetDevice(c->device));
  if (c->plan.d_views) { (void)hipFree(c->plan.d_views); c->plan.d_views = nullptr; }
  if (c->plan.d_tile_view) { (void)hipFree(c->plan.d_tile_view); c->plan.d_tile_view = nullptr; }
  c->plan.valid = false;
  GS_HIP(c, hipMalloc(&pl.d_views, sizeof(ViewInfo) * n_views));
  GS_HIP(c, hipMalloc(&pl.d_tile_view, sizeof(int32_t) * (tiles > 0 ? tiles : 1)));
  GS_HIP(c, hipMemcpy(pl.d_views, pl.views, sizeof(ViewInfo) * n_views, hipMemcpyHostToDevice));
  GS_HIP(c, hipMemcpy(pl.d_tile_view, tv.data(), sizeof(int32_t) * tiles, hipMemcpyHostToDevice));
  pl.valid = true;
  c->plan = pl;
  c->plan_gen += 1;
  c->capacity_exceeded = false;
  *ws_bytes = pl.ws.total;
  return GS_OK;
}

gs_status gs_frame_layout(gs_ctx c, int64_t* pix, int32_t* tiles) {
  if (!c) return GS_ERR_INVALID;
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "gs_frame_layout: no plan");
  const Plan& pl = c->plan;
  for (int v = 0; v <= pl.n_views; ++v) {
    if (pix) pix[v] = v < pl.n_views ? pl.views[v].pix_off : pl.total_pixels;
    if (tiles) tiles[v] = v < pl.n_views ? pl.views[v].tile_base : pl.total_tiles;
  }
  return GS_OK;
}

gs_status gs_workspace_init(gs_ctx c, void* ws, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "gs_workspace_init: no plan");
  if (!ws) return fail(c, GS_ERR_INVALID, "gs_workspace_init: null workspace");
  const Plan& pl = c->plan;
  GS_HIP(c, launch_fill_u32(seg<uint32_t>(ws, pl.ws.g2), 0u, (int64_t)kG2Fields * pl.ws.vn, st));
  GS_HIP(c, launch_fill_u32(seg<uint32_t>(ws, pl.ws.counters), 0u, (int64_t)(sizeof(Counters) / 4), st));
  return GS_OK;
}

gs_status gs_project(gs_ctx c, const gs_params* params, const gs_camera* cams, int32_t v0, int32_t nv, void* ws,
                     hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  gs_status s = check_range(c, v0, nv, ws, "gs_project");
  if (s != GS_OK) return s;
  if ((s = check_capacity(c, "gs_project")) != GS_OK) return s;
  if ((s = check_params(c, params, "gs_project")) != GS_OK) return s;
  if (!cams) return fail(c, GS_ERR_INVALID, "gs_project: null cameras");
  const Plan& pl = c->plan;
  if (v0 == 0) {   // a new step starts: clear the sticky overflow flag
    Counters* ctr = seg<Counters>(ws, pl.ws.counters);
    GS_HIP(c, launch_fill_u32(&ctr->overflow, 0u, 1, st));
  }
  GS_HIP(c, timed(c, ST_PROJECT, st, [&] { return launch_project(pl, ptrs(params), cams, v0, nv, ws, st); }));
  return GS_OK;
}

gs_status gs_build_tile_lists(gs_ctx c, int32_t v0, int32_t nv, void* ws, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  gs_status s = check_range(c, v0, nv, ws, "gs_build_tile_lists");
  if (s != GS_OK) return s;
  if ((s = check_capacity(c, "gs_build_tile_lists")) != GS_OK) return s;
  GS_HIP(c, timed(c, ST_LISTS, st, [&] { return launch_tile_lists(c->plan, v0, nv, ws, st); }));
  return GS_OK;
}

gs_status gs_composite(gs_ctx c, int32_t v0, int32_t nv, void* ws, float* img, float* T, uint32_t* nc,
                       hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  gs_status s = check_range(c, v0, nv, ws, "gs_composite");
  if (s != GS_OK) return s;
  if ((s = check_capacity(c, "gs_composite")) != GS_OK) return s;
  if (!img || !T || !nc) return fail(c, GS_ERR_INVALID, "gs_composite: null output");
  GS_HIP(c, timed(c, ST_COMPOSITE, st, [&] { return launch_composite(c->plan, v0, nv, ws, img, T, nc, st); }));
  return GS_OK;
}

gs_status gs_backward(gs_ctx c, const gs_params* params, const gs_camera* cams, int32_t v0, int32_t nv, void* ws,
                      const float* img, const float* T, const float* up, int32_t mode, const gs_params* grads,
                      int32_t accumulate, float* loss, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  gs_status s = check_range(c, v0, nv, ws, "gs_backward");
  if (s != GS_OK) return s;
  if ((s = check_capacity(c, "gs_backward")) != GS_OK) return s;
  if ((s = check_params(c, params, "gs_backward")) != GS_OK) return s;
  if ((s = check_trainable(c, grads, "gs_backward(grads)")) != GS_OK) return s;
  if (!cams || !img || !T || !up) return fail(c, GS_ERR_INVALID, "gs_backward: null input");
  if (mode != 0 && mode != 1) return fail(c, GS_ERR_INVALID, "gs_backward: mode=%d", mode);
  if (mode == 1 && !loss) return fail(c, GS_ERR_INVALID, "gs_backward: mode 1 needs a loss pointer");
  if (accumulate != 0 && accumulate != 1) return fail(c, GS_ERR_INVALID, "gs_backward: accumulate=%d", accumulate);
  const Plan& pl = c->plan;
  GS_HIP(c, timed(c, ST_COMPOSITE_BWD, st,
                  [&] { return launch_composite_bwd(pl, v0, nv, ws, img, T, up, mode, loss, grads->n, st); }));
  GS_HIP(c, timed(c, ST_PROJECT_BWD, st, [&] {
    return launch_project_bwd(pl, ptrs(params), cams, v0, nv, ws, *grads, accumulate, st);
  }));
  return GS_OK;
}

// Adam over the active pool; dev_hp (optional) makes the kernels read the
// hyper-parameters from device memory when they run (hp is then only
// validated as given).
static gs_status adam_step(gs_ctx c, const gs_params* p, const gs_params* g, const gs_params* m, const gs_params* v,
                           int32_t* step, const gs_adam_hparams* hp, const gs_adam_hparams* dev_hp, hipStream_t st) {
  if (!p || !g || !m || !v || !step || !hp) return fail(c, GS_ERR_INVALID, "gs_adam_step: null argument");
  const gs_params* all[4] = {p, g, m, v};
  for (int k = 0; k < 4; ++k) {
    if (all[k]->n != (k == 0 ? p->n : g->n) || all[k]->sh_degree != p->sh_degree || all[k]->n < 0)
      return fail(c, GS_ERR_INVALID, "gs_adam_step: gradients and moments must share n (the active pool) and "
                                     "sh_degree with the parameters");
    if (all[k]->n > 0 && (!all[k]->mean || !all[k]->log_scale || !all[k]->quat || !all[k]->opacity_logit ||
                          !all[k]->sh))
      return fail(c, GS_ERR_INVALID, "gs_adam_step: null tensor pointer");
  }
  if (g->n > p->n) return fail(c, GS_ERR_INVALID, "gs_adam_step: active pool %d larger than n=%d", g->n, p->n);
  if (p->sh_degree < 0 || p->sh_degree > 3) return fail(c, GS_ERR_INVALID, "gs_adam_step: sh_degree");
  if (!(hp->beta1 >= 0.f && hp->beta1 < 1.f && hp->beta2 >= 0.f && hp->beta2 < 1.f && hp->eps >= 0.f))
    return fail(c, GS_ERR_INVALID, "gs_adam_step: betas must lie in [0,1) and eps >= 0");
  if (g->n == 0) return GS_OK;
  GS_HIP(c, timed(c, ST_ADAM, st, [&] { return launch_adam(*p, *g, *m, *v, step, *hp, dev_hp, st); }));
  return GS_OK;
}

gs_status gs_adam_step(gs_ctx c, const gs_params* p, const gs_params* g, const gs_params* m, const gs_params* v,
                       int32_t* step, const gs_adam_hparams* hp, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  return adam_step(c, p, g, m, v, step, hp, nullptr, st);
}

static gs_status check_grid(gs_ctx c, const gs_grid* g, const char* what) {
  if (!g) return fail(c, GS_ERR_INVALID, "%s: null grid", what);
  const int64_t nc = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
  if (g->dims[0] < 1 || g->dims[1] < 1 || g->dims[2] < 1 || nc >= (1ll << 31) || !(g->cell_size > 0.f) ||
      !std::isfinite(g->cell_size) || !std::isfinite(g->origin[0]) || !std::isfinite(g->origin[1]) ||
      !std::isfinite(g->origin[2]))
    return fail(c, GS_ERR_INVALID, "%s: grid needs dims >= 1 (fewer than 2^31 cells), a finite origin and a "
                                   "positive cell size", what);
  return GS_OK;
}

gs_status gs_assign_cells(gs_ctx c, const gs_params* params, const gs_grid* grid, uint32_t* cell_of,
                          uint32_t* cell_sigma, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  gs_status s;
  if ((s = check_grid(c, grid, "gs_assign_cells")) != GS_OK) return s;
  if (!params || params->n < 0 || (params->n > 0 && (!params->mean || !params->log_scale)))
    return fail(c, GS_ERR_INVALID, "gs_assign_cells: bad params");
  if ((params->n > 0 && !cell_of) || !cell_sigma) return fail(c, GS_ERR_INVALID, "gs_assign_cells: null output");
  GS_HIP(c, launch_assign_cells(ptrs(params), *grid, cell_of, cell_sigma, st));
  return GS_OK;
}

gs_status gs_visible_cells(gs_ctx c, const gs_grid* grid, const gs_camera* cams, int32_t v0, int32_t nv,
                           const uint32_t* cell_sigma, uint8_t* mask, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  gs_status s;
  if ((s = check_grid(c, grid, "gs_visible_cells")) != GS_OK) return s;
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "gs_visible_cells: no plan");
  if (v0 < 0 || nv < 1 || v0 + nv > c->plan.n_views)
    return fail(c, GS_ERR_INVALID, "gs_visible_cells: view range [%d, %d) outside [0, %d)", v0, v0 + nv,
                c->plan.n_views);
  if (!cams || !cell_sigma || !mask) return fail(c, GS_ERR_INVALID, "gs_visible_cells: null pointer");
  GS_HIP(c, launch_visible_cells(*grid, cams, v0, nv, cell_sigma, mask, st));
  return GS_OK;
}

gs_status gs_set_precull(gs_ctx c, const uint32_t* cell_of, const uint8_t* mask, int32_t n_cells) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "gs_set_precull: no plan");
  if ((cell_of == nullptr) != (mask == nullptr))
    return fail(c, GS_ERR_INVALID, "gs_set_precull: give both cell_of and mask, or neither");
  if (mask && n_cells < 1) return fail(c, GS_ERR_INVALID, "gs_set_precull: n_cells=%d", n_cells);
  c->plan.cell_of = cell_of;
  c->plan.cell_mask = mask;
  c->plan.cell_row = mask ? n_cells + 1 : 0;
  ++c->plan_gen;   // a captured step used the previous setting
  return GS_OK;
}

gs_status gs_freeze(gs_ctx c, gs_params* params, gs_params* m, gs_params* v, const uint8_t* flags, uint32_t* ids,
                    gs_params* baseline, void* ws, int32_t* new_active, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "gs_freeze: no plan");
  gs_status s;
  if ((s = check_params(c, params, "gs_freeze(params)")) != GS_OK) return s;
  if ((s = check_trainable(c, m, "gs_freeze(m)")) != GS_OK) return s;
  if ((s = check_trainable(c, v, "gs_freeze(v)")) != GS_OK) return s;
  if (m->n != v->n) return fail(c, GS_ERR_INVALID, "gs_freeze: m and v describe different active pools");
  if (baseline && (s = check_params(c, baseline, "gs_freeze(baseline)")) != GS_OK) return s;
  if (!ws || !new_active || (m->n > 0 && !flags))
    return fail(c, GS_ERR_INVALID, "gs_freeze: null workspace, flags or new_active");
  GS_HIP(c, launch_freeze(c->plan, *params, *m, *v, flags, ids, baseline, ws, new_active, st));
  return GS_OK;
}

gs_status gs_sort_cells(gs_ctx c, gs_params* params, gs_params* m, gs_params* v, uint32_t* cell_of, int32_t n_cells,
                        uint32_t* ids, gs_params* baseline, void* ws, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "gs_sort_cells: no plan");
  gs_status s;
  if ((s = check_params(c, params, "gs_sort_cells(params)")) != GS_OK) return s;
  if ((m == nullptr) != (v == nullptr)) return fail(c, GS_ERR_INVALID, "gs_sort_cells: give both m and v, or neither");
  if (m) {
    if ((s = check_trainable(c, m, "gs_sort_cells(m)")) != GS_OK) return s;
    if ((s = check_trainable(c, v, "gs_sort_cells(v)")) != GS_OK) return s;
    if (m->n != v->n) return fail(c, GS_ERR_INVALID, "gs_sort_cells: m and v describe different active pools");
  }
  if (baseline && (s = check_params(c, baseline, "gs_sort_cells(baseline)")) != GS_OK) return s;
  if (!ws || (params->n > 0 && !cell_of)) return fail(c, GS_ERR_INVALID, "gs_sort_cells: null workspace or cell_of");
  if (n_cells < 1) return fail(c, GS_ERR_INVALID, "gs_sort_cells: n_cells=%d", n_cells);
  GS_HIP(c, launch_sort_cells(c->plan, *params, m, v, cell_of, n_cells, m ? (int64_t)m->n : (int64_t)params->n, ids,
                              baseline, ws, st));
  return GS_OK;
}

gs_status gs_delta_extract(gs_ctx c, const gs_params* cur, const gs_params* base, uint32_t mask, float tau,
                           uint32_t* out, int64_t cap_words, void* ws, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "gs_delta_extract: no plan");
  gs_status s;
  if ((s = check_params(c, cur, "gs_delta_extract(cur)")) != GS_OK) return s;
  if ((s = check_params(c, base, "gs_delta_extract(baseline)")) != GS_OK) return s;
  if (!out || !ws) return fail(c, GS_ERR_INVALID, "gs_delta_extract: null output or workspace");
  if (mask & ~0x3Fu) return fail(c, GS_ERR_INVALID, "gs_delta_extract: group_mask 0x%x has bits above 5", mask);
  if (!(tau >= 0.f) || !std::isfinite(tau)) return fail(c, GS_ERR_INVALID, "gs_delta_extract: rel_tau must be >= 0");
  const int64_t n = cur->n;
  const int nk = (cur->sh_degree + 1) * (cur->sh_degree + 1);
  const int widths[6] = {1, 3, 3 * (nk - 1), 3, 3, 4};
  int64_t need = 6;
  for (int g = 0; g < 6; ++g)
    if ((mask >> g) & 1u) need += n * (1 + widths[g]);
  if (cap_words < need)
    return fail(c, GS_ERR_INVALID, "gs_delta_extract: out_cap_words=%lld < %lld", (long long)cap_words,
                (long long)need);
  if (need > (int64_t)0xffffffffll) return fail(c, GS_ERR_INVALID, "gs_delta_extract: output above 2^32 words");
  GS_HIP(c, timed(c, ST_DELTA, st, [&] { return launch_delta(c->plan, *cur, *base, mask, tau, out, ws, st); }));
  return GS_OK;
}

static bool codec_ok(const gs_codec& k) {
  if (k.mode == GS_CODEC_RAW) return k.rel_tau >= 0.f && std::isfinite(k.rel_tau);
  if (k.mode != GS_CODEC_RESIDUAL && k.mode != GS_CODEC_QUANT) return false;
  if (k.bits != 8 && k.bits != 16) return false;
  return k.step > 0.f && std::isfinite(k.step) && std::isfinite(1.0f / k.step) && std::isfinite(k.lo);
}

static int64_t codec_capacity(int64_t n, int sh_degree, const gs_codec* codecs, uint32_t mask) {
  const int nk = (sh_degree + 1) * (sh_degree + 1);
  const int widths[6] = {1, 3, 3 * (nk - 1), 3, 3, 4};
  int64_t need = 9;
  for (int g = 0; g < 6; ++g)
    if ((mask >> g) & 1u) need += n * (1 + codec_row_words(codecs[g], widths[g]));
  return need;
}

int64_t gs_codec_capacity_words(int32_t n, int32_t sh_degree, const gs_codec* codecs, uint32_t mask) {
  if (!codecs || n < 0 || sh_degree < 0 || sh_degree > 3 || (mask & ~0x3Fu)) return -1;
  for (int g = 0; g < 6; ++g)
    if (!codec_ok(codecs[g])) return -1;
  return codec_capacity(n, sh_degree, codecs, mask);
}

static gs_status check_codecs(gs_ctx c, const gs_codec* codecs, const char* what) {
  if (!codecs) return fail(c, GS_ERR_INVALID, "%s: null codecs", what);
  for (int g = 0; g < 6; ++g)
    if (!codec_ok(codecs[g]))
      return fail(c, GS_ERR_INVALID, "%s: codec of group %d invalid (mode %d, bits %d, step %g, lo %g, rel_tau %g)",
                  what, g, codecs[g].mode, codecs[g].bits, (double)codecs[g].step, (double)codecs[g].lo,
                  (double)codecs[g].rel_tau);
  return GS_OK;
}

gs_status gs_delta_encode(gs_ctx c, const gs_params* cur, gs_params* base, const gs_codec* codecs, uint32_t mask,
                          const uint32_t* epoch, uint32_t* out, int64_t cap_words, void* ws, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "gs_delta_encode: no plan");
  gs_status s;
  if ((s = check_params(c, cur, "gs_delta_encode(cur)")) != GS_OK) return s;
  if ((s = check_params(c, base, "gs_delta_encode(baseline)")) != GS_OK) return s;
  if ((s = check_codecs(c, codecs, "gs_delta_encode")) != GS_OK) return s;
  if (!out || !ws || !epoch) return fail(c, GS_ERR_INVALID, "gs_delta_encode: null output, epoch or workspace");
  if (mask & ~0x3Fu) return fail(c, GS_ERR_INVALID, "gs_delta_encode: group_mask 0x%x has bits above 5", mask);
  const int64_t need = codec_capacity(cur->n, cur->sh_degree, codecs, mask);
  if (cap_words < need)
    return fail(c, GS_ERR_INVALID, "gs_delta_encode: out_cap_words=%lld < %lld", (long long)cap_words,
                (long long)need);
  if (need > (int64_t)0xffffffffll) return fail(c, GS_ERR_INVALID, "gs_delta_encode: output above 2^32 words");
  GS_HIP(c, timed(c, ST_DELTA, st,
                  [&] { return launch_delta_encode(c->plan, *cur, *base, codecs, mask, epoch, out, ws, st); }));
  return GS_OK;
}

static gs_status check_tensor(gs_ctx c, const gs_params* t, const char* what) {
  if (!t || t->n < 0 || t->sh_degree < 0 || t->sh_degree > 3) return fail(c, GS_ERR_INVALID, "%s: invalid", what);
  if (t->n > 0 && (!t->mean || !t->log_scale || !t->quat || !t->opacity_logit || !t->sh))
    return fail(c, GS_ERR_INVALID, "%s: null tensor pointer", what);
  return GS_OK;
}

gs_status gs_delta_encode_noalloc(gs_ctx c, const gs_params* cur, gs_params* base, const gs_codec* codecs,
                                  uint32_t mask, const uint32_t* epoch, uint32_t* out, int64_t cap_words,
                                  hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  gs_status s;
  if ((s = check_tensor(c, cur, "gs_delta_encode_noalloc(cur)")) != GS_OK) return s;
  if ((s = check_tensor(c, base, "gs_delta_encode_noalloc(baseline)")) != GS_OK) return s;
  if (base->n != cur->n || base->sh_degree != cur->sh_degree)
    return fail(c, GS_ERR_INVALID, "gs_delta_encode_noalloc: baseline (n=%d, degree %d) differs from cur (n=%d, degree %d)",
                base->n, base->sh_degree, cur->n, cur->sh_degree);
  if (cur->n > GS_NOALLOC_MAX_N)
    return fail(c, GS_ERR_INVALID, "gs_delta_encode_noalloc: n=%d above GS_NOALLOC_MAX_N=%d", cur->n,
                (int)GS_NOALLOC_MAX_N);
  if ((s = check_codecs(c, codecs, "gs_delta_encode_noalloc")) != GS_OK) return s;
  if (!out || !epoch) return fail(c, GS_ERR_INVALID, "gs_delta_encode_noalloc: null output or epoch");
  if (mask & ~0x3Fu)
    return fail(c, GS_ERR_INVALID, "gs_delta_encode_noalloc: group_mask 0x%x has bits above 5", mask);
  const int64_t need = codec_capacity(cur->n, cur->sh_degree, codecs, mask);
  if (cap_words < need)
    return fail(c, GS_ERR_INVALID, "gs_delta_encode_noalloc: out_cap_words=%lld < %lld", (long long)cap_words,
                (long long)need);
  GS_HIP(c, launch_delta_encode_noalloc(c->device, *cur, *base, codecs, mask, epoch, out, st));
  return GS_OK;
}

gs_status gs_delta_apply(gs_ctx c, gs_params* model, const gs_codec* codecs, const uint32_t* packet,
                         int64_t packet_words, const uint32_t* epoch, uint32_t* status, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!model || model->n < 0 || model->sh_degree < 0 || model->sh_degree > 3)
    return fail(c, GS_ERR_INVALID, "gs_delta_apply: invalid model");
  if (model->n > 0 && (!model->mean || !model->log_scale || !model->quat || !model->opacity_logit || !model->sh))
    return fail(c, GS_ERR_INVALID, "gs_delta_apply: null model tensor");
  gs_status s;
  if ((s = check_codecs(c, codecs, "gs_delta_apply")) != GS_OK) return s;
  if (!packet || !epoch || !status || packet_words < 0)
    return fail(c, GS_ERR_INVALID, "gs_delta_apply: null packet, epoch or status");
  GS_HIP(c, launch_delta_apply(*model, codecs, packet, packet_words, epoch, status, st));
  return GS_OK;
}

gs_status gs_object_transform(gs_ctx c, gs_params* params, const int32_t* object_of, const gs_transform* tf,
                              int32_t n_objects, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  gs_status s;
  if ((s = check_tensor(c, params, "gs_object_transform(params)")) != GS_OK) return s;
  if (n_objects < 0) return fail(c, GS_ERR_INVALID, "gs_object_transform: n_objects=%d", n_objects);
  if (params->n > 0 && n_objects > 0 && (!object_of || !tf))
    return fail(c, GS_ERR_INVALID, "gs_object_transform: null object_of or transforms");
  GS_HIP(c, launch_object_transform(*params, object_of, tf, n_objects, st));
  return GS_OK;
}

gs_status gs_relight_dc(gs_ctx c, gs_params* params, const float* gain, int32_t channels, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  gs_status s;
  if ((s = check_tensor(c, params, "gs_relight_dc(params)")) != GS_OK) return s;
  if (channels != 1 && channels != 3) return fail(c, GS_ERR_INVALID, "gs_relight_dc: channels=%d", channels);
  if (params->n > 0 && !gain) return fail(c, GS_ERR_INVALID, "gs_relight_dc: null gain");
  GS_HIP(c, launch_relight_dc(*params, gain, channels, st));
  return GS_OK;
}

gs_status gs_append(gs_ctx c, const gs_params* old_p, const gs_params* old_m, const gs_params* old_v,
                    int32_t n_active, const gs_params* add, gs_params* new_p, gs_params* new_m, gs_params* new_v,
                    const uint32_t* const* old_cols, const uint32_t* const* add_cols, uint32_t* const* new_cols,
                    int32_t n_cols, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  gs_status s;
  if ((s = check_tensor(c, old_p, "gs_append(old_params)")) != GS_OK) return s;
  if ((s = check_tensor(c, add, "gs_append(add)")) != GS_OK) return s;
  if ((s = check_tensor(c, new_p, "gs_append(new_params)")) != GS_OK) return s;
  const int deg = old_p->sh_degree;
  if (add->sh_degree != deg || new_p->sh_degree != deg)
    return fail(c, GS_ERR_INVALID, "gs_append: SH degrees differ");
  if ((int64_t)new_p->n != (int64_t)old_p->n + add->n)
    return fail(c, GS_ERR_INVALID, "gs_append: new n=%d != old n %d + added %d", new_p->n, old_p->n, add->n);
  if (n_active < 0 || n_active > old_p->n)
    return fail(c, GS_ERR_INVALID, "gs_append: n_active=%d outside [0, %d]", n_active, old_p->n);
  const bool moments = old_m || old_v || new_m || new_v;
  if (moments) {
    if (!old_m || !old_v || !new_m || !new_v)
      return fail(c, GS_ERR_INVALID, "gs_append: give all four moment tensors or none");
    const gs_params* mv[4] = {old_m, old_v, new_m, new_v};
    const int32_t want[4] = {n_active, n_active, n_active + add->n, n_active + add->n};
    for (int q = 0; q < 4; ++q) {
      if ((s = check_tensor(c, mv[q], "gs_append(moments)")) != GS_OK) return s;
      if (mv[q]->n != want[q] || mv[q]->sh_degree != deg)
        return fail(c, GS_ERR_INVALID, "gs_append: moment tensor %d has n=%d, want %d", q, mv[q]->n, want[q]);
    }
  }
  if (n_cols < 0 || (n_cols > 0 && (!old_cols || !add_cols || !new_cols)))
    return fail(c, GS_ERR_INVALID, "gs_append: n_cols=%d with null column arrays", n_cols);
  for (int q = 0; q < n_cols; ++q)
    if ((old_p->n > 0 && !old_cols[q]) || (add->n > 0 && !add_cols[q]) || (new_p->n > 0 && !new_cols[q]))
      return fail(c, GS_ERR_INVALID, "gs_append: null column %d", q);
  GS_HIP(c, launch_append(*old_p, moments ? old_m : nullptr, moments ? old_v : nullptr, n_active, *add, *new_p,
                          moments ? new_m : nullptr, moments ? new_v : nullptr, old_cols, add_cols, new_cols, n_cols,
                          st));
  return GS_OK;
}

gs_status gs_delta_reset_baseline(gs_ctx c, const gs_params* cur, const gs_params* base, uint32_t* epoch,
                                  hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!cur || !base || !epoch) return fail(c, GS_ERR_INVALID, "gs_delta_reset_baseline: null argument");
  if (cur->n != base->n || cur->sh_degree != base->sh_degree || cur->sh_degree < 0 || cur->sh_degree > 3)
    return fail(c, GS_ERR_INVALID, "gs_delta_reset_baseline: tensors disagree on n / sh_degree");
  const size_t n = (size_t)cur->n;
  const size_t nk = (size_t)(cur->sh_degree + 1) * (cur->sh_degree + 1);
  if (n > 0) {
    GS_HIP(c, hipMemcpyAsync(base->mean, cur->mean, 12 * n, hipMemcpyDeviceToDevice, st));
    GS_HIP(c, hipMemcpyAsync(base->log_scale, cur->log_scale, 12 * n, hipMemcpyDeviceToDevice, st));
    GS_HIP(c, hipMemcpyAsync(base->quat, cur->quat, 16 * n, hipMemcpyDeviceToDevice, st));
    GS_HIP(c, hipMemcpyAsync(base->opacity_logit, cur->opacity_logit, 4 * n, hipMemcpyDeviceToDevice, st));
    GS_HIP(c, hipMemcpyAsync(base->sh, cur->sh, 12 * nk * n, hipMemcpyDeviceToDevice, st));
  }
  GS_HIP(c, launch_epoch_bump(epoch, st));
  return GS_OK;
}

gs_status gs_workspace_segment(gs_ctx c, int32_t which, int32_t v0, int32_t nv, size_t* offset, size_t* bytes) {
  if (!c || !offset || !bytes) return GS_ERR_INVALID;
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "gs_workspace_segment: no plan");
  const Plan& pl = c->plan;
  const WsLayout& L = pl.ws;
  const size_t vn = (size_t)L.vn;
  switch (which) {
    case GS_SEG_DEPTH: *offset = L.depth; *bytes = 4 * vn; break;
    case GS_SEG_COUNT: *offset = L.count; *bytes = 4 * vn; break;
    case GS_SEG_RECT: *offset = L.rect; *bytes = 8 * vn; break;
    case GS_SEG_RECORD: *offset = L.rec; *bytes = sizeof(float) * kRecFloats * vn; break;
    case GS_SEG_GRAD2D: *offset = L.g2; *bytes = sizeof(float) * kG2Fields * vn; break;
    case GS_SEG_SORTED_VALUES:
      if (v0 < 0 || nv < 1 || v0 + nv > pl.n_views) return fail(c, GS_ERR_INVALID, "gs_workspace_segment: range");
      *offset = sorted_values_in_b(pl, v0, nv) ? L.vals_b : L.vals_a;
      *bytes = 4 * (size_t)L.cap;
      break;
    case GS_SEG_RANGES: *offset = L.ranges; *bytes = 8 * (size_t)pl.total_tiles; break;
    case GS_SEG_LAST: *offset = L.last; *bytes = 4 * (size_t)pl.total_pixels; break;
    default: return fail(c, GS_ERR_INVALID, "gs_workspace_segment: unknown segment %d", which);
  }
  return GS_OK;
}

gs_status gs_profile_enable(gs_ctx c, int32_t on) {
  if (!c) return GS_ERR_INVALID;
  c->prof = on != 0;
  return GS_OK;
}

gs_status gs_profile_read(gs_ctx c, const char* stage, double* total_ms, int64_t* calls) {
  if (!c || !stage || !total_ms || !calls) return GS_ERR_INVALID;
  GS_HIP(c, flush_timers(c));
  for (int k = 0; k < kStages; ++k) {
    if (std::strcmp(stage, kStageNames[k]) == 0) {
      *total_ms = c->stage_ms[k];
      *calls = c->stage_calls[k];
      return GS_OK;
    }
  }
  return fail(c, GS_ERR_INVALID, "gs_profile_read: unknown stage '%s'", stage);
}

gs_status gs_profile_reset(gs_ctx c) {
  if (!c) return GS_ERR_INVALID;
  GS_HIP(c, flush_timers(c));
  for (int k = 0; k < kStages; ++k) {
    c->stage_ms[k] = 0.0;
    c->stage_calls[k] = 0;
  }
  return GS_OK;
}

gs_status gs_read_counters(gs_ctx c, const void* ws, hipStream_t st, gs_counters* out) {
  if (!c || !ws || !out) return GS_ERR_INVALID;
  if (!c->plan.valid) return fail(c, GS_ERR_INVALID, "gs_read_counters: no plan");
  GS_HIP(c, hipStreamSynchronize(st));
  Counters h{};
  GS_HIP(c, hipMemcpy(&h, seg<const char>(const_cast<void*>(ws), c->plan.ws.counters), sizeof(h),
                      hipMemcpyDeviceToHost));
  out->visible = h.nvis;
  out->keys = h.keys;
  out->key_capacity = c->plan.cap;
  out->overflow = h.overflow;
  out->overflow_any = (h.overflow_any | h.overflow) != 0u ? 1u : 0u;
  if (out->overflow_any) {
    // reported once here; the context keeps refusing to render until re-planned
    c->capacity_exceeded = true;
    const uint32_t zero = 0u;
    GS_HIP(c, hipMemcpy(seg<char>(const_cast<void*>(ws), c->plan.ws.counters + offsetof(Counters, overflow_any)),
                        &zero, sizeof(zero), hipMemcpyHostToDevice));
  }
  return GS_OK;
}

static gs_status run_step(gs_ctx c, const gs_step_args* a, hipStream_t st) {
  gs_status s;
  const Plan& pl = c->plan;
  if (!pl.valid) return fail(c, GS_ERR_INVALID, "gs_step: no plan");
  if (!a->dev_cams || !a->dev_target || !a->dev_images || !a->dev_T_final || !a->dev_n_contrib || !a->dev_loss ||
      !a->dev_step || !a->dev_workspace)
    return fail(c, GS_ERR_INVALID, "gs_step: null pointer in arguments");
  GS_HIP(c, launch_fill_u32(reinterpret_cast<uint32_t*>(a->dev_loss), 0u, 1, st));
  const int V = pl.n_views;
  const int nstep = a->plain ? V : 1;
  const int per = a->plain ? 1 : V;
  for (int k = 0; k < nstep; ++k) {
    const int v0 = k * per;
    if ((s = gs_project(c, &a->params, a->dev_cams, v0, per, a->dev_workspace, st)) != GS_OK) return s;
    if ((s = gs_build_tile_lists(c, v0, per, a->dev_workspace, st)) != GS_OK) return s;
    if ((s = gs_composite(c, v0, per, a->dev_workspace, a->dev_images, a->dev_T_final, a->dev_n_contrib, st)) !=
        GS_OK)
      return s;
    if ((s = gs_backward(c, &a->params, a->dev_cams, v0, per, a->dev_workspace, a->dev_images, a->dev_T_final,
                         a->dev_target, 1, &a->grads, k > 0 ? 1 : 0, a->dev_loss, st)) != GS_OK)
      return s;
  }
  if ((s = adam_step(c, &a->params, &a->grads, &a->adam_m, &a->adam_v, a->dev_step, &a->hp, a->dev_hp, st)) != GS_OK)
    return s;
  if (a->do_delta) {
    if ((s = gs_delta_extract(c, &a->params, &a->baseline, a->group_mask, a->rel_tau, a->dev_delta_out,
                              a->delta_cap_words, a->dev_workspace, st)) != GS_OK)
      return s;
  }
  return GS_OK;
}

gs_status gs_step(gs_ctx c, const gs_step_args* a, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!a) return fail(c, GS_ERR_INVALID, "gs_step: null arguments");
  gs_status s = check_capacity(c, "gs_step");
  if (s != GS_OK) return s;
  return run_step(c, a, st);
}

gs_status gs_step_capture(gs_ctx c, const gs_step_args* a, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!a) return fail(c, GS_ERR_INVALID, "gs_step_capture: null arguments");
  if (st == nullptr) return fail(c, GS_ERR_INVALID, "gs_step_capture: capture needs a non-default stream");
  if (check_capacity(c, "gs_step_capture") != GS_OK) return GS_ERR_CAPACITY;
  if (c->exec) { (void)hipGraphExecDestroy(c->exec); c->exec = nullptr; }
  if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
  GS_HIP(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  gs_status s = run_step(c, a, st);
  c->capturing = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(st, &g);
  if (s != GS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  GS_HIP(c, e);
  c->graph = g;
  GS_HIP(c, hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0));
  c->captured = *a;
  c->graph_gen = c->plan_gen;
  return GS_OK;
}

gs_status gs_step_launch(gs_ctx c, const gs_step_args* a, hipStream_t st) {
  if (!c) return GS_ERR_INVALID;
  c->err.clear();
  if (!a) return fail(c, GS_ERR_INVALID, "gs_step_launch: null arguments");
  if (!c->exec) return fail(c, GS_ERR_INVALID, "gs_step_launch: nothing captured");
  if (c->graph_gen != c->plan_gen || !same_args(*a, c->captured))
    return fail(c, GS_ERR_STALE, "gs_step_launch: arguments or plan changed since capture");
  if (check_capacity(c, "gs_step_launch") != GS_OK) return GS_ERR_CAPACITY;
  GS_HIP(c, hipGraphLaunch(c->exec, st));
  return GS_OK;
}

}  // extern "C"
