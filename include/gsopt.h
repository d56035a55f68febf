/*
 * gsopt: MI355X (gfx950) library for the online 3D Gaussian Splatting
 * optimize step and its streaming deltas.
 *
 * The method (Sec. 3.1, overview): the server repeatedly renders the current
 * Gaussian model from reference viewpoints, optionally grouped as
 * mini-batches, compares the result with the captured ground-truth images
 * under the configured loss, and updates the trainable parameters (means,
 * scales, quaternions, opacities, spherical-harmonic coefficients) with the
 * configured learning rates.  The optimized parameters are those of prior
 * 3DGS work (Sec. 3.2.3), i.e. EWA projection of each Gaussian and
 * front-to-back alpha compositing of depth-sorted splats per tile.  Changed
 * attributes are streamed as per-tensor deltas relative to the previously
 * transmitted state (Sec. 3.5).
 *
 * Conventions shared by every call
 *  - Every pointer named dev_* or inside gs_params is DEVICE memory owned by
 *    the caller; the library never allocates, frees or retains caller
 *    memory.  host_* pointers are host memory read during the call only.
 *  - Parameters are planar FP32 ("SoA"): mean[3][n], log_scale[3][n],
 *    quat[4][n] as (w,x,y,z), opacity_logit[n], sh[(D+1)^2*3][n] where row
 *    (k*3 + channel) holds SH coefficient k of that colour channel.
 *  - Every call enqueues asynchronously on the given stream and returns
 *    after host-side validation; it never synchronises the device unless
 *    its description says so.  A context is not thread-safe: use one per
 *    stream.
 *  - Errors: GS_ERR_INVALID for bad arguments (nothing is enqueued),
 *    GS_ERR_HIP for a HIP launch/runtime failure, GS_ERR_CAPACITY when a
 *    previous step reported key overflow and the plan was not enlarged,
 *    GS_ERR_STALE for a graph launch whose bound arguments changed,
 *    GS_ERR_UNSUPPORTED for an option outside the built kernels.
 *    gs_last_error() returns a message for the last failing call.
 *  - Key capacity: the number of (tile, Gaussian) keys is data dependent and
 *    is never synchronised on.  A tile-list build that needs more keys than
 *    the plan holds emits only the first key_capacity ones (their lists, and
 *    every image and gradient computed from them, are then invalid) and sets
 *    a device flag that stays set across later steps and graph replays.
 *    gs_read_counters reports and clears it and marks the context: from then
 *    on gs_project, gs_build_tile_lists, gs_composite, gs_backward, gs_step,
 *    gs_step_capture and gs_step_launch return GS_ERR_CAPACITY without
 *    enqueueing anything, until gs_plan is called again (with a larger
 *    key_capacity).
 */
#ifndef GSOPT_H
#define GSOPT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GS_OK = 0,
  GS_ERR_INVALID = -1,
  GS_ERR_CAPACITY = -2,
  GS_ERR_HIP = -3,
  GS_ERR_UNSUPPORTED = -4,
  GS_ERR_STALE = -5
} gs_status;

typedef struct gs_context* gs_ctx;

/* Gaussian model tensors (device pointers, layout above). sh_degree 0..3. */
typedef struct {
  float* mean;
  float* log_scale;
  float* quat;
  float* opacity_logit;
  float* sh;
  int32_t n;
  int32_t sh_degree;
} gs_params;

/* Pinhole reference camera, OpenCV axes (x right, y down, z forward).
 * A world point p maps to camera space x = R p + t (R row-major) and to
 * pixel (fx x0/x2 + cx, fy x1/x2 + cy); pixel (i, j) samples at
 * (i + 0.5, j + 0.5).  campos is the camera centre (for view-dependent
 * colour).  84 bytes, 4-byte aligned. */
typedef struct {
  float R[9];
  float t[3];
  float campos[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} gs_camera;

/* Rendering options fixed at plan time.
 *  tile_w, tile_h    : tile size in pixels, one of 8x8, 16x8, 16x16, 32x16, 32x32
 *  batch_depth       : splat records staged in LDS per batch: 32, 64, 128 or 256
 *  pixels_per_thread : 1, 2 or 4 (0 means 1); a workgroup has
 *                      tile_w*tile_h/pixels_per_thread threads
 *  wave_w            : width of the sub-tile one wavefront owns (0 = tile_w;
 *                      16 is also built for 32-wide tiles)
 *  schedule          : how the compositing kernels and their adjoint take
 *                      the call's tiles (all views of the call together):
 *                      0 = one workgroup per tile, tiles in row-major order;
 *                      1 = one workgroup per tile, each XCD a contiguous run;
 *                      2 = persistent: as many workgroups as are resident
 *                          at once, each taking tiles from a work queue in
 *                          row-major order until it is empty;
 *                      3 = persistent, the queue handing out the tiles with
 *                          the longest lists first (bucketed by the bit
 *                          length of the list length)
 *  Unsupported combinations give GS_ERR_UNSUPPORTED; results do not depend on
 *  tile size, batch depth, pixels per thread, wave shape or schedule.
 *  bg                : background colour added with the final transmittance
 *  loss_mode         : L1 reduction, 0 = sum over pixels and channels,
 *                      1 = mean per view (1/(3HW)), summed over views */
typedef struct {
  int32_t tile_w, tile_h;
  int32_t batch_depth;
  int32_t pixels_per_thread;
  int32_t wave_w;
  int32_t schedule;
  float bg[3];
  int32_t loss_mode;
} gs_render_opts;

/* Adam hyper-parameters (torch.optim.Adam semantics, no weight decay).
 * lr per parameter group: 0 mean, 1 log_scale, 2 quat, 3 opacity_logit,
 * 4 SH DC (rows 0..2 of sh), 5 SH higher bands (rows 3..). */
typedef struct {
  float lr[6];
  float beta1, beta2, eps;
} gs_adam_hparams;

/* Counters of the last step, read by gs_read_counters. */
typedef struct {
  int64_t visible;       /* visible (view, Gaussian) pairs */
  int64_t keys;          /* (tile, Gaussian) keys needed */
  int64_t key_capacity;  /* keys the plan can hold */
  uint32_t overflow;     /* 1 if the last build's keys > key_capacity (its outputs are invalid) */
  uint32_t overflow_any; /* 1 if any build since the previous gs_read_counters (or since
                            gs_workspace_init) overflowed; reading it marks the context
                            (GS_ERR_CAPACITY until the next gs_plan) */
} gs_counters;

/* ---- context ------------------------------------------------------------ */
gs_status gs_create(int32_t hip_device, gs_ctx* out);
gs_status gs_destroy(gs_ctx ctx);
/* Message of the last failing call on ctx (valid until the next call). */
const char* gs_last_error(gs_ctx ctx);

/* Fixes the frame layout for n Gaussians and n_views cameras: per-view
 * pixel and tile offsets (views concatenated in order, tiles row-major per
 * view), kernel variants, and the workspace size for up to key_capacity
 * (tile, Gaussian) keys.  Host-side only (a small library-owned device table
 * of view sizes is uploaded synchronously).  *workspace_bytes receives the
 * size of the caller-allocated workspace that every later call takes. */
gs_status gs_plan(gs_ctx ctx, int32_t n, int32_t sh_degree, int32_t n_views,
                  const gs_camera* host_cams, const gs_render_opts* opts,
                  int64_t key_capacity, size_t* workspace_bytes);

/* Prepares a freshly allocated workspace of the current plan (enqueued on
 * stream): clears the per-(view, Gaussian) screen-space gradient slots and
 * the counters.  Call once after allocating the workspace and before its
 * first use; later steps keep the slots cleared themselves (the projection
 * adjoint clears every slot it has consumed).  GS_ERR_INVALID without a plan
 * or with a NULL workspace. */
gs_status gs_workspace_init(gs_ctx ctx, void* workspace, hipStream_t stream);

/* Layout of the current plan: pixel_offsets[n_views+1] (pixel index of each
 * view's first pixel; images are planar CHW per view at 3*pixel_offsets[v])
 * and tile_offsets[n_views+1].  Either pointer may be NULL. */
gs_status gs_frame_layout(gs_ctx ctx, int64_t* pixel_offsets, int32_t* tile_offsets);

/* Stage "project/cull" (Sec. 3.1 render of the model; lineage EWA projection)
 * for views [view_begin, view_begin + view_count): per (view, Gaussian) the
 * FP32 depth key, the near/non-finite/off-screen cull, the screen-space
 * conic, the projected mean (as a float pair), opacity, SH colour and the
 * tile rectangle of the 3-sigma box.  dev_cams holds all planned views. */
gs_status gs_project(gs_ctx ctx, const gs_params* params, const gs_camera* dev_cams,
                     int32_t view_begin, int32_t view_count, void* dev_workspace, hipStream_t stream);

/* Stage "tile keys + sort + ranges": one key per (tile, visible Gaussian),
 * ordered by (tile, FP32 depth bits, Gaussian index) with a radix sort, then
 * [start, end) per tile.  Key count is data dependent: kernels are driven by
 * device-side counts and set the overflow flag instead of writing past the
 * plan's capacity. */
gs_status gs_build_tile_lists(gs_ctx ctx, int32_t view_begin, int32_t view_count,
                              void* dev_workspace, hipStream_t stream);

/* Stage "composite": per pixel, front-to-back alpha compositing of its tile's
 * list with the 3-sigma ellipse test, alpha = min(0.99, o e^P), skip below
 * 1/255, stop once transmittance would fall below 1e-4.  Writes images
 * (planar CHW per view at 3*pixel_offsets[v]), final transmittance and
 * contributor count per pixel (at pixel_offsets[v]); keeps the last list
 * position of each pixel and the strip bits of each list entry (which pixel
 * strips its splat may reach) internally for the backward pass. */
gs_status gs_composite(gs_ctx ctx, int32_t view_begin, int32_t view_count, void* dev_workspace,
                       float* dev_images, float* dev_T_final, uint32_t* dev_n_contrib,
                       hipStream_t stream);

/* Stage "backward": walks each pixel's list back to front from its last
 * composited entry, recomputing alphas and transmittance, accumulates the
 * per-(view, Gaussian) screen-space gradient, then applies the projection
 * chain rule and sums over the views of the call into grads.
 *  mode 0: dev_upstream is dL/dimage (image layout);
 *  mode 1: dev_upstream is the target image; L1 loss with the plan's
 *          loss_mode; *dev_loss (device FP32) receives the loss of these views.
 *  accumulate 0 writes grads, 1 adds to them.  dev_loss may be NULL in mode 0.
 * Active and frozen pools (Sec. 3.3, Gaussian freezing): grads->n may be
 * smaller than params->n.  Then only the first grads->n Gaussians (the
 * active pool) are differentiated, and grads rows are strided by grads->n;
 * the others (the frozen pool) are rendered and shape every pixel's
 * transmittance and colour as before but receive no gradient work.
 * The views of the call must have been projected by the latest gs_project
 * call (whose per-Gaussian visibility lets the adjoint skip Gaussians seen
 * in none of them). */
gs_status gs_backward(gs_ctx ctx, const gs_params* params, const gs_camera* dev_cams,
                      int32_t view_begin, int32_t view_count, void* dev_workspace,
                      const float* dev_images, const float* dev_T_final, const float* dev_upstream,
                      int32_t mode, const gs_params* grads, int32_t accumulate, float* dev_loss,
                      hipStream_t stream);

/* Fused Adam over all parameter tensors (configured learning rates,
 * Sec. 3.1).  *dev_step holds the number of steps taken so far; the update
 * uses t = *dev_step + 1 and a following kernel stores t.  grads, m and v
 * describe the active pool (n <= params->n, rows strided by their n): only
 * the first grads->n Gaussians of each parameter row are updated; frozen
 * Gaussians keep their values and need no moments (Sec. 3.3). */
gs_status gs_adam_step(gs_ctx ctx, const gs_params* params, const gs_params* grads,
                       const gs_params* m, const gs_params* v, int32_t* dev_step,
                       const gs_adam_hparams* hp, hipStream_t stream);

/* ---- preculling by grid cells (Sec. 3.3) ---------------------------------
 * A regular world grid of dims[0] x dims[1] x dims[2] cubic cells of edge
 * cell_size starting at origin; cell index = cx + dims[0] (cy + dims[1] cz).
 * Gaussians whose mean lies outside the grid belong to an extra cell,
 * index dims[0] dims[1] dims[2], which is never culled. */
typedef struct {
  float origin[3];
  float cell_size;
  int32_t dims[3];
  int32_t reserved;
} gs_grid;

/* Assigns every Gaussian (params->n) to its cell: cell_of[n] (device uint32)
 * and cell_sigma[n_cells + 1] (device uint32 holding FP32 bits: the largest
 * exp(log-scale) among the cell's Gaussians), both caller-owned. */
gs_status gs_assign_cells(gs_ctx ctx, const gs_params* params, const gs_grid* grid, uint32_t* cell_of,
                          uint32_t* cell_sigma, hipStream_t stream);

/* Per-view cell visibility for views [view_begin, view_begin + view_count):
 * mask[(v - view_begin) * (n_cells + 1) + c] = 1 unless no Gaussian of cell c
 * can be visible in view v (conservative: derived from the projection's own
 * visibility rule with the cell's largest scale, so culling never changes a
 * result).  Engines with their own visibility (a depth test) may write the
 * mask themselves instead. */
gs_status gs_visible_cells(gs_ctx ctx, const gs_grid* grid, const gs_camera* dev_cams, int32_t view_begin,
                           int32_t view_count, const uint32_t* cell_sigma, uint8_t* mask, hipStream_t stream);

/* Turns preculling on for later gs_project calls (and steps): Gaussian i is
 * skipped for view v when mask[v * (n_cells + 1) + cell_of[i]] == 0 (rows
 * for every view of the plan).  NULL pointers turn it off.  The pointers are
 * recorded, not their contents: the caller may rewrite the mask between
 * steps; changing the pointers invalidates a captured step graph, and a new
 * gs_plan turns preculling off. */
gs_status gs_set_precull(gs_ctx ctx, const uint32_t* cell_of, const uint8_t* mask, int32_t n_cells);

/* Moves active Gaussians into the frozen pool (Sec. 3.3: as regions become
 * stable their Gaussians leave the trainable set but stay renderable).
 * flags[i] != 0 (device bytes, i < m->n) marks active Gaussian i for
 * freezing.  In place, as a stable partition of the active prefix: the
 * Gaussians that stay active keep their order at the front, followed by the
 * newly frozen ones in their order, followed by the Gaussians frozen before
 * (unchanged).  The same permutation is applied to every row of params
 * (n = planned n), to baseline (optional, n = planned n) and to ids
 * (optional, uint32 per Gaussian, e.g. stable Gaussian IDs for the delta
 * stream).  m and v (n = current active count) are compacted to the new
 * active count n' (rows strided by n').  *new_active (device int32)
 * receives n'; after synchronising the caller describes grads, m and v with
 * n = n' (the same storage).  Enqueued on stream; uses the workspace. */
gs_status gs_freeze(gs_ctx ctx, gs_params* params, gs_params* m, gs_params* v, const uint8_t* flags,
                    uint32_t* ids, gs_params* baseline, void* dev_workspace, int32_t* new_active,
                    hipStream_t stream);

/* Reorders the model in place so that Gaussians are grouped by grid cell
 * (Sec. 3.3: Gaussians are assigned to cells and visibility is decided per
 * cell; keeping each cell's Gaussians together lets whole wavefronts of the
 * projection and its adjoints skip a culled cell).  A stable sort by
 * cell_of[i] (device uint32 per Gaussian, from gs_assign_cells; values of
 * n_cells or more sort as the outside cell n_cells), done separately within
 * the active prefix [0, m->n) and the frozen suffix, so the pools stay where
 * they are.  The permutation is applied to every row of params (n = planned
 * n), to baseline (optional), ids (optional, uint32 per Gaussian) and
 * cell_of itself, and to the first m->n entries of every row of m and v
 * (rows strided by m->n).  m and v may both be NULL (no optimizer state: the
 * whole model is one pool).  Results of later calls are unchanged except for
 * the order of Gaussians with equal depth keys.  Enqueued on stream; uses
 * the workspace (the projection's buffers: project again afterwards). */
gs_status gs_sort_cells(gs_ctx ctx, gs_params* params, gs_params* m, gs_params* v, uint32_t* cell_of,
                        int32_t n_cells, uint32_t* ids, gs_params* baseline, void* ws, hipStream_t stream);

/* ---- scene dynamics and expansion ---------------------------------------- */

/* Rigid motion of one object: x -> R (x - pivot) + pivot + t, R the rotation
 * of the quaternion q / |q| (w, x, y, z; q must be nonzero). */
typedef struct {
  float q[4];
  float pivot[3];
  float t[3];
} gs_transform;   /* 40 bytes */

/* Rigid-object dynamics (Sec. 3.4: Gaussians are tied to engine objects by
 * identifiers, and the objects' motion is applied to them before each
 * optimization).  For every Gaussian i with 0 <= object_of[i] < n_objects
 * (device int32 per Gaussian; other values: static), the mean moves by
 * dev_transforms[object_of[i]] (device array of n_objects) and the
 * orientation becomes (q / |q|) * quat (Hamilton product); scales, opacity
 * and colour do not change.  FP64 arithmetic, each stored value rounded once
 * to FP32.  In place on params (any n; no plan needed). */
gs_status gs_object_transform(gs_ctx ctx, gs_params* params, const int32_t* object_of,
                              const gs_transform* dev_transforms, int32_t n_objects, hipStream_t stream);

/* Relighting of the diffuse term (Sec. 3.4; the paper's full combination of
 * Gaussian SH with lighting SH is not specified, so only the DC colour is
 * rescaled): the DC colour C0 dc + 1/2 of Gaussian i and channel c becomes
 * gain[(channels == 3 ? c : 0) * n + i] times itself (device FP32, channels
 * 1 or 3 rows of n); a gain of exactly 1 leaves the coefficient unchanged.
 * FP64 arithmetic, rounded once.  In place on params->sh (any n). */
gs_status gs_relight_dc(gs_ctx ctx, gs_params* params, const float* dev_gain, int32_t channels,
                        hipStream_t stream);

/* Model expansion (Sec. 3.3: new Gaussians are appended to the trainable part
 * and the trainable tensors and optimizer state are extended): writes into
 * new_params (n = old n + add n) every row as the old active prefix
 * [0, n_active), then the add Gaussians, then the old frozen suffix; new_m
 * and new_v (n = n_active + add n) get the old moments followed by zeros
 * (old_m, old_v, new_m, new_v all NULL when there is no optimizer state;
 * old moments have n = n_active).  n_cols extra per-Gaussian uint32 columns
 * (IDs, object indices, cells) are extended the same way: old_cols[c] (old
 * n), add_cols[c] (add n), new_cols[c] (new n), host arrays of device
 * pointers.  Out of place; all tensors share the SH degree.  Afterwards the
 * caller plans for the new n (gs_plan) and, when streaming, sends a
 * snapshot. */
gs_status gs_append(gs_ctx ctx, const gs_params* old_params, const gs_params* old_m, const gs_params* old_v,
                    int32_t n_active, const gs_params* add, gs_params* new_params, gs_params* new_m,
                    gs_params* new_v, const uint32_t* const* old_cols, const uint32_t* const* add_cols,
                    uint32_t* const* new_cols, int32_t n_cols, hipStream_t stream);

/* Changed-Gaussian delta (Sec. 3.5: per-attribute tensor deltas relative to
 * the previously transmitted state, Gaussian-ID ordering).  Groups, in this
 * order and bit position of group_mask: 0 opacity (1 value), 1 SH DC (3),
 * 2 SH higher bands (3((D+1)^2-1)), 3 mean (3), 4 log_scale (3), 5 quat (4).
 * Row i of a masked group is emitted when some element has
 * fl32(|cur - base|) > fl32(rel_tau * |base|).  dev_out (uint32 words):
 * [6 counts], then per group in order: count indices ascending, followed by
 * count*width FP32 values row-major.  Emitted baseline rows are overwritten
 * with the current values.  out_cap_words must be at least
 * 6 + sum over masked groups of n*(1+width); otherwise GS_ERR_INVALID.
 * Uses the plan's workspace (n must equal the planned n). */
gs_status gs_delta_extract(gs_ctx ctx, const gs_params* cur, const gs_params* baseline,
                           uint32_t group_mask, float rel_tau, uint32_t* dev_out,
                           int64_t out_cap_words, void* dev_workspace, hipStream_t stream);

/* Delta codecs (Sec. 3.5: means and scales may be coded as residuals against
 * the previously transmitted state, the other attributes as quantized
 * updates; the codecs are configured per tensor before streaming).  Bit
 * widths, steps and rounding are not given by the paper; this library's
 * reading, per group with inv = fl32(1 / step), every operation a separately
 * rounded FP32 operation, rint rounding half to even, NaN codes 0:
 *   GS_CODEC_RAW       the rule of gs_delta_extract (rel_tau); FP32 values.
 *   GS_CODEC_RESIDUAL  c = clamp(rint((cur - base) inv), +-(2^(bits-1) - 1));
 *                      a row is sent when some c != 0; the baseline becomes
 *                      base + c step (closed loop: what the receiver rebuilds).
 *   GS_CODEC_QUANT     q(x) = clamp(rint((x - lo) inv), 0, 2^bits - 1); a row
 *                      is sent when some q(cur) != q(base); the baseline
 *                      becomes lo + q(cur) step.
 * bits is 8 or 16 for the coded modes; step > 0 with a finite 1/step. */
typedef enum { GS_CODEC_RAW = 0, GS_CODEC_RESIDUAL = 1, GS_CODEC_QUANT = 2 } gs_codec_mode;
typedef struct {
  int32_t mode;     /* gs_codec_mode */
  int32_t bits;     /* 8 or 16 (residual, quant); ignored for raw */
  float step;       /* quantization step (residual, quant) */
  float lo;         /* quant: the value of code 0 */
  float rel_tau;    /* raw: relative gate */
} gs_codec;         /* 20 bytes */

/* Words of the largest packet gs_delta_encode can write for n Gaussians of
 * degree sh_degree under codecs[6] and group_mask: 9 + sum over masked
 * groups of n (1 + row words), row words = width for raw, else
 * ceil(width / (32 / bits)).  Host only; -1 for an invalid codec. */
int64_t gs_codec_capacity_words(int32_t n, int32_t sh_degree, const gs_codec* codecs, uint32_t group_mask);

/* Coded tensor-delta packet for the masked groups (group order and bits as in
 * gs_delta_extract).  dev_out (uint32 words): [0] *dev_epoch (the
 * transmission epoch that gs_delta_reset_baseline advances), [1] group_mask,
 * [2..7] sent-row counts per group, [8] total words, then per masked group
 * in order: the ascending indices, then each sent row's words (raw: FP32
 * values; coded: codes packed little-endian, 32/bits per word, each row
 * starting on a word).  Baseline rows that are sent are updated to the
 * receiver's reconstruction.  out_cap_words below gs_codec_capacity_words
 * gives GS_ERR_INVALID.  Uses the plan's workspace (n = planned n). */
gs_status gs_delta_encode(gs_ctx ctx, const gs_params* cur, gs_params* baseline, const gs_codec* codecs,
                          uint32_t group_mask, const uint32_t* dev_epoch, uint32_t* dev_out, int64_t out_cap_words,
                          void* dev_workspace, hipStream_t stream);

/* Largest model (Gaussians) that gs_delta_encode_noalloc accepts. */
#define GS_NOALLOC_MAX_N (1 << 22)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * packet of gs_delta_encode, computed by the same kernels, without a plan or
 * a workspace.  Its scratch (a flag byte per Gaussian, per-block counts, scan
 * partials and section bases: about 4.6 MB) is a fixed device array of the
 * library, one per GPU, held until the process ends; gs_create looks up its
 * address on the context's device.  Arguments, packet layout and baseline
 * update as in gs_delta_encode; cur->n and baseline->n must be equal and at
 * most GS_NOALLOC_MAX_N (else GS_ERR_INVALID, nothing enqueued); n may
 * differ from call to call.  Calls this function makes: kernel launches
 * only, no hipMalloc, hipFree or other allocating call.  Every call on one
 * GPU shares that GPU's scratch: calls that overlap in time on one GPU (two
 * streams, two contexts, two threads) race and must be serialised by the
 * caller; calls enqueued in order on one stream are safe.  Nothing in the
 * scratch needs clearing between calls (each call writes every word it
 * reads). */
gs_status gs_delta_encode_noalloc(gs_ctx ctx, const gs_params* cur, gs_params* baseline, const gs_codec* codecs,
                                  uint32_t group_mask, const uint32_t* dev_epoch, uint32_t* dev_out,
                                  int64_t out_cap_words, hipStream_t stream);

/* Client replay (Sec. 3.5: the receiver keeps a local model and applies
 * incoming deltas): applies a gs_delta_encode packet (packet_words words on
 * the device, e.g. as received) to `model` with the sender's codecs.
 * *dev_status (device uint32) receives 0 when applied, else bits 1 (the
 * packet's epoch differs from *dev_epoch, the receiver's) and 2 (malformed:
 * shorter than its header says, mask bits above 5, rows in an unmasked
 * group, a count above n, an index >= n, or indices not strictly ascending
 * within a group); a packet with a nonzero status changes nothing.  Needs
 * no plan (any context); model->n is the receiver's Gaussian count. */
gs_status gs_delta_apply(gs_ctx ctx, gs_params* model, const gs_codec* codecs, const uint32_t* dev_packet,
                         int64_t packet_words, const uint32_t* dev_epoch, uint32_t* dev_status, hipStream_t stream);

/* Snapshot bookkeeping (Sec. 3.5): baseline := cur for every tensor and
 * *dev_epoch += 1. */
gs_status gs_delta_reset_baseline(gs_ctx ctx, const gs_params* cur, const gs_params* baseline,
                                  uint32_t* dev_epoch, hipStream_t stream);

/* Internal arrays of the current plan, for tests and tools (read-only use).
 * Per (view, Gaussian) pair, indexed v*n + i:
 *   GS_SEG_DEPTH   u32 FP32 depth-key bits (valid where COUNT > 0)
 *   GS_SEG_COUNT   u32 tiles touched, 0 when culled
 *   GS_SEG_RECT    4 x u16 tile rectangle (tx0, ty0, tx1, ty1), inclusive
 *   GS_SEG_RECORD  12 x f32 splat record (u_hi, w_hi, u_lo, w_lo, a, r, s, o,
 *                  red, green, blue, 0) with conic
 *                  P = -1/2 (a (dx + r dy)^2 + s dy^2)
 *   GS_SEG_GRAD2D  9 planes of [VN] f32 (field f of pair v*n + i at
 *                  f * VN + v*n + i, VN = n * planned views):
 *                  dL/d(u, w, a, b, c, o, red, green, blue) where (a, b, c)
 *                  is the conic [[a, b], [b, c]]; zero between steps
 * Per key / tile / pixel:
 *   GS_SEG_SORTED_VALUES  u32 v*n + i in (tile, depth, index) order for the
 *                         tile lists last built over [view_begin, +view_count)
 *   GS_SEG_RANGES         u32 pairs [start, end) per global tile
 *   GS_SEG_LAST           u32 one past the last composited list position per pixel
 * *offset and *bytes are byte offsets/sizes inside the workspace. */
typedef enum {
  GS_SEG_DEPTH = 0,
  GS_SEG_COUNT = 1,
  GS_SEG_RECT = 2,
  GS_SEG_RECORD = 3,
  GS_SEG_GRAD2D = 4,
  GS_SEG_SORTED_VALUES = 5,
  GS_SEG_RANGES = 6,
  GS_SEG_LAST = 7
} gs_segment;
gs_status gs_workspace_segment(gs_ctx ctx, int32_t which, int32_t view_begin, int32_t view_count,
                               size_t* offset, size_t* bytes);

/* Stage timers: HIP events recorded around each stage's kernels on the
 * stream of the call (eager calls only; capture ignores them).  Stages:
 * "project", "tile_lists", "composite", "composite_bwd", "project_bwd",
 * "adam", "delta".  gs_profile_read waits for the recorded events and returns
 * the total milliseconds and number of timed calls since the last reset;
 * unknown names give GS_ERR_INVALID. */
gs_status gs_profile_enable(gs_ctx ctx, int32_t on);
gs_status gs_profile_read(gs_ctx ctx, const char* stage, double* total_ms, int64_t* calls);
gs_status gs_profile_reset(gs_ctx ctx);

/* Synchronous: waits for `stream` and reads the counters of the last step.
 * When a build overflowed the key capacity since the previous read, sets
 * out->overflow_any, clears the workspace's sticky flag and marks ctx, so
 * that the rendering calls return GS_ERR_CAPACITY until the next gs_plan
 * (the read itself returns GS_OK). */
gs_status gs_read_counters(gs_ctx ctx, const void* dev_workspace, hipStream_t stream, gs_counters* out);

/* ---- whole optimize step ------------------------------------------------ */
typedef struct {
  gs_params params, grads, adam_m, adam_v;  /* same n and sh_degree */
  const gs_camera* dev_cams;                /* all planned views */
  const float* dev_target;                  /* target images, image layout */
  float* dev_images;
  float* dev_T_final;
  uint32_t* dev_n_contrib;
  float* dev_loss;                          /* 1 float */
  int32_t* dev_step;                        /* Adam step counter */
  void* dev_workspace;
  gs_adam_hparams hp;
  int32_t plain;        /* 0: batched (every stage covers all views in one launch);
                           1: plain (the same kernels one view per launch) */
  int32_t do_delta;     /* 1: run gs_delta_extract after Adam */
  gs_params baseline;   /* delta baselines (if do_delta) */
  uint32_t group_mask;
  float rel_tau;
  uint32_t* dev_delta_out;
  int64_t delta_cap_words;
  const gs_adam_hparams* dev_hp;  /* optional (NULL: use hp): Adam hyper-parameters in device
                                     memory, read by the update kernels each time the step runs,
                                     so a captured step follows learning-rate changes the caller
                                     writes there between replays (hp is then only validated) */
} gs_step_args;

/* Enqueues one optimize step: project, tile lists, composite, L1 backward
 * (gradients summed over all views, Sec. 3.1 mini-batch), Adam, optional
 * delta extraction. */
gs_status gs_step(gs_ctx ctx, const gs_step_args* args, hipStream_t stream);

/* Captures gs_step(args) (batched or plain) into a HIP graph owned by ctx.
 * The stream must be a non-default stream. */
gs_status gs_step_capture(gs_ctx ctx, const gs_step_args* args, hipStream_t stream);

/* Replays the captured graph.  Returns GS_ERR_STALE without launching if any
 * field of *args differs from the captured arguments (hp excepted when
 * dev_hp is set) or the plan changed.  Contents of device buffers (cameras,
 * targets, dev_hp) may change between replays. */
gs_status gs_step_launch(gs_ctx ctx, const gs_step_args* args, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* GSOPT_H */
