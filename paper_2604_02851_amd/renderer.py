"""Renderer, autograd wrapper and optimize step over the gsopt C ABI.

PyTorch supplies device memory and streams only; every stage of the path
(project/cull, tile lists, composite, backward, Adam, delta) runs in
libgsopt.so.
"""
from __future__ import annotations

import os

import numpy as np
import torch

from . import native as N
from .native import Context, DeviceParams, GsAdamHparams, GsParams, GsStepArgs

# Learning rates per parameter group: mean, log_scale, quat, opacity_logit,
# SH DC, SH higher bands.
DEFAULT_LR = (1e-3, 5e-3, 1e-3, 5e-2, 5e-3, 5e-3)


class Renderer:
    """A planned frame: cameras, tile layout, workspace and output buffers."""

    def __init__(self, cams: np.ndarray, n: int, sh_degree: int, tile=(16, 16), batch_depth: int = 64,
                 bg=(0.0, 0.0, 0.0), loss_mode: int = 0, key_capacity: int | None = None, device: int = 0,
                 ctx: Context | None = None, pixels_per_thread: int = 1, wave_w: int = 0, schedule: int = 0):
        self.device = torch.device("cuda", device)
        self.ctx = ctx or Context(device)
        self.cams = np.ascontiguousarray(cams)
        self.n, self.sh_degree = n, sh_degree
        self.tile, self.batch_depth, self.bg, self.loss_mode = tuple(tile), batch_depth, tuple(bg), loss_mode
        self.ppt, self.wave_w, self.schedule = pixels_per_thread, wave_w or tile[0], schedule
        self.dev_cams = torch.from_numpy(self.cams.view(np.uint8).copy()).to(self.device)
        self.key_capacity = int(key_capacity or max(1 << 16, 8 * n * len(self.cams)))
        self.max_need = 0          # largest key count any fit_capacity call has seen
        # incremented whenever the workspace's lists and per-pixel state change
        self.forward_count = 0
        self._plan()
        P = int(self.pix_off[-1])
        self.images = torch.zeros(3 * P, dtype=torch.float32, device=self.device)
        self.T = torch.zeros(P, dtype=torch.float32, device=self.device)
        self.n_contrib = torch.zeros(P, dtype=torch.int32, device=self.device)

    @property
    def n_views(self) -> int:
        return len(self.cams)

    def _plan(self):
        nbytes = self.ctx.plan(self.n, self.sh_degree, self.cams, self.tile, self.batch_depth, self.bg,
                               self.loss_mode, self.key_capacity, self.ppt, self.wave_w, self.schedule)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ctx.workspace_init(self.ws)
        self.capacity_exceeded = False
        self.pix_off, self.tile_off = self.ctx.frame_layout()
        if getattr(self, "precull", None) is not None:   # a new plan turns preculling off: restore it
            self.ctx.set_precull(*self.precull)

    def enable_precull(self, params: DeviceParams, origin, cell_size: float, dims, update_mask: bool = True):
        """Preculling by grid cells (Sec. 3.3): assigns the Gaussians to the
        cells of the grid and lets the projection skip, per view, the cells
        that view cannot see (conservative: results do not change).  Returns
        (cell_of, mask); call update_precull() after the cameras or the model
        move."""
        g = N.GsGrid((N.c_float * 3)(*origin), float(cell_size), (N.c_int32 * 3)(*dims), 0)
        n_cells = int(dims[0]) * int(dims[1]) * int(dims[2])
        self.grid, self.n_cells = g, n_cells
        self.cell_of = torch.zeros(max(params.n, 1), dtype=torch.int32, device=self.device)
        self.cell_sigma = torch.zeros(n_cells + 1, dtype=torch.int32, device=self.device)
        self.cell_mask = torch.ones(self.n_views * (n_cells + 1), dtype=torch.uint8, device=self.device)
        self.update_precull(params)
        self.precull = (self.cell_of, self.cell_mask, n_cells)
        self.ctx.set_precull(*self.precull)
        return self.cell_of, self.cell_mask

    def update_precull(self, params: DeviceParams, stream=None):
        self.ctx.assign_cells(params, self.grid, self.cell_of, self.cell_sigma, stream)
        self.ctx.visible_cells(self.grid, self.dev_cams, 0, self.n_views, self.cell_sigma, self.cell_mask, stream)

    def sort_cells(self, params: DeviceParams, stream=None, **state):
        """Reorders the model in place so that Gaussians are grouped by grid
        cell (stable, within the active and frozen pools), refreshing the cell
        assignment and the cell mask first; needs enable_precull()'s grid.  `state` passes the
        optimizer's m, v, ids and baseline, permuted alike.  Results change
        only in the order of Gaussians with equal depth keys."""
        assert getattr(self, "grid", None) is not None, "sort_cells needs the grid of enable_precull()"
        self.forward_count += 1     # the regrouping reuses the projection's buffers
        self.update_precull(params, stream)
        self.ctx.sort_cells(params, self.cell_of, self.n_cells, self.ws, stream=stream, **state)

    def disable_precull(self):
        self.precull = None
        self.ctx.set_precull(None, None, 0)

    def resize(self, n: int):
        """Plans the frame for a model of n Gaussians (after appending): new
        workspace; the cell assignment buffer of preculling grows with it
        (call update_precull() before the next step)."""
        self.n = int(n)
        if getattr(self, "precull", None) is not None:
            self.cell_of = torch.zeros(max(self.n, 1), dtype=torch.int32, device=self.device)
            self.precull = (self.cell_of, self.cell_mask, self.n_cells)
        self.ws = None
        self._plan()

    def replan(self, key_capacity: int):
        self.key_capacity = int(key_capacity)
        self.ws = None
        self._plan()

    def view_image(self, images: torch.Tensor, v: int) -> torch.Tensor:
        H, W = int(self.cams[v]["height"]), int(self.cams[v]["width"])
        return images[3 * self.pix_off[v]: 3 * self.pix_off[v + 1]].view(3, H, W)

    def counters(self):
        """The counters of the last step (synchronises).  When a build
        overflowed the key capacity since the previous read, overflow_any is
        set and the context refuses to render (GsError GS_ERR_CAPACITY) until
        replan()."""
        c = self.ctx.read_counters(self.ws)
        if c.overflow_any:
            self.capacity_exceeded = True
        return c

    def check_capacity(self):
        """Raises GsError(GS_ERR_CAPACITY) when a tile-list build since the
        last read overflowed the key capacity (its outputs were invalid)."""
        c = self.counters()
        if c.overflow_any:
            raise N.GsError(N.GS_ERR_CAPACITY, f"a tile-list build needed {int(c.keys)} keys of a capacity of "
                                               f"{int(c.key_capacity)}: replan() with a larger capacity")
        return c

    def fit_capacity(self, params: DeviceParams, per_view: bool = False, margin: float = 1.15):
        """Runs project + tile lists for `params` (all views at once, or one
        view per call) and re-plans when the key capacity is short of the
        largest need this renderer has seen, or far above it (sort grids and
        histogram scans are sized by the capacity).  Capacity never drops
        below a need seen before, so fitting several models (targets, then
        the trained model) leaves room for all of them.  Returns this
        model's need."""
        if self.capacity_exceeded:   # an overflow was reported: the context needs a new plan first
            self.replan(self.key_capacity)
        need = 0
        ranges = [(v, 1) for v in range(self.n_views)] if per_view else [(0, self.n_views)]
        for v0, nv in ranges:
            self.forward_count += 1
            self.ctx.project(params, self.dev_cams, v0, nv, self.ws)
            self.ctx.build_tile_lists(v0, nv, self.ws)
            c = self.counters()
            need = max(need, int(c.keys))
            if c.overflow_any:      # the context renders again only after a new plan
                self.replan(max(1024, int(need * margin) + 1024))
        self.max_need = max(self.max_need, need)
        if self.max_need > self.key_capacity or self.max_need * margin * 1.5 < self.key_capacity:
            self.replan(max(1024, int(self.max_need * margin) + 1024))
        return need

    # ---- stages -------------------------------------------------------------
    def forward(self, params: DeviceParams, v0: int = 0, nv: int | None = None):
        nv = self.n_views - v0 if nv is None else nv
        self.forward_count += 1
        self.ctx.project(params, self.dev_cams, v0, nv, self.ws)
        self.ctx.build_tile_lists(v0, nv, self.ws)
        self.ctx.composite(v0, nv, self.ws, self.images, self.T, self.n_contrib)
        return self.images, self.T, self.n_contrib

    def backward(self, params: DeviceParams, upstream: torch.Tensor, mode: int, grads: DeviceParams,
                 v0: int = 0, nv: int | None = None, accumulate: int = 0, loss: torch.Tensor | None = None):
        nv = self.n_views - v0 if nv is None else nv
        self.ctx.backward(params, self.dev_cams, v0, nv, self.ws, self.images, self.T, upstream, mode, grads,
                          accumulate, loss)


class GaussianRasterize(torch.autograd.Function):
    """images = render(params) over every view of `renderer`, with the
    hand-written adjoint of the library as backward.  The renderer keeps the
    tile lists and per-pixel state of the last forward only, so a backward
    must follow its own forward before the renderer runs another one (or an
    optimize step, a capacity fit or a regrouping); otherwise the backward
    raises instead of returning gradients of another forward."""

    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity_logit, sh, renderer: Renderer):
        params = DeviceParams(mean.detach().contiguous(), log_scale.detach().contiguous(),
                              quat.detach().contiguous(), opacity_logit.detach().contiguous(),
                              sh.detach().contiguous(), renderer.sh_degree)
        images, T, _ = renderer.forward(params)
        ctx.renderer = renderer
        ctx.forward_id = renderer.forward_count
        ctx.params = params
        out = images.clone()
        ctx.save_for_backward(out)
        return out

    @staticmethod
    def backward(ctx, grad_images):
        r: Renderer = ctx.renderer
        if r.forward_count != ctx.forward_id:
            raise RuntimeError("GaussianRasterize.backward: the renderer has run another forward pass since this "
                               "one (its tile lists and per-pixel state belong to that pass); use one renderer per "
                               "pending backward")
        (images,) = ctx.saved_tensors
        grads = DeviceParams.zeros_like(ctx.params)
        up = grad_images.contiguous().float()
        r.ctx.backward(ctx.params, r.dev_cams, 0, r.n_views, r.ws, images, r.T, up, 0, grads, 0, None)
        return (*grads.tensors(), None)


def rasterize(params_tensors, renderer: Renderer):
    return GaussianRasterize.apply(*params_tensors, renderer)


class Optimizer:
    """Online optimize step (render reference views, L1 against targets,
    backward, Adam), batched or plain, eager or replayed from a HIP graph."""

    def __init__(self, renderer: Renderer, params: DeviceParams, targets: torch.Tensor, lr=DEFAULT_LR,
                 betas=(0.9, 0.999), eps=1e-15, stream: torch.cuda.Stream | None = None, n_active: int | None = None):
        """n_active: the first n_active Gaussians form the active (trainable)
        pool, the rest the frozen pool (rendered, not optimised)."""
        self.r = renderer
        self.params = params
        self.targets = targets.contiguous()
        na = params.n if n_active is None else int(n_active)
        dev = renderer.device
        self.grads = DeviceParams.zeros(na, params.sh_degree, dev)
        self.m = DeviceParams.zeros(na, params.sh_degree, dev)
        self.v = DeviceParams.zeros(na, params.sh_degree, dev)
        self.ids = None
        self.step_count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.lr, self.betas, self.eps = tuple(lr), tuple(betas), eps
        self.stream = stream
        # the hyper-parameters also live in device memory (gs_adam_hparams
        # layout), where the update kernels read them each time a step runs:
        # set_hparams changes them without recapturing the step
        self.hp_dev = torch.zeros(9, dtype=torch.float32, device=dev)
        self._write_hparams()
        self.delta = None
        self._args_cache = {}

    def _write_hparams(self):
        host = torch.tensor(list(self.lr) + [self.betas[0], self.betas[1], self.eps], dtype=torch.float32)
        with torch.cuda.stream(self.stream or torch.cuda.current_stream()):
            self.hp_dev.copy_(host)

    def set_hparams(self, lr=None, betas=None, eps=None):
        """New learning rates (six groups), betas or eps for the following
        steps, eager or replayed (enqueued on the optimizer's stream)."""
        if lr is not None:
            assert len(lr) == 6
            self.lr = tuple(float(x) for x in lr)
        if betas is not None:
            self.betas = tuple(float(x) for x in betas)
        if eps is not None:
            self.eps = float(eps)
        if not (all(0.0 <= b < 1.0 for b in self.betas) and self.eps >= 0.0):
            raise ValueError("betas must lie in [0, 1) and eps >= 0")
        self._write_hparams()

    def enable_delta(self, baseline: DeviceParams, group_mask: int = 0x3F, rel_tau: float = 1e-3):
        words = N.delta_capacity_words(self.params.n, self.params.sh_degree, group_mask)
        self.delta = dict(baseline=baseline, mask=group_mask, tau=rel_tau,
                          out=torch.zeros(words, dtype=torch.int32, device=self.r.device))
        self._args_cache.clear()

    def args(self, plain: bool) -> GsStepArgs:
        key = bool(plain)
        if key in self._args_cache:
            return self._args_cache[key]
        a = GsStepArgs()
        a.params, a.grads, a.adam_m, a.adam_v = (x.struct() for x in (self.params, self.grads, self.m, self.v))
        a.dev_cams = N.ptr(self.r.dev_cams)
        a.dev_target = N.ptr(self.targets)
        a.dev_images = N.ptr(self.r.images)
        a.dev_T_final = N.ptr(self.r.T)
        a.dev_n_contrib = N.ptr(self.r.n_contrib)
        a.dev_loss = N.ptr(self.loss)
        a.dev_step = N.ptr(self.step_count)
        a.dev_workspace = N.ptr(self.r.ws)
        a.hp = GsAdamHparams((N.c_float * 6)(*self.lr), self.betas[0], self.betas[1], self.eps)
        a.dev_hp = N.ptr(self.hp_dev)
        a.plain = 1 if plain else 0
        if self.delta is not None:
            a.do_delta = 1
            a.baseline = self.delta["baseline"].struct()
            a.group_mask = self.delta["mask"]
            a.rel_tau = self.delta["tau"]
            a.dev_delta_out = N.ptr(self.delta["out"])
            a.delta_cap_words = self.delta["out"].numel()
        self._args_cache[key] = a
        return a

    def invalidate(self):
        self._args_cache.clear()

    @property
    def n_active(self) -> int:
        return self.grads.n

    def freeze(self, flags: torch.Tensor) -> int:
        """Moves the active Gaussians with flags[i] != 0 (uint8, one per active
        Gaussian) into the frozen pool; parameters, delta baseline and ids are
        permuted in place, moments compacted.  Synchronises; returns the new
        active count.  A captured graph must be captured again afterwards."""
        assert flags.dtype == torch.uint8 and flags.numel() == self.n_active and flags.is_contiguous()
        out = torch.zeros(1, dtype=torch.int32, device=self.r.device)
        base = self.delta["baseline"] if self.delta is not None else None
        self.r.ctx.freeze(self.params, self.m, self.v, flags, self.r.ws, out, ids=self.ids, baseline=base,
                          stream=self.stream)
        (self.stream or torch.cuda.current_stream()).synchronize()
        na = int(out.item())
        self.grads, self.m, self.v = (x.narrowed(na) for x in (self.grads, self.m, self.v))
        self._args_cache.clear()
        return na

    def sort_cells(self):
        """Groups the model by grid cell (Renderer.sort_cells) together with
        the moments, ids and delta baseline.  Buffers stay where they are, so
        a captured graph remains valid."""
        base = self.delta["baseline"] if self.delta is not None else None
        self.r.sort_cells(self.params, stream=self.stream, m=self.m, v=self.v, ids=self.ids, baseline=base)

    def append(self, add: DeviceParams, add_ids: torch.Tensor | None = None) -> DeviceParams:
        """Model expansion: appends `add` to the end of the active pool
        (ahead of the frozen pool), extends the moments with zeros, the ids
        (`add_ids`, default: continuing after the largest id) and the delta
        baseline (with the new values: send a snapshot), and re-plans the
        renderer for the new size.  Returns the new parameters, which
        replace `params` (the old tensors are no longer used).  Synchronises;
        a captured graph must be captured again."""
        dev, deg = self.r.device, self.params.sh_degree
        n, na, k = self.params.n, self.n_active, add.n
        new_p = DeviceParams.zeros(n + k, deg, dev)
        new_m, new_v = DeviceParams.zeros(na + k, deg, dev), DeviceParams.zeros(na + k, deg, dev)
        cols = []
        if self.ids is not None:
            if add_ids is None:
                start = int(self.ids.max().item()) + 1 if n > 0 else 0
                add_ids = torch.arange(start, start + k, dtype=self.ids.dtype, device=dev)
            new_ids = torch.zeros(n + k, dtype=self.ids.dtype, device=dev)
            cols.append((self.ids, add_ids.contiguous(), new_ids))
        self.r.ctx.append(self.params, add, new_p, na, moments=(self.m, self.v, new_m, new_v), cols=cols,
                          stream=self.stream)
        if self.delta is not None:
            nb = DeviceParams.zeros(n + k, deg, dev)
            self.r.ctx.append(self.delta["baseline"], add, nb, na, stream=self.stream)
            self.delta["baseline"] = nb
            words = N.delta_capacity_words(n + k, deg, self.delta["mask"])
            self.delta["out"] = torch.zeros(words, dtype=torch.int32, device=dev)
        (self.stream or torch.cuda.current_stream()).synchronize()
        self.params, self.m, self.v = new_p, new_m, new_v
        self.grads = DeviceParams.zeros(na + k, deg, dev)
        if cols:
            self.ids = cols[0][2]
        self.r.resize(n + k)
        if getattr(self.r, "precull", None) is not None:
            self.r.update_precull(self.params, self.stream)
        self.r.fit_capacity(self.params)
        self._args_cache.clear()
        return new_p

    def step(self, plain: bool = False):
        self.r.forward_count += 1
        self.r.ctx.step(self.args(plain), self.stream)

    def capture(self, plain: bool = False):
        self.r.ctx.step_capture(self.args(plain), self.stream)

    def replay(self, plain: bool = False):
        """Replays the captured step.  Raises GsError GS_ERR_CAPACITY once a
        counter read (check_capacity, or Renderer.counters) has found a key
        overflow, until the renderer is re-planned and the step captured
        again."""
        self.r.forward_count += 1
        self.r.ctx.step_launch(self.args(plain), self.stream)

    def check_capacity(self):
        """Synchronises and raises GsError(GS_ERR_CAPACITY) if any step since
        the last check overflowed the key capacity."""
        (self.stream or torch.cuda.current_stream()).synchronize()
        return self.r.check_capacity()


# ---------------------------------------------------------------------------
# Autotuner: launch shape of the compositing kernels, timed on the actual
# workload and cached by (device arch, Gaussian-count bucket, view-set
# signature).
# ---------------------------------------------------------------------------
# Built (tile, pixels per thread, wave sub-tile width) combinations, batch
# depths and tile schedules (0/1: one workgroup per tile, row-major or
# XCD-contiguous; 2/3: persistent workgroups on a work queue, row-major or
# longest lists first).
TUNE_SHAPES = (((8, 8), 1, 8), ((16, 8), 1, 16), ((16, 8), 2, 16), ((16, 16), 1, 16), ((16, 16), 2, 16),
               ((16, 16), 4, 16), ((32, 16), 1, 32), ((32, 16), 2, 32), ((32, 16), 4, 32), ((32, 16), 2, 16),
               ((32, 16), 4, 16), ((32, 32), 1, 32), ((32, 32), 2, 32), ((32, 32), 4, 32), ((32, 32), 2, 16),
               ((32, 32), 4, 16))
TUNE_BATCHES = (32, 64, 128, 256)
TUNE_SCHEDULES = (0, 1, 2, 3)
SHAPE_KEYS = ("tile", "batch_depth", "pixels_per_thread", "wave_w", "schedule")


def tune_search(time_of, shapes=TUNE_SHAPES, batches=TUNE_BATCHES, schedules=TUNE_SCHEDULES, start_batch=64,
                start_schedule=0, recheck: int = 3):
    """Coordinate search over the launch shape: every (tile, pixels per
    thread, wave width) at the starting batch depth and schedule, then every
    batch depth for the best of those, then every schedule, then the
    runners-up of the first stage again with the chosen batch depth and
    schedule.  time_of(candidate) -> ms per step, candidate = (tile, batch
    depth, pixels per thread, wave width, schedule); each candidate is timed
    once.  Returns (best candidate, {candidate: ms})."""
    times = {}

    def t(c):
        if c not in times:
            times[c] = time_of(c)
        return times[c]

    stage1 = sorted(((tile, start_batch, ppt, sw, start_schedule) for tile, ppt, sw in shapes), key=t)
    best = stage1[0]
    best = min(((best[0], b, best[2], best[3], best[4]) for b in batches), key=t)
    best = min(((best[0], best[1], best[2], best[3], sc) for sc in schedules), key=t)
    for c in stage1[1:1 + recheck]:
        t((c[0], best[1], c[2], c[3], best[4]))
    return min(times, key=times.get), times


def _tune_key(cams, n, sh_degree, device=0):
    import hashlib
    arch = torch.cuda.get_device_properties(device).gcnArchName if torch.cuda.is_available() else "cpu"
    sig = hashlib.sha256(np.ascontiguousarray(cams).tobytes()).hexdigest()[:16]
    bucket = 1 << max(0, int(n - 1).bit_length())
    return f"{arch}|n<={bucket}|sh{sh_degree}|views{len(cams)}|{sig}"


def _cache_path():
    return os.environ.get("GSOPT_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "gsopt", "tune.json"))


def autotune(cams, params: DeviceParams, target_params: DeviceParams, stream=None, steps: int = 3, log=print,
             use_cache: bool = True, **search) -> dict:
    """Times the batched optimize step (eager, `steps` steps after one
    warm-up) for the launch shapes tune_search visits and returns the fastest
    as Renderer keyword arguments; the parameters given are not modified."""
    import json
    key = _tune_key(cams, params.n, params.sh_degree)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except Exception:
            cache = {}
    hit = cache.get(key)
    if hit and all(k in hit for k in SHAPE_KEYS):
        res = {k: hit[k] for k in SHAPE_KEYS}
        res["tile"] = tuple(res["tile"])
        return dict(res, cached=True, times=hit.get("times"))
    state = {"ctx": None}

    def time_of(cand):
        shape = dict(zip(SHAPE_KEYS, cand))
        r = Renderer(cams, params.n, params.sh_degree, loss_mode=1, ctx=state["ctx"], **shape)
        state["ctx"] = r.ctx
        r.fit_capacity(target_params)
        r.fit_capacity(params)
        targets = r.forward(target_params)[0].clone()
        opt = Optimizer(r, params.clone(), targets, stream=stream)
        opt.step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s = stream or torch.cuda.current_stream()
        e0.record(s)
        for _ in range(steps):
            opt.step()
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        log(f"[autotune] tile/batch/px-per-thread/wave-width/schedule {_shape_name(cand)}: {ms:.3f} ms/step")
        del opt, r, targets
        torch.cuda.empty_cache()
        return ms

    best, times = tune_search(time_of, **search)
    res = dict(zip(SHAPE_KEYS, best))
    times = {_shape_name(c): round(ms, 3) for c, ms in times.items()}
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            cache[key] = dict(res, tile=list(best[0]), times=times)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return dict(res, cached=False, times=times)


def _shape_name(c) -> str:
    return "{}x{}/{}/{}/{}/{}".format(*c[0], *c[1:])
