"""ctypes binding of libgsopt.so (include/gsopt.h): argument marshalling only.

Every stage runs in the HIP library; this module only converts torch device
tensors into raw pointers and streams.  Loading fails loudly when the library
has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_int64, c_size_t, c_uint32, c_void_p

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsopt.so")

GS_OK, GS_ERR_INVALID, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_UNSUPPORTED, GS_ERR_STALE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "GS_OK", -1: "GS_ERR_INVALID", -2: "GS_ERR_CAPACITY", -3: "GS_ERR_HIP",
                -4: "GS_ERR_UNSUPPORTED", -5: "GS_ERR_STALE"}

EXPORTED = ("gs_create", "gs_destroy", "gs_last_error", "gs_plan", "gs_frame_layout", "gs_workspace_init", "gs_project",
            "gs_build_tile_lists", "gs_composite", "gs_backward", "gs_adam_step", "gs_delta_extract",
            "gs_delta_reset_baseline", "gs_codec_capacity_words", "gs_delta_encode", "gs_delta_encode_noalloc", "gs_delta_apply", "gs_object_transform", "gs_relight_dc", "gs_append", "gs_freeze", "gs_sort_cells", "gs_assign_cells", "gs_visible_cells", "gs_set_precull",
            "gs_workspace_segment", "gs_read_counters", "gs_step", "gs_step_capture",
            "gs_step_launch", "gs_profile_enable", "gs_profile_read", "gs_profile_reset")
STAGES = ("project", "tile_lists", "composite", "composite_bwd", "project_bwd", "adam", "delta")
SEG = {"depth": 0, "count": 1, "rect": 2, "record": 3, "grad2d": 4, "sorted_values": 5, "ranges": 6, "last": 7}


class GsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class GsParams(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("log_scale", c_void_p), ("quat", c_void_p),
                ("opacity_logit", c_void_p), ("sh", c_void_p), ("n", c_int32), ("sh_degree", c_int32)]


class GsRenderOpts(ctypes.Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("batch_depth", c_int32), ("pixels_per_thread", c_int32),
                ("wave_w", c_int32), ("schedule", c_int32), ("bg", c_float * 3), ("loss_mode", c_int32)]


class GsAdamHparams(ctypes.Structure):
    _fields_ = [("lr", c_float * 6), ("beta1", c_float), ("beta2", c_float), ("eps", c_float)]


class GsGrid(ctypes.Structure):
    _fields_ = [("origin", c_float * 3), ("cell_size", c_float), ("dims", c_int32 * 3), ("reserved", c_int32)]


class GsCodec(ctypes.Structure):
    _fields_ = [("mode", c_int32), ("bits", c_int32), ("step", c_float), ("lo", c_float), ("rel_tau", c_float)]


CODEC_RAW, CODEC_RESIDUAL, CODEC_QUANT = 0, 1, 2


class GsTransform(ctypes.Structure):
    _fields_ = [("q", c_float * 4), ("pivot", c_float * 3), ("t", c_float * 3)]


def transforms_tensor(transforms, device="cuda") -> torch.Tensor:
    """[(q (w, x, y, z), pivot, t), ...] -> a device buffer of gs_transform."""
    a = np.asarray([list(q) + list(p) + list(t) for q, p, t in transforms], np.float32).reshape(-1, 10)
    return torch.from_numpy(a.copy()).to(device)


def codec_array(codecs):
    """Six (mode, bits, step, lo, rel_tau) tuples -> a gs_codec[6] array."""
    assert len(codecs) == 6
    return (GsCodec * 6)(*[GsCodec(int(m), int(b), float(st), float(lo), float(t)) for m, b, st, lo, t in codecs])


class GsCounters(ctypes.Structure):
    _fields_ = [("visible", c_int64), ("keys", c_int64), ("key_capacity", c_int64),
                ("overflow", c_uint32), ("overflow_any", c_uint32)]


class GsStepArgs(ctypes.Structure):
    _fields_ = [("params", GsParams), ("grads", GsParams), ("adam_m", GsParams), ("adam_v", GsParams),
                ("dev_cams", c_void_p), ("dev_target", c_void_p), ("dev_images", c_void_p),
                ("dev_T_final", c_void_p), ("dev_n_contrib", c_void_p), ("dev_loss", c_void_p),
                ("dev_step", c_void_p), ("dev_workspace", c_void_p), ("hp", GsAdamHparams),
                ("plain", c_int32), ("do_delta", c_int32), ("baseline", GsParams),
                ("group_mask", c_uint32), ("rel_tau", c_float), ("dev_delta_out", c_void_p),
                ("delta_cap_words", c_int64), ("dev_hp", c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2604_02851_amd.build.build() "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        st = c_int32
        ctx = c_void_p
        L.gs_create.argtypes = [c_int32, POINTER(c_void_p)]
        L.gs_destroy.argtypes = [ctx]
        L.gs_last_error.argtypes = [ctx]
        L.gs_last_error.restype = ctypes.c_char_p
        L.gs_plan.argtypes = [ctx, c_int32, c_int32, c_int32, c_void_p, POINTER(GsRenderOpts), c_int64,
                              POINTER(c_size_t)]
        L.gs_frame_layout.argtypes = [ctx, c_void_p, c_void_p]
        L.gs_workspace_init.argtypes = [ctx, c_void_p, c_void_p]
        L.gs_project.argtypes = [ctx, POINTER(GsParams), c_void_p, c_int32, c_int32, c_void_p, c_void_p]
        L.gs_build_tile_lists.argtypes = [ctx, c_int32, c_int32, c_void_p, c_void_p]
        L.gs_composite.argtypes = [ctx, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.gs_backward.argtypes = [ctx, POINTER(GsParams), c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_int32, POINTER(GsParams), c_int32, c_void_p, c_void_p]
        L.gs_adam_step.argtypes = [ctx, POINTER(GsParams), POINTER(GsParams), POINTER(GsParams), POINTER(GsParams),
                                   c_void_p, POINTER(GsAdamHparams), c_void_p]
        L.gs_delta_extract.argtypes = [ctx, POINTER(GsParams), POINTER(GsParams), c_uint32, c_float, c_void_p,
                                       c_int64, c_void_p, c_void_p]
        L.gs_codec_capacity_words.argtypes = [c_int32, c_int32, POINTER(GsCodec), c_uint32]
        L.gs_delta_encode.argtypes = [ctx, POINTER(GsParams), POINTER(GsParams), POINTER(GsCodec), c_uint32, c_void_p,
                                      c_void_p, c_int64, c_void_p, c_void_p]
        L.gs_delta_encode_noalloc.argtypes = [ctx, POINTER(GsParams), POINTER(GsParams), POINTER(GsCodec), c_uint32,
                                              c_void_p, c_void_p, c_int64, c_void_p]
        L.gs_delta_apply.argtypes = [ctx, POINTER(GsParams), POINTER(GsCodec), c_void_p, c_int64, c_void_p, c_void_p,
                                     c_void_p]
        L.gs_object_transform.argtypes = [ctx, POINTER(GsParams), c_void_p, c_void_p, c_int32, c_void_p]
        L.gs_relight_dc.argtypes = [ctx, POINTER(GsParams), c_void_p, c_int32, c_void_p]
        L.gs_append.argtypes = [ctx, POINTER(GsParams), POINTER(GsParams), POINTER(GsParams), c_int32,
                                POINTER(GsParams), POINTER(GsParams), POINTER(GsParams), POINTER(GsParams),
                                c_void_p, c_void_p, c_void_p, c_int32, c_void_p]
        L.gs_delta_reset_baseline.argtypes = [ctx, POINTER(GsParams), POINTER(GsParams), c_void_p, c_void_p]
        L.gs_assign_cells.argtypes = [ctx, POINTER(GsParams), POINTER(GsGrid), c_void_p, c_void_p, c_void_p]
        L.gs_visible_cells.argtypes = [ctx, POINTER(GsGrid), c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p]
        L.gs_set_precull.argtypes = [ctx, c_void_p, c_void_p, c_int32]
        L.gs_freeze.argtypes = [ctx, POINTER(GsParams), POINTER(GsParams), POINTER(GsParams), c_void_p, c_void_p,
                                c_void_p, c_void_p, c_void_p, c_void_p]
        L.gs_sort_cells.argtypes = [ctx, POINTER(GsParams), POINTER(GsParams), POINTER(GsParams), c_void_p, c_int32,
                                    c_void_p, c_void_p, c_void_p, c_void_p]
        L.gs_read_counters.argtypes = [ctx, c_void_p, c_void_p, POINTER(GsCounters)]
        L.gs_workspace_segment.argtypes = [ctx, c_int32, c_int32, c_int32, POINTER(c_size_t), POINTER(c_size_t)]
        L.gs_profile_enable.argtypes = [ctx, c_int32]
        L.gs_profile_read.argtypes = [ctx, ctypes.c_char_p, POINTER(ctypes.c_double), POINTER(c_int64)]
        L.gs_profile_reset.argtypes = [ctx]
        L.gs_step.argtypes = [ctx, POINTER(GsStepArgs), c_void_p]
        L.gs_step_capture.argtypes = [ctx, POINTER(GsStepArgs), c_void_p]
        L.gs_step_launch.argtypes = [ctx, POINTER(GsStepArgs), c_void_p]
        for name in EXPORTED:
            if name not in ("gs_last_error", "gs_codec_capacity_words"):
                getattr(L, name).restype = st
        L.gs_codec_capacity_words.restype = c_int64
        _lib = L
    return _lib


def ptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return t.data_ptr()


def codec_capacity_words(n: int, sh_degree: int, codecs, group_mask: int = 0x3F) -> int:
    w = lib().gs_codec_capacity_words(int(n), int(sh_degree), codec_array(codecs), int(group_mask))
    if w < 0:
        raise ValueError(f"invalid codecs {codecs} or arguments")
    return int(w)


def stream_handle(stream: torch.cuda.Stream | None = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


PARAM_NAMES = ("mean", "log_scale", "quat", "opacity_logit", "sh")


class DeviceParams:
    """Planar FP32 Gaussian tensors on the GPU (layout of gs_params)."""

    def __init__(self, mean, log_scale, quat, opacity_logit, sh, sh_degree: int):
        self.mean, self.log_scale, self.quat, self.opacity_logit, self.sh = mean, log_scale, quat, opacity_logit, sh
        self.sh_degree = sh_degree

    @property
    def n(self) -> int:
        return int(self.opacity_logit.shape[0])

    def tensors(self):
        return [getattr(self, k) for k in PARAM_NAMES]

    @classmethod
    def from_scene(cls, scene, device="cuda"):
        t = [torch.from_numpy(np.ascontiguousarray(a)).to(device) for _, a in scene.tensors()]
        return cls(*t, scene.sh_degree)

    @classmethod
    def zeros_like(cls, other: "DeviceParams"):
        return cls(*[torch.zeros_like(t) for t in other.tensors()], other.sh_degree)

    def clone(self):
        return DeviceParams(*[t.clone() for t in self.tensors()], self.sh_degree)

    @classmethod
    def zeros(cls, n: int, sh_degree: int, device="cuda"):
        nk = (sh_degree + 1) ** 2
        f = dict(dtype=torch.float32, device=device)
        return cls(torch.zeros(3, n, **f), torch.zeros(3, n, **f), torch.zeros(4, n, **f), torch.zeros(n, **f),
                   torch.zeros(3 * nk, n, **f), sh_degree)

    def narrowed(self, n: int) -> "DeviceParams":
        """The same storage described with n Gaussians per row (rows packed at
        stride n), as left by an in-place compaction to n."""
        assert 0 <= n <= self.n
        out = []
        for t in self.tensors():
            rows = 1 if t.dim() == 1 else t.shape[0]
            flat = t.view(-1) if t.is_contiguous() else t.reshape(-1)
            v = flat[:rows * n]
            out.append(v if t.dim() == 1 else v.view(rows, n))
        return DeviceParams(*out, self.sh_degree)

    def struct(self) -> GsParams:
        return GsParams(*[ptr(t) for t in self.tensors()], self.n, self.sh_degree)

    def to_scene(self):
        from .scenes import Scene
        return Scene(*[t.detach().cpu().numpy() for t in self.tensors()], self.sh_degree)


class Context:
    """One gs_ctx (one per stream)."""

    def __init__(self, device: int = 0):
        self.L = lib()
        h = c_void_p()
        s = self.L.gs_create(device, ctypes.byref(h))
        if s != GS_OK:
            raise GsError(s, f"gs_create({device}) failed")
        self.h = h
        self.n_views = 0

    def close(self):
        if self.h:
            self.L.gs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, s: int):
        if s != GS_OK:
            raise GsError(s, self.L.gs_last_error(self.h).decode())

    def plan(self, n, sh_degree, cams: np.ndarray, tile=(16, 16), batch_depth=64, bg=(0.0, 0.0, 0.0),
             loss_mode=0, key_capacity=1 << 20, pixels_per_thread=1, wave_w=0, schedule=0) -> int:
        cams = np.ascontiguousarray(cams)
        opts = GsRenderOpts(tile[0], tile[1], batch_depth, pixels_per_thread, wave_w, schedule, (c_float * 3)(*bg),
                            loss_mode)
        out = c_size_t()
        self._chk(self.L.gs_plan(self.h, n, sh_degree, len(cams), cams.ctypes.data_as(c_void_p), ctypes.byref(opts),
                                 int(key_capacity), ctypes.byref(out)))
        self.n_views = len(cams)
        return int(out.value)

    def frame_layout(self):
        pix = np.zeros(self.n_views + 1, np.int64)
        til = np.zeros(self.n_views + 1, np.int32)
        self._chk(self.L.gs_frame_layout(self.h, pix.ctypes.data_as(c_void_p), til.ctypes.data_as(c_void_p)))
        return pix, til

    def workspace_init(self, ws, stream=None):
        self._chk(self.L.gs_workspace_init(self.h, ptr(ws), stream_handle(stream)))

    def project(self, params: DeviceParams, dev_cams, v0, nv, ws, stream=None):
        p = params.struct()
        self._chk(self.L.gs_project(self.h, ctypes.byref(p), ptr(dev_cams), v0, nv, ptr(ws), stream_handle(stream)))

    def build_tile_lists(self, v0, nv, ws, stream=None):
        self._chk(self.L.gs_build_tile_lists(self.h, v0, nv, ptr(ws), stream_handle(stream)))

    def composite(self, v0, nv, ws, images, T, n_contrib, stream=None):
        self._chk(self.L.gs_composite(self.h, v0, nv, ptr(ws), ptr(images), ptr(T), ptr(n_contrib),
                                      stream_handle(stream)))

    def backward(self, params: DeviceParams, dev_cams, v0, nv, ws, images, T, upstream, mode,
                 grads: DeviceParams, accumulate=0, loss=None, stream=None):
        p, g = params.struct(), grads.struct()
        self._chk(self.L.gs_backward(self.h, ctypes.byref(p), ptr(dev_cams), v0, nv, ptr(ws), ptr(images), ptr(T),
                                     ptr(upstream), mode, ctypes.byref(g), accumulate, ptr(loss),
                                     stream_handle(stream)))

    def adam_step(self, params, grads, m, v, dev_step, lr, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
        hp = GsAdamHparams((c_float * 6)(*lr), beta1, beta2, eps)
        ps = [x.struct() for x in (params, grads, m, v)]
        self._chk(self.L.gs_adam_step(self.h, *[ctypes.byref(x) for x in ps], ptr(dev_step), ctypes.byref(hp),
                                      stream_handle(stream)))

    def delta_extract(self, cur, baseline, group_mask, rel_tau, out, ws, stream=None):
        c, b = cur.struct(), baseline.struct()
        self._chk(self.L.gs_delta_extract(self.h, ctypes.byref(c), ctypes.byref(b), group_mask, rel_tau, ptr(out),
                                          out.numel(), ptr(ws), stream_handle(stream)))

    def delta_encode(self, cur, baseline, codecs, group_mask, dev_epoch, out, ws, stream=None):
        c, b = cur.struct(), baseline.struct()
        self._chk(self.L.gs_delta_encode(self.h, ctypes.byref(c), ctypes.byref(b), codec_array(codecs), group_mask,
                                         ptr(dev_epoch), ptr(out), out.numel(), ptr(ws), stream_handle(stream)))

    def delta_encode_noalloc(self, cur, baseline, codecs, group_mask, dev_epoch, out, stream=None):
        c, b = cur.struct(), baseline.struct()
        self._chk(self.L.gs_delta_encode_noalloc(self.h, ctypes.byref(c), ctypes.byref(b), codec_array(codecs),
                                                 group_mask, ptr(dev_epoch), ptr(out), out.numel(),
                                                 stream_handle(stream)))

    def delta_apply(self, model, codecs, packet, packet_words, dev_epoch, dev_status, stream=None):
        m = model.struct()
        self._chk(self.L.gs_delta_apply(self.h, ctypes.byref(m), codec_array(codecs), ptr(packet), int(packet_words),
                                        ptr(dev_epoch), ptr(dev_status), stream_handle(stream)))

    def object_transform(self, params, object_of, dev_transforms, n_objects: int, stream=None):
        p = params.struct()
        self._chk(self.L.gs_object_transform(self.h, ctypes.byref(p), ptr(object_of), ptr(dev_transforms),
                                             int(n_objects), stream_handle(stream)))

    def relight_dc(self, params, gain, channels: int, stream=None):
        p = params.struct()
        self._chk(self.L.gs_relight_dc(self.h, ctypes.byref(p), ptr(gain), int(channels), stream_handle(stream)))

    def append(self, old, add, new, n_active: int, moments=None, cols=(), stream=None):
        """moments: (old_m, old_v, new_m, new_v) or None; cols: [(old, add,
        new)] per-Gaussian 32-bit columns."""
        o, a, nw = old.struct(), add.struct(), new.struct()
        ms = [x.struct() for x in moments] if moments is not None else [None] * 4
        ref = lambda x: ctypes.byref(x) if x is not None else None
        nc = len(cols)
        arr = lambda k: (c_void_p * max(nc, 1))(*[ptr(c[k]) for c in cols])
        self._chk(self.L.gs_append(self.h, ctypes.byref(o), ref(ms[0]), ref(ms[1]), int(n_active), ctypes.byref(a),
                                   ctypes.byref(nw), ref(ms[2]), ref(ms[3]), arr(0), arr(1), arr(2), nc,
                                   stream_handle(stream)))

    def delta_reset_baseline(self, cur, baseline, dev_epoch, stream=None):
        c, b = cur.struct(), baseline.struct()
        self._chk(self.L.gs_delta_reset_baseline(self.h, ctypes.byref(c), ctypes.byref(b), ptr(dev_epoch),
                                                 stream_handle(stream)))

    def assign_cells(self, params, grid: "GsGrid", cell_of, cell_sigma, stream=None):
        p = params.struct()
        self._chk(self.L.gs_assign_cells(self.h, ctypes.byref(p), ctypes.byref(grid), ptr(cell_of), ptr(cell_sigma),
                                         stream_handle(stream)))

    def visible_cells(self, grid: "GsGrid", dev_cams, v0, nv, cell_sigma, mask, stream=None):
        self._chk(self.L.gs_visible_cells(self.h, ctypes.byref(grid), ptr(dev_cams), v0, nv, ptr(cell_sigma),
                                          ptr(mask), stream_handle(stream)))

    def set_precull(self, cell_of, mask, n_cells: int):
        self._chk(self.L.gs_set_precull(self.h, ptr(cell_of), ptr(mask), int(n_cells)))

    def sort_cells(self, params, cell_of, n_cells: int, ws, m=None, v=None, ids=None, baseline=None, stream=None):
        p = params.struct()
        mm = m.struct() if m is not None else None
        vv = v.struct() if v is not None else None
        b = baseline.struct() if baseline is not None else None
        ref = lambda x: ctypes.byref(x) if x is not None else None
        self._chk(self.L.gs_sort_cells(self.h, ctypes.byref(p), ref(mm), ref(vv), ptr(cell_of), int(n_cells),
                                       ptr(ids), ref(b), ptr(ws), stream_handle(stream)))

    def freeze(self, params, m, v, flags, ws, new_active, ids=None, baseline=None, stream=None):
        p, mm, vv = params.struct(), m.struct(), v.struct()
        b = baseline.struct() if baseline is not None else None
        self._chk(self.L.gs_freeze(self.h, ctypes.byref(p), ctypes.byref(mm), ctypes.byref(vv), ptr(flags), ptr(ids),
                                   ctypes.byref(b) if b is not None else None, ptr(ws), ptr(new_active),
                                   stream_handle(stream)))

    def read_counters(self, ws, stream=None) -> GsCounters:
        out = GsCounters()
        self._chk(self.L.gs_read_counters(self.h, ptr(ws), stream_handle(stream), ctypes.byref(out)))
        return out

    def segment(self, ws: torch.Tensor, name: str, v0: int = 0, nv: int | None = None) -> torch.Tensor:
        """A view (uint8) of one internal workspace array."""
        nv = self.n_views - v0 if nv is None else nv
        off, nb = c_size_t(), c_size_t()
        self._chk(self.L.gs_workspace_segment(self.h, SEG[name], v0, nv, ctypes.byref(off), ctypes.byref(nb)))
        return ws[off.value: off.value + nb.value]

    def profile(self, on: bool = True):
        self._chk(self.L.gs_profile_enable(self.h, 1 if on else 0))

    def profile_reset(self):
        self._chk(self.L.gs_profile_reset(self.h))

    def profile_read(self) -> dict:
        out = {}
        for s in STAGES:
            ms, calls = ctypes.c_double(), c_int64()
            self._chk(self.L.gs_profile_read(self.h, s.encode(), ctypes.byref(ms), ctypes.byref(calls)))
            out[s] = (float(ms.value), int(calls.value))
        return out

    def step(self, args: GsStepArgs, stream=None):
        self._chk(self.L.gs_step(self.h, ctypes.byref(args), stream_handle(stream)))

    def step_capture(self, args: GsStepArgs, stream=None):
        self._chk(self.L.gs_step_capture(self.h, ctypes.byref(args), stream_handle(stream)))

    def step_launch(self, args: GsStepArgs, stream=None):
        self._chk(self.L.gs_step_launch(self.h, ctypes.byref(args), stream_handle(stream)))


def delta_capacity_words(n: int, sh_degree: int, mask: int = 0x3F) -> int:
    widths = [1, 3, 3 * ((sh_degree + 1) ** 2 - 1), 3, 3, 4]
    return 6 + sum(n * (1 + w) for g, w in enumerate(widths) if (mask >> g) & 1)
