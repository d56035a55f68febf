"""Streaming the live model (Sec. 3.5): sender-side delta codecs with
per-attribute schedules and transmission epochs, and the client's replay of
snapshots and deltas into its own copy of the model.

The arithmetic runs in the library (`gs_delta_encode`, `gs_delta_apply`,
`gs_delta_reset_baseline`); this module only keeps the state: the
baselines, the epoch, the packet buffer and which groups are due in a frame.

Codec defaults (the paper gives no bit widths, ranges or steps): means and
log-scales are residual-coded with 16-bit codes (steps 2^-12 world units and
2^-10), the other groups are quantized updates with 16-bit codes (opacity
logits over [-8, 8), DC over [-4, 4), quaternion components over [-2, 2))
except the higher SH bands, 8-bit over [-1, 1).  Schedule defaults: opacity
and DC every frame, the other groups every fourth frame (the paper sends the
former every frame and the latter less often).
"""
from __future__ import annotations

import torch

from . import native as N
from .native import DeviceParams

GROUPS = ("opacity", "dc", "sh_rest", "mean", "log_scale", "quat")
DEFAULT_CODECS = (
    (N.CODEC_QUANT, 16, 2.0 ** -12, -8.0, 0.0),      # opacity logit
    (N.CODEC_QUANT, 16, 2.0 ** -13, -4.0, 0.0),      # SH DC
    (N.CODEC_QUANT, 8, 2.0 ** -7, -1.0, 0.0),        # SH higher bands
    (N.CODEC_RESIDUAL, 16, 2.0 ** -12, 0.0, 0.0),    # mean
    (N.CODEC_RESIDUAL, 16, 2.0 ** -10, 0.0, 0.0),    # log-scale
    (N.CODEC_QUANT, 16, 2.0 ** -14, -2.0, 0.0),      # quaternion
)
DEFAULT_PERIODS = (1, 1, 4, 4, 4, 4)


def schedule_mask(frame: int, periods=DEFAULT_PERIODS) -> int:
    """Groups due in `frame` (group g when frame % periods[g] == 0; a period
    of 0 never sends the group)."""
    return sum(1 << g for g, p in enumerate(periods) if p > 0 and frame % p == 0)


class Sender:
    """Sender side: baselines (what the receiver holds), the epoch and the
    packet buffer; `frame()` encodes the groups due in a frame."""

    def __init__(self, ctx, params: DeviceParams, ws, codecs=DEFAULT_CODECS, periods=DEFAULT_PERIODS, stream=None):
        self.ctx, self.params, self.ws, self.stream = ctx, params, ws, stream
        self.codecs, self.periods = tuple(codecs), tuple(periods)
        self.baseline = params.clone()
        self.epoch = torch.zeros(1, dtype=torch.int32, device=params.mean.device)
        words = N.codec_capacity_words(params.n, params.sh_degree, self.codecs, 0x3F)
        self.out = torch.zeros(words, dtype=torch.int32, device=params.mean.device)
        self.frames = 0

    def snapshot(self):
        """Baselines := the current model, epoch + 1 (after a full snapshot
        has been sent)."""
        self.ctx.delta_reset_baseline(self.params, self.baseline, self.epoch, self.stream)

    def frame(self, mask: int | None = None) -> torch.Tensor:
        """Encodes this frame's packet into `out` (device); returns `out`.
        The packet's length is out[8] (read it after synchronising)."""
        m = schedule_mask(self.frames, self.periods) if mask is None else mask
        self.frames += 1
        self.ctx.delta_encode(self.params, self.baseline, self.codecs, m, self.epoch, self.out, self.ws, self.stream)
        return self.out


class Receiver:
    """Client side: a local copy of the model, its epoch and the status of the
    last packet."""

    def __init__(self, ctx, n: int, sh_degree: int, codecs=DEFAULT_CODECS, device="cuda", stream=None):
        self.ctx, self.codecs, self.stream = ctx, tuple(codecs), stream
        self.model = DeviceParams.zeros(n, sh_degree, device)
        self.epoch = torch.zeros(1, dtype=torch.int32, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)

    def load_snapshot(self, params: DeviceParams, epoch: torch.Tensor):
        """Replaces the local model by a decoded snapshot of the sender's model
        and adopts its epoch."""
        for dst, src in zip(self.model.tensors(), params.tensors()):
            dst.copy_(src)
        self.epoch.copy_(epoch)

    def apply(self, packet: torch.Tensor, words: int | None = None):
        """Applies a received packet (device int32 words); the status lands in
        `status` (0 applied, bit 1 stale epoch, bit 2 malformed)."""
        n = packet.numel() if words is None else int(words)
        self.ctx.delta_apply(self.model, self.codecs, packet, n, self.epoch, self.status, self.stream)
