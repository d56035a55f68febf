#!/usr/bin/env python3
"""Optimize-step throughput of the 3DGS hot path on one MI355X.

Workload (default): 1M Gaussians, SH degree 3, 16 reference views of mixed
resolution (640x360 / 1280x720 / 1920x1080) on a sphere of radius 6-12, L1
loss against targets rendered from a perturbed copy of the model.  A step is
project/cull -> tile lists -> composite -> backward -> fused Adam over all 16
views.  `value` is the batched step (one launch per stage for all views, the
whole step replayed from a HIP graph) in steps/s; the plain path (the same
kernels one view per launch, eager) is reported beside it.

Also printed: per-stage times from the library's HIP-event timers, the
roofline position of the dominant kernel, and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "optimize steps/sec (fwd+bwd+Adam, 1M Gaussians, 16 mixed views) batched vs plain"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0
# Algorithmic FP32 operations per examined (pixel, splat) pair and per
# composited pair (counted from the compositing rule and its adjoint).
FLOPS_TEST = 12
FLOPS_FWD_COMPOSITED = 12
FLOPS_BWD_COMPOSITED = 55
# The plain path: the same kernels, one view per launch, eager, 16x16 tiles,
# batch depth 64, one pixel per thread, one workgroup per tile.
PLAIN_SHAPE = dict(tile=(16, 16), batch_depth=64, pixels_per_thread=1, wave_w=16, schedule=0)


def stage_floors(u: dict) -> dict:
    """Algorithmic bytes and FP32 operations of each stage of one optimize
    step, from the counts measured in the run (u: gaussians, pairs = views x
    Gaussians, visible pairs, keys, examined and composited pairs, pixels,
    trainable scalars, SH coefficient floats per Gaussian), and the stage's
    time floor max(bytes / 8 TB/s, ops / 157.3 TFLOP/s) in ms.
      project      params read once (4 B x floats per Gaussian); per visible
                   pair a 48 B splat record and 16 B of depth key, tile
                   rectangle and tile count; 4 B tile count per (view,
                   Gaussian) pair; 8 B view mask per Gaussian
      tile_lists   12 B read per visible pair; 12 B per key emitted and one
                   permutation of the keys (24 B per key)
      composite    40 B per key (index and splat record); 24 B written per
                   pixel; 12 ops per examined and 12 per composited pair
      composite_bwd 40 B per key; 32 B read per pixel; 12 ops per examined
                   and 55 per composited pair (gradient atomics not counted)
      project_bwd  36 B read per visible pair; params read and gradients
                   written once per Gaussian
      adam         28 B per trainable scalar"""
    fl = u["floats_per_gaussian"]
    st = {
        "project": (4 * fl * u["gaussians"] + 64 * u["visible"] + 4 * u["pairs"] + 8 * u["gaussians"], 0),
        "tile_lists": (12 * u["visible"] + 36 * u["keys"], 0),
        "composite": (40 * u["keys"] + 24 * u["pixels"], FLOPS_TEST * u["examined"] + FLOPS_FWD_COMPOSITED * u["composited"]),
        "composite_bwd": (40 * u["keys"] + 32 * u["pixels"],
                          FLOPS_TEST * u["examined"] + FLOPS_BWD_COMPOSITED * u["composited"]),
        "project_bwd": (36 * u["visible"] + 8 * fl * u["gaussians"], 0),
        "adam": (28 * u["trainable"], 0),
    }
    out = {}
    for k, (b, ops) in st.items():
        t_b = b / (PEAK_HBM_GBS * 1e9) * 1e3
        t_o = ops / (PEAK_FP32_TFLOPS * 1e12) * 1e3
        out[k] = {"bytes": int(b), "ops": int(ops), "floor_ms": round(max(t_b, t_o), 5),
                  "bound": "hbm" if t_b >= t_o else "alu"}
    return out


def roofline_fractions(floors: dict, stage_ms: dict, step_ms: float) -> dict:
    """Per stage: floor / measured stage time; per step: sum of the floors /
    measured step time."""
    per = {k: round(f["floor_ms"] / stage_ms[k], 4) for k, f in floors.items() if stage_ms.get(k)}
    total = sum(f["floor_ms"] for f in floors.values())
    return {"per_stage": per, "step": round(total / step_ms, 4), "step_floor_ms": round(total, 4)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse_tile(s):
    w, h = s.lower().split("x")
    return int(w), int(h)


def pair_counts(r, torch):
    """(examined pairs up to each pixel's last composited splat, composited
    pairs) of the last forward pass."""
    import numpy as np
    ranges = r.ctx.segment(r.ws, "ranges").view(torch.int32).view(-1, 2).long()
    last = r.ctx.segment(r.ws, "last").view(torch.int32).long()
    E = 0
    for v in range(r.n_views):
        W, H = int(r.cams[v]["width"]), int(r.cams[v]["height"])
        tw, th = r.tile
        tx = (W + tw - 1) // tw
        ys = torch.arange(H, device=r.device).view(-1, 1) // th
        xs = torch.arange(W, device=r.device).view(1, -1) // tw
        tiles = (int(r.tile_off[v]) + ys * tx + xs).view(-1)
        p0, p1 = int(r.pix_off[v]), int(r.pix_off[v + 1])
        E += int((last[p0:p1] - ranges[tiles, 0]).sum().item())
    C = int(r.n_contrib.long().sum().item())
    return E, C


def cpu_info() -> dict:
    """Host CPU of this run: model name, logical CPUs and the ones this
    process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "logical_cpus": os.cpu_count()}


def single_core_oracle(cfgs=(1, 2), timeout: float = 120.0) -> dict:
    """The oracle's optimize step (forward, L1 backward with projection
    adjoint, Adam) on whole small workloads with one OpenMP thread, in a
    child process (the thread count is fixed when the oracle library
    loads)."""
    import subprocess
    code = ("import sys, time, numpy as np; sys.path.insert(0, %r)\n"
            "from oracle import oracle as O\nfrom paper_2604_02851_amd import scenes as S\nO.lib()\n"
            "for cfg in %r:\n"
            "    w = S.workload(cfg); t = time.perf_counter()\n"
            "    O.backward(w.scene, w.cams, np.full(3 * w.n_pixels, 0.5, np.float32), mode=1, loss_mode=1)\n"
            "    for name, a in w.scene.tensors():\n"
            "        z = np.zeros_like(a); O.adam(a, z, z, z, 1e-3, 0.9, 0.999, 1e-15, 1)\n"
            "    print(cfg, time.perf_counter() - t, flush=True)\n") % (ROOT, tuple(cfgs))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=timeout)
    except subprocess.TimeoutExpired:
        return {}
    out = {}
    for line in r.stdout.split("\n"):
        if line.strip():
            cfg, sec = line.split()
            out[f"cfg{cfg}"] = {"steps_per_s": round(1.0 / float(sec), 4), "seconds": round(float(sec), 3)}
    return out


def cpu_baseline(w, min_seconds: float):
    """Times the FP64 oracle's optimize step on whole views of the workload,
    in view order, until at least `min_seconds` have passed (forward,
    L1 backward with its projection adjoint, then Adam over all parameters),
    and scales the view part to the step by pixel count.  The oracle as it
    stands: its backward also computes the tolerance bookkeeping the parity
    tests use (magnitude and transmittance scales, decision slack)."""
    import numpy as np
    from oracle import oracle as O
    O.lib()
    t0 = time.perf_counter()
    done_px, views = 0, 0
    for v in range(len(w.cams)):
        c = w.cams[v:v + 1].copy()
        npx = int(c[0]["width"]) * int(c[0]["height"])
        O.backward(w.scene, c, np.full(3 * npx, 0.5, np.float32), mode=1, loss_mode=1)
        done_px += npx
        views += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    t_views = time.perf_counter() - t0
    t = time.perf_counter()
    g = np.zeros_like(w.scene.sh)
    O.adam(w.scene.sh, g, g, g, 5e-3, 0.9, 0.999, 1e-15, 1)
    for name in ("mean", "log_scale", "quat", "opacity_logit"):
        a = getattr(w.scene, name)
        O.adam(a, np.zeros_like(a), np.zeros_like(a), np.zeros_like(a), 1e-3, 0.9, 0.999, 1e-15, 1)
    t_adam = time.perf_counter() - t
    total_px = sum(int(c["width"]) * int(c["height"]) for c in w.cams)
    t_step = t_views * total_px / done_px + t_adam
    info = cpu_info()
    # the oracle's OpenMP loops run on OMP_NUM_THREADS threads when it is set,
    # else on every usable CPU
    cores = int(os.environ.get("OMP_NUM_THREADS") or info["nproc"] or 1)
    return {"value": 1.0 / t_step, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 oracle step on views 0-{views - 1} of {len(w.cams)} ({done_px} of {total_px} px: "
                       f"forward, L1 backward, projection adjoint of all {w.scene.n} Gaussians per view, "
                       f"including the oracle's tolerance bookkeeping) in {t_views:.1f} s, Adam over all "
                       f"parameters in {t_adam:.1f} s; view part scaled by pixel count to {t_step:.1f} s per step"),
            **info}


def config_rate(cfg: int, shape: dict, steps: int, warmup: int, torch, log, frozen: float = 0.0) -> dict:
    """Steps/s of one synthetic workload (graph replay of the batched step, the
    given launch shape; cfg5 also extracts the delta of all six attribute
    groups after each step, on the scene after one round of object motion and
    relighting).  frozen: fraction of the Gaussians in the frozen pool
    (rendered, not optimised; the last ones)."""
    from paper_2604_02851_amd import scenes as S
    from paper_2604_02851_amd.native import DeviceParams
    from paper_2604_02851_amd.renderer import Optimizer, Renderer
    import numpy as np
    w = S.workload(cfg)
    stream = torch.cuda.current_stream()
    pert = w.extra.get("perturbed")
    if cfg == 5:
        S.Dynamics(w.extra["rng_dyn"], w.scene).step([w.scene, pert])
    params = DeviceParams.from_scene(w.scene)
    r = Renderer(w.cams, w.scene.n, w.scene.sh_degree, loss_mode=1, **shape)
    r.fit_capacity(params)
    if pert is not None:            # targets: render of the perturbed copy
        pdev = DeviceParams.from_scene(pert)
        r.fit_capacity(pdev)
        targets = r.forward(pdev)[0].clone()
        del pdev
    else:                           # the workload's own target image
        targets = torch.from_numpy(np.ascontiguousarray(w.extra["target"], np.float32).reshape(-1)).to(r.device)
    n_active = w.scene.n - int(round(frozen * w.scene.n))
    opt = Optimizer(r, params, targets, stream=stream, n_active=n_active)
    if cfg == 5:
        opt.enable_delta(params.clone(), 0x3F, 1e-3)
    opt.step()
    torch.cuda.synchronize()
    opt.capture()
    for _ in range(warmup):
        opt.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        opt.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    if r.counters().overflow_any:
        raise SystemExit(f"cfg{cfg}: key capacity overflowed during the timed steps")
    out = {"steps_per_s": round(1000.0 / ms, 3), "ms_per_step": round(ms, 4), "views": len(w.cams),
           "views_per_s": round(len(w.cams) * 1000.0 / ms, 2), "gaussians": w.scene.n, "pixels": w.n_pixels,
           "keys": int(r.counters().keys), "delta": cfg == 5, "active_gaussians": n_active}
    log(f"[bench] {w.name} ({n_active} active): {ms:.3f} ms/step ({1000 / ms:.2f} steps/s)")
    del opt, r, params, targets
    torch.cuda.empty_cache()
    return out


def oracle_step_seconds(w, runs: int) -> float:
    """Median wall time of the FP64 oracle's whole optimize step on the
    workload (forward, L1 backward against a constant target with the
    projection adjoint, Adam over every parameter, and for the dynamics
    workload the delta of all six groups), OpenMP on the host's cores."""
    import numpy as np
    from oracle import oracle as O
    O.lib()
    times = []
    for _ in range(runs):
        t = time.perf_counter()
        O.backward(w.scene, w.cams, np.full(3 * w.n_pixels, 0.5, np.float32), mode=1, loss_mode=1)
        for name, a in w.scene.tensors():
            z = np.zeros_like(a)
            O.adam(a, z, z, z, 1e-3, 0.9, 0.999, 1e-15, 1)
        if w.name == "cfg5":
            O.delta(w.scene, w.scene, 0x3F, 1e-3)
        times.append(time.perf_counter() - t)
    return float(np.median(times))


def table_row(cfg: int, shape: dict | None, torch, log, steps: int = 10, warmup: int = 2, plain_steps: int = 2,
              oracle_runs: int = 1) -> dict:
    """One row of the per-workload table: batched steps/s (graph replay,
    `shape`, or the autotuner's shape for this workload when None), plain
    steps/s (one view per launch, eager, 16x16 tiles, batch depth 64),
    views/s, the step's roofline fraction (sum of the stage floors over the
    batched step time) and the oracle's steps/s."""
    from paper_2604_02851_amd import scenes as S
    from paper_2604_02851_amd.native import DeviceParams
    from paper_2604_02851_amd.renderer import SHAPE_KEYS, Optimizer, Renderer, autotune
    import numpy as np
    w = S.workload(cfg)
    stream = torch.cuda.current_stream()
    pert = w.extra.get("perturbed")
    if cfg == 5:
        S.Dynamics(w.extra["rng_dyn"], w.scene).step([w.scene, pert])
    params = DeviceParams.from_scene(w.scene)
    if shape is None:
        tgt_params = DeviceParams.from_scene(pert) if pert is not None else params
        tuned = autotune(w.cams, params, tgt_params, stream=stream, log=log)
        shape = {k: tuned[k] for k in SHAPE_KEYS}
        del tgt_params

    def setup(sh, p):
        r = Renderer(w.cams, w.scene.n, w.scene.sh_degree, loss_mode=1, **sh)
        r.fit_capacity(p)
        if pert is not None:
            pdev = DeviceParams.from_scene(pert)
            r.fit_capacity(pdev)
            tg = r.forward(pdev)[0].clone()
        else:
            tg = torch.from_numpy(np.ascontiguousarray(w.extra["target"], np.float32).reshape(-1)).to(r.device)
        o = Optimizer(r, p, tg, stream=stream)
        if cfg == 5:
            o.enable_delta(p.clone(), 0x3F, 1e-3)
        return r, o

    r, opt = setup(shape, params.clone())
    opt.step()
    torch.cuda.synchronize()
    opt.capture()
    for _ in range(warmup):
        opt.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        opt.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1) / steps
    r.ctx.profile(True)
    r.ctx.profile_reset()
    for _ in range(3):
        opt.step()
    stages = r.ctx.profile_read()
    r.ctx.profile(False)
    stage_ms = {k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1] > 0}
    E, C = pair_counts(r, torch)
    c = r.counters()
    if c.overflow_any:
        raise SystemExit(f"cfg{cfg}: key capacity overflowed")
    floats = 14 + 3 * ((w.scene.sh_degree + 1) ** 2 - 1)
    units = {"gaussians": w.scene.n, "pairs": w.scene.n * len(w.cams), "visible": int(c.visible),
             "keys": int(c.keys), "examined": E, "composited": C, "pixels": w.n_pixels,
             "trainable": floats * w.scene.n, "floats_per_gaussian": floats}
    fr = roofline_fractions(stage_floors(units), stage_ms, ms_b)
    del opt, r
    torch.cuda.empty_cache()
    rp, optp = setup(PLAIN_SHAPE, params.clone())
    optp.step(plain=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(plain_steps):
        optp.step(plain=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1) / plain_steps
    if rp.counters().overflow_any:
        raise SystemExit(f"cfg{cfg}: key capacity overflowed in the plain path")
    del optp, rp
    torch.cuda.empty_cache()
    t_o = oracle_step_seconds(w, oracle_runs)
    row = {"shape": {k: (list(v) if k == "tile" else v) for k, v in shape.items()},
           "batched_steps_per_s": round(1000.0 / ms_b, 2), "plain_steps_per_s": round(1000.0 / ms_p, 2),
           "batched_over_plain": round(ms_p / ms_b, 3), "views_per_s": round(len(w.cams) * 1000.0 / ms_b, 1),
           "roofline_step": fr["step"], "roofline_per_stage": fr["per_stage"], "stages_ms": stage_ms,
           "oracle_steps_per_s": round(1.0 / t_o, 5), "oracle_seconds": round(t_o, 2), "oracle_runs": oracle_runs,
           "keys": int(c.keys), "visible_pairs": int(c.visible), "examined_pairs": E, "composited_pairs": C}
    log(f"[table] cfg{cfg}: " + json.dumps(row))
    return row


def stream_rate(shape: dict, steps: int, torch, log) -> dict:
    """The streaming path on the 3M-Gaussian dynamics workload: after each
    optimize step (graph replay), the sender encodes the groups due in that
    frame with the default codecs and schedule, and a receiver on the same
    GPU replays the packet (the full buffer is handed over: the header's
    total bounds it).  Encode and replay are timed with events of their own,
    after the step has finished."""
    from paper_2604_02851_amd import scenes as S
    from paper_2604_02851_amd import stream as ST
    from paper_2604_02851_amd.native import DeviceParams
    from paper_2604_02851_amd.renderer import Optimizer, Renderer
    w = S.workload(5)
    stream = torch.cuda.current_stream()
    pert = w.extra["perturbed"]
    S.Dynamics(w.extra["rng_dyn"], w.scene).step([w.scene, pert])
    params = DeviceParams.from_scene(w.scene)
    r = Renderer(w.cams, w.scene.n, w.scene.sh_degree, loss_mode=1, **shape)
    r.fit_capacity(params)
    pdev = DeviceParams.from_scene(pert)
    r.fit_capacity(pdev)
    targets = r.forward(pdev)[0].clone()
    del pdev
    opt = Optimizer(r, params, targets, stream=stream)
    snd = ST.Sender(r.ctx, params, r.ws, stream=stream)
    rcv = ST.Receiver(r.ctx, w.scene.n, w.scene.sh_degree, stream=stream)
    rcv.load_snapshot(params, snd.epoch)
    opt.step()
    torch.cuda.synchronize()
    opt.capture()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    words = []
    for k in range(steps):
        opt.replay()
        # an event recorded right behind a graph launch can take its time
        # stamp before the graph's last kernels end: wait for the step, so
        # the events bracket the encoder and the replay alone
        stream.synchronize()
        ev[k][0].record(stream)
        pk = snd.frame()
        ev[k][1].record(stream)
        ev[k][2].record(stream)
        rcv.apply(pk)
        ev[k][3].record(stream)
        words.append(pk[8].clone())
    torch.cuda.synchronize()
    enc = [e[0].elapsed_time(e[1]) for e in ev]
    app = [e[2].elapsed_time(e[3]) for e in ev]
    words = [int(x.item()) for x in words]
    ok = int(rcv.status.item()) == 0 and all(torch.equal(a.view(torch.int32), b.view(torch.int32))
                                             for a, b in zip(rcv.model.tensors(), snd.baseline.tensors()))
    if not ok:
        raise SystemExit("streaming: the receiver's model differs from the sender's baseline")
    out = {"gaussians": w.scene.n, "encode_ms": round(sum(enc) / steps, 4), "apply_ms": round(sum(app) / steps, 4),
           "packet_words_mean": int(sum(words) / steps), "packet_words_all_groups": words[0],
           "full_model_words": 11 * w.scene.n + 48 * w.scene.n, "frames": steps}
    log(f"[bench] streaming 3M: encode {out['encode_ms']:.3f} ms, replay {out['apply_ms']:.3f} ms per frame, "
        f"{out['packet_words_mean']} words per packet on average (first, all groups: {words[0]})")
    del opt, r, params, targets, snd, rcv
    torch.cuda.empty_cache()
    return out


def dynamics_rate(shape: dict, steps: int, torch, log) -> dict:
    """Scene dynamics on the device, on the 3M-Gaussian workload: before each
    optimize step (graph replay) the 20 objects of the dynamics harness move
    rigidly (a random rotation of up to 5 degrees about the object's initial
    centroid and a N(0, 0.02) translation, drawn on the host beforehand) and
    10% of the Gaussians get their DC colour rescaled by U[0.5, 1.5] (a dense
    gain array, 1 elsewhere).  The dynamics kernels are timed with events of
    their own; afterwards, appending 100k Gaussians to the model (parameters
    and moments, new buffers) is timed the same way."""
    import math
    import numpy as np
    from paper_2604_02851_amd import native as N
    from paper_2604_02851_amd import scenes as S
    from paper_2604_02851_amd.native import DeviceParams
    from paper_2604_02851_amd.renderer import Optimizer, Renderer
    w = S.workload(5)
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(2604)
    dyn = S.Dynamics(w.extra["rng_dyn"], w.scene)
    obj = np.full(w.scene.n, -1, np.int32)
    pivots = []
    for k, idx in enumerate(dyn.members):
        obj[idx] = k
        pivots.append(w.scene.mean[:, idx].astype(np.float64).mean(1))
    tfs, gains = [], []
    for _ in range(steps):
        frame = []
        for c in pivots:
            axis = rng.normal(size=3)
            axis /= np.linalg.norm(axis)
            ang = math.radians(rng.uniform(0.0, 5.0))
            frame.append((np.r_[math.cos(ang / 2), math.sin(ang / 2) * axis], c, rng.normal(0.0, 0.02, 3)))
        tfs.append(N.transforms_tensor(frame))
        g = np.ones((1, w.scene.n), np.float32)
        g[0, rng.choice(w.scene.n, w.scene.n // 10, replace=False)] = rng.uniform(0.5, 1.5, w.scene.n // 10)
        gains.append(torch.from_numpy(g).cuda())
    obj_dev = torch.from_numpy(obj).cuda()
    params = DeviceParams.from_scene(w.scene)
    r = Renderer(w.cams, w.scene.n, w.scene.sh_degree, loss_mode=1, **shape)
    pdev = DeviceParams.from_scene(w.extra["perturbed"])
    r.fit_capacity(pdev)
    r.fit_capacity(params)
    targets = r.forward(pdev)[0].clone()
    del pdev
    opt = Optimizer(r, params, targets, stream=stream)
    opt.step()
    torch.cuda.synchronize()
    opt.capture()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(steps):
        r.ctx.object_transform(params, obj_dev, tfs[k], len(pivots), stream)
        r.ctx.relight_dc(params, gains[k], 1, stream)
        opt.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    if r.counters().overflow_any:
        raise SystemExit("dynamics: key capacity overflowed during the timed steps")
    # the two dynamics kernels alone (after the timed steps, each call on an
    # idle stream so that its events bracket only these kernels)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    for k in range(steps):
        stream.synchronize()
        ev[k][0].record(stream)
        r.ctx.object_transform(params, obj_dev, tfs[k], len(pivots), stream)
        r.ctx.relight_dc(params, gains[k], 1, stream)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    dyn_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    add = DeviceParams.from_scene(S.draw_scene(rng, 100_000, 5.0, w.scene.sh_degree))
    n, na, k = params.n, opt.n_active, add.n
    new_p = DeviceParams.zeros(n + k, w.scene.sh_degree)
    new_m, new_v = DeviceParams.zeros(na + k, w.scene.sh_degree), DeviceParams.zeros(na + k, w.scene.sh_degree)
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record(stream)
    r.ctx.append(params, add, new_p, na, moments=(opt.m, opt.v, new_m, new_v), stream=stream)
    a1.record(stream)
    torch.cuda.synchronize()
    out = {"steps_per_s": round(1000.0 / ms, 3), "ms_per_step": round(ms, 4), "dynamics_ms": round(dyn_ms, 4),
           "moved_gaussians": int((obj >= 0).sum()), "relit_gaussians": w.scene.n // 10,
           "append_100k_ms": round(a0.elapsed_time(a1), 4), "gaussians": w.scene.n}
    log(f"[bench] dynamics 3M: {ms:.3f} ms/step ({1000 / ms:.2f} steps/s) including object transforms and "
        f"relighting {dyn_ms:.3f} ms; append 100k: {out['append_100k_ms']:.3f} ms")
    del opt, r, params, targets, new_p, new_m, new_v, add
    torch.cuda.empty_cache()
    return out


def rig_rate(precull: bool, grouped: bool, shape: dict, steps: int, warmup: int, torch, log,
             freeze_unseen: bool = False) -> dict:
    """Steps/s of a large-world workload: 2M Gaussians over an 80 x 8 x 80
    region seen from a rig of 8 outward-looking 1280x720 cameras at its
    centre spread over a 60-degree arc, with or without preculling by 4-unit
    grid cells (the cell assignment and per-view visibility are recomputed
    every step, inside the timed region), with the model in its generated
    order or grouped by cell once before the timed steps.  freeze_unseen:
    before the timed steps, the Gaussians of every cell that no view of the
    rig can see move to the frozen pool (Gaussian freezing of the regions
    away from the player), so Adam and the projection adjoint cover only the
    part of the world in view."""
    from paper_2604_02851_amd import scenes as S
    from paper_2604_02851_amd.native import DeviceParams
    from paper_2604_02851_amd.renderer import Optimizer, Renderer
    w = S.rig_workload(7, 2_000_000, half=40.0, height=4.0, views=8, size=(1280, 720), arc=60.0)
    stream = torch.cuda.current_stream()
    params = DeviceParams.from_scene(w.scene)
    pdev = DeviceParams.from_scene(w.extra["perturbed"])
    r = Renderer(w.cams, w.scene.n, w.scene.sh_degree, loss_mode=1, **shape)
    if precull or grouped:
        r.enable_precull(params, origin=(-40.0, -4.0, -40.0), cell_size=4.0, dims=(20, 2, 20))
    if grouped:
        r.sort_cells(pdev)      # targets come from the perturbed model: its own order does not matter
        r.sort_cells(params)
    if grouped and not precull:
        r.disable_precull()
    r.fit_capacity(pdev)
    r.fit_capacity(params)
    targets = r.forward(pdev)[0].clone()
    del pdev
    s2 = torch.cuda.Stream()
    torch.cuda.synchronize()
    opt = Optimizer(r, params, targets, stream=s2)
    frozen = 0
    if freeze_unseen:
        if r.precull is None:   # the cell mask of the current model, without preculling the steps
            r.enable_precull(params, origin=(-40.0, -4.0, -40.0), cell_size=4.0, dims=(20, 2, 20))
            r.disable_precull()
        else:
            r.update_precull(params)
        seen = r.cell_mask.view(len(w.cams), -1).amax(0)
        flags = (seen[r.cell_of[:params.n].long()] == 0).to(torch.uint8).contiguous()
        torch.cuda.synchronize()
        frozen = params.n - opt.freeze(flags)
        if precull:
            r.update_precull(params)
    opt.step()
    torch.cuda.synchronize()
    opt.capture()

    def one():
        if precull:
            with torch.cuda.stream(s2):
                r.update_precull(params)
        opt.replay()

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s2)
    for _ in range(steps):
        one()
    e1.record(s2)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    if r.counters().overflow_any:
        raise SystemExit("rig workload: key capacity overflowed during the timed steps")
    c = r.counters()
    log(f"[bench] rig 2M/8 views/60deg, precull={precull}, grouped={grouped}, frozen {frozen}: {ms:.3f} ms/step "
        f"({1000 / ms:.2f} steps/s), visible pairs {int(c.visible)}")
    out = {"steps_per_s": round(1000.0 / ms, 3), "ms_per_step": round(ms, 4), "views": len(w.cams),
           "gaussians": w.scene.n, "precull": precull, "grouped_by_cell": grouped, "visible_pairs": int(c.visible),
           "keys": int(c.keys), "frozen_gaussians": frozen}
    del opt, r, params, targets
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--tile", default=None, help="e.g. 16x16 (default: autotuned)")
    ap.add_argument("--batch-depth", type=int, default=None)
    ap.add_argument("--ppt", type=int, default=None, help="pixels per thread (default: autotuned)")
    ap.add_argument("--wave-w", type=int, default=None, help="wave sub-tile width (default: autotuned)")
    ap.add_argument("--schedule", type=int, default=None,
                    help="tile schedule 0-3 (2, 3: persistent work queue; default: autotuned)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="minimum oracle time of the CPU baseline sample")
    ap.add_argument("--no-configs", action="store_true", help="skip the steps/s of the other workloads")
    ap.add_argument("--calib-copy", action="store_true", help="run only a plain 1 GiB device copy (PMC calibration)")
    ap.add_argument("--table", action="store_true",
                    help="instead of the benchmark line: one row per workload (batched and plain steps/s, views/s, "
                         "step roofline fraction, oracle steps/s on the host cores)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the optimize step "
              "runs on a single GPU (the multi-GPU design would shard views and reduce-scatter gradients)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": src.numel() * 4}))
        return

    from paper_2604_02851_amd import scenes as S
    from paper_2604_02851_amd.native import DeviceParams
    from paper_2604_02851_amd.renderer import SHAPE_KEYS, Optimizer, Renderer, autotune

    if args.table:
        stream = torch.cuda.Stream()      # graph capture needs a non-default stream
        torch.cuda.set_stream(stream)
        manual = {k: v for k, v in dict(tile=args.tile and parse_tile(args.tile), batch_depth=args.batch_depth,
                                        pixels_per_thread=args.ppt, wave_w=args.wave_w,
                                        schedule=args.schedule).items() if v is not None}
        shape = None   # each workload with its own autotuned launch shape
        if manual or args.no_autotune:
            shape = dict(tile=(32, 32), batch_depth=64, pixels_per_thread=4, wave_w=16, schedule=0)
            shape.update(manual)
        rows = {f"cfg{k}": table_row(k, shape, torch, log, oracle_runs=3 if k <= 3 else 1) for k in (1, 2, 3, 4, 5)}
        print(json.dumps({"table": rows, "cpu": cpu_info(), "oracle_threads": os.environ.get("OMP_NUM_THREADS")}),
              flush=True)
        return

    t0 = time.perf_counter()
    w = S.workload(args.config)
    log(f"[bench] workload {w.name}: {w.scene.n} Gaussians, {len(w.cams)} views, {w.n_pixels} pixels "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    params = DeviceParams.from_scene(w.scene)
    pert = DeviceParams.from_scene(w.extra["perturbed"])

    shape = dict(tile=(32, 32), batch_depth=128, pixels_per_thread=4, wave_w=0, schedule=0)
    tuned = None
    manual = dict(tile=args.tile and parse_tile(args.tile), batch_depth=args.batch_depth,
                  pixels_per_thread=args.ppt, wave_w=args.wave_w, schedule=args.schedule)
    if all(v is None for v in manual.values()) and not args.no_autotune:
        tuned = autotune(w.cams, params, pert, stream=stream, log=log)
        shape.update({k: tuned[k] for k in SHAPE_KEYS})
    else:
        shape.update({k: v for k, v in manual.items() if v is not None})
    tile, batch, ppt = shape["tile"], shape["batch_depth"], shape["pixels_per_thread"]
    log(f"[bench] launch shape {shape}")

    r = Renderer(w.cams, w.scene.n, w.scene.sh_degree, loss_mode=1, **shape)
    need = r.fit_capacity(pert)
    need = max(need, r.fit_capacity(params))
    log(f"[bench] keys {need}, capacity {r.key_capacity}, workspace {r.ws.numel() / 2**30:.2f} GiB")
    # targets: the perturbed model rendered by the same renderer
    targets = r.forward(pert)[0].clone()
    opt = Optimizer(r, params, targets, stream=stream)

    # ---- batched, graph-replayed ------------------------------------------
    opt.step()                       # eager warm-up (also loads kernels)
    torch.cuda.synchronize()
    opt.capture()
    for _ in range(args.warmup):
        opt.replay()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        opt.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_batched = ev0.elapsed_time(ev1) / args.steps
    c = r.counters()
    if c.overflow_any:
        raise SystemExit("key capacity overflowed during the timed steps: measurement invalid")
    log(f"[bench] batched graph: {ms_batched:.3f} ms/step ({1000 / ms_batched:.2f} steps/s), "
        f"wall {t_wall / args.steps * 1000:.3f} ms/step, loss {opt.loss.item():.5f}")

    def time_plain(o, label):
        o.step(plain=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.plain_steps):
            o.step(plain=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.plain_steps
        if o.r.counters().overflow_any:
            raise SystemExit("key capacity overflowed in the plain path")
        log(f"[bench] plain eager ({label}): {ms:.3f} ms/step ({1000 / ms:.2f} steps/s)")
        return ms

    # ---- plain with the tuned launch shape: one view per launch, eager -------
    ms_plain_tuned = time_plain(opt, "tuned shape") if args.plain_steps > 0 else None

    # ---- stage timers (eager batched steps) -------------------------------
    r.ctx.profile(True)
    r.ctx.profile_reset()
    nprof = 3
    for _ in range(nprof):
        opt.step()
    stages = r.ctx.profile_read()
    r.ctx.profile(False)
    stage_ms = {k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1] > 0}
    log("[bench] stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in stage_ms.items()))
    E, C = pair_counts(r, torch)
    c = r.counters()
    floats = 14 + 3 * ((w.scene.sh_degree + 1) ** 2 - 1)
    units = {"gaussians": w.scene.n, "pairs": w.scene.n * len(w.cams), "visible": int(c.visible),
             "keys": int(c.keys), "examined": E, "composited": C, "pixels": w.n_pixels,
             "trainable": floats * w.scene.n, "floats_per_gaussian": floats}
    floors = stage_floors(units)
    fractions = roofline_fractions(floors, stage_ms, ms_batched)
    log("[bench] roofline fraction per stage: " + ", ".join(f"{k} {v:.3f}" for k, v in fractions["per_stage"].items())
        + f"; step {fractions['step']:.3f} (sum of floors {fractions['step_floor_ms']:.3f} ms)")
    # dominant kernel and its roofline position
    dom = max(("composite", "composite_bwd"), key=lambda k: stage_ms.get(k, 0.0))
    per_c = FLOPS_FWD_COMPOSITED if dom == "composite" else FLOPS_BWD_COMPOSITED
    flops = FLOPS_TEST * E + per_c * C
    achieved = flops / (stage_ms[dom] * 1e-3) / 1e12
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            tj = json.load(open(tfile))
            if tj.get("kernel_stage") == dom and tj.get("source_hash") == _source_hash():
                traffic = tj.get("bytes_per_launch")
        except Exception:
            traffic = None
    roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
            "units": {"examined_pairs": E, "composited_pairs": C,
                      "flops_per_examined": FLOPS_TEST, "flops_per_composited": per_c},
            "avg_ms": round(stage_ms[dom], 4)}

    wave_w, schedule = r.wave_w, r.schedule
    # ---- plain as defined for the metric: 16x16 tiles, batch depth 64 ----------
    ms_plain = None
    if args.plain_steps > 0:
        plain_params = params.clone()
        del opt, r
        torch.cuda.empty_cache()
        rp = Renderer(w.cams, w.scene.n, w.scene.sh_degree, loss_mode=1, **PLAIN_SHAPE)
        rp.fit_capacity(pert)
        rp.fit_capacity(plain_params)
        # images do not depend on the launch shape: the same targets serve
        optp = Optimizer(rp, plain_params, targets, stream=stream)
        ms_plain = time_plain(optp, "16x16 tiles, batch depth 64")
        del optp, rp, plain_params
        torch.cuda.empty_cache()
    else:
        del opt, r

    cpu = None
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        cpu = cpu_baseline(w, args.cpu_seconds)
        cpu["single_core"] = single_core_oracle()
        log(f"[bench] cpu baseline {cpu['value']:.3g} steps/s on {cpu['cores']} threads ({cpu['cpu_model']}, "
            f"nproc {cpu['nproc']}); single core: {cpu['single_core']} ({time.perf_counter() - t:.1f} s)")

    others = None
    if not args.no_configs:
        del targets, params, pert
        torch.cuda.empty_cache()
        others = {f"cfg{k}": config_rate(k, shape, 10, 2, torch, log) for k in (1, 2, 3, 5)}
        # Gaussian freezing: cfg4 with half of the model in the frozen pool
        others["cfg4_half_frozen"] = config_rate(4, shape, 10, 2, torch, log, frozen=0.5)
        # delta codecs and client replay after each step of the dynamics workload
        others["cfg5_stream"] = stream_rate(shape, 8, torch, log)
        # object transforms and DC relighting on the device before each step
        others["cfg5_dynamics"] = dynamics_rate(shape, 8, torch, log)
        # preculling by grid cells: a large world seen from a camera rig
        others["rig2M"] = rig_rate(False, False, shape, 10, 2, torch, log)
        others["rig2M_grouped"] = rig_rate(False, True, shape, 10, 2, torch, log)
        others["rig2M_grouped_precull"] = rig_rate(True, True, shape, 10, 2, torch, log)
        # the same with the Gaussians of the cells no view sees in the frozen pool
        others["rig2M_grouped_frozen"] = rig_rate(False, True, shape, 10, 2, torch, log, freeze_unseen=True)
        others["rig2M_grouped_frozen_precull"] = rig_rate(True, True, shape, 10, 2, torch, log, freeze_unseen=True)

    out = {
        "metric": METRIC, "value": round(1000.0 / ms_batched, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_batched, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded; perturbed-copy targets rendered on the GPU)",
        "config": {"workload": f"{w.name}: {w.scene.n} Gaussians SH{w.scene.sh_degree}, {len(w.cams)} views "
                               f"({w.n_pixels} px, mixed 640x360/1280x720/1920x1080), batched step "
                               "replayed from a HIP graph",
                   "gaussians": w.scene.n, "views": len(w.cams), "pixels": w.n_pixels,
                   "tile": f"{tile[0]}x{tile[1]}", "batch_depth": batch, "pixels_per_thread": ppt,
                   "wave_w": wave_w, "schedule": schedule,
                   "autotuned": tuned is not None,
                   "keys": int(c.keys), "visible_pairs": int(c.visible), "parallelism": "1 GPU"},
        "views_per_s": round(len(w.cams) * 1000.0 / ms_batched, 2),
        "plain": None if ms_plain is None else {"value": round(1000.0 / ms_plain, 3), "unit": "steps/s",
                                                "ms_per_step": round(ms_plain, 4),
                                                "shape": "16x16 tiles, batch depth 64, 1 px/thread, eager, "
                                                         "one view per launch"},
        "batched_over_plain": None if ms_plain is None else round(ms_plain / ms_batched, 3),
        "plain_tuned_shape": None if ms_plain_tuned is None else {
            "value": round(1000.0 / ms_plain_tuned, 3), "unit": "steps/s", "ms_per_step": round(ms_plain_tuned, 4)},
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "roofline_stages": dict(fractions, floors=floors, units=units),
        "roofline": roof,
        "cpu_baseline": cpu,
        "other_workloads": others,
    }
    print(json.dumps(out), flush=True)


def _source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2604_02851_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
