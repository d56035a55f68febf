"""Helpers shared by the GPU parity tests (imported by tests only)."""
from __future__ import annotations

import numpy as np
import torch

IMG_TOL = 1e-5          # absolute per channel (FP32 image vs FP64 oracle)
GRAD_REL = 1e-4         # relative
GRAD_ABS = 1e-6         # absolute floor
# FP32 accumulation allowance: |error| <= EPS_ACC * (sum of |terms|), the
# oracle's magnitude scale; 2^-17 is 128 units of FP32 rounding.  It covers
# the per-term evaluation error (an alpha evaluated in FP32 is off by up to
# ~14 units at the 3-sigma cut-off, where the exponent's argument is largest)
# and the rounding of summing up to millions of terms in an order set by
# atomics.
EPS_ACC = 2.0 ** -17
# FP32 transmittance allowance: the forward product of (1 - alpha) and the
# adjoint's reciprocal chain leave each rebuilt transmittance within
# c u E_p of its exact value, E_p = sum over the pixel's composited splats
# of 1 / (1 - alpha); the float32 emulation of that arithmetic
# (test_fp32_bounds) measures c <= 2.94, so 4 units are allowed.  The
# oracle's depth-weighted scale carries E_p.
EPS_T = 4 * 2.0 ** -24


def renderer_for(w, tile=(16, 16), batch=64, bg=(0.0, 0.0, 0.0), loss_mode=0, cap=None, ppt=1, wave_w=0,
                 schedule=0):
    from paper_2604_02851_amd.renderer import Renderer
    r = Renderer(w.cams, w.scene.n, w.scene.sh_degree, tile=tile, batch_depth=batch, bg=bg, loss_mode=loss_mode,
                 key_capacity=cap, pixels_per_thread=ppt, wave_w=wave_w, schedule=schedule)
    return r


def seg_np(r, name, dtype, v0=0, nv=None):
    torch.cuda.synchronize()
    return r.ctx.segment(r.ws, name, v0, nv).cpu().numpy().view(dtype)


def compare_images(oracle, w, gpu_img, bg=(0.0, 0.0, 0.0), tol=IMG_TOL, ref=None):
    """Every pixel within tol of the oracle, or, at pixels with
    near-threshold decisions, within tol of one of their outcomes.
    Returns (max error at clean pixels, number of pixels matched through an
    alternative outcome)."""
    ref = ref if ref is not None else oracle.render(w.scene, w.cams, bg=bg)
    off = oracle.pixel_offsets(w.cams)
    worst = 0.0
    via_alt = 0
    for v, cam in enumerate(w.cams):
        H, W = int(cam["height"]), int(cam["width"])
        a = gpu_img[3 * off[v]:3 * off[v + 1]].reshape(3, H * W).astype(np.float64)
        b = ref.image[3 * off[v]:3 * off[v + 1]].reshape(3, H * W)
        d = np.abs(a - b).max(0)
        fl = ref.flags[off[v]:off[v + 1]] > 0
        clean = d[~fl]
        if clean.size:
            worst = max(worst, float(clean.max()))
        bad_clean = np.nonzero((d > tol) & ~fl)[0]
        assert bad_clean.size == 0, f"view {v}: {bad_clean.size} pixels off by up to {d[bad_clean].max():.3g}"
        bad = np.nonzero((d > tol) & fl)[0]
        if bad.size:
            xy = np.stack([bad % W, bad // W], 1)
            alts = oracle.render_alternatives(w.scene, w.cams, v, xy, bg=bg)
            for q, p in enumerate(bad):
                best = np.abs(alts[q][:, :3] - a[:, p][None, :]).max(1).min()
                assert best <= tol, f"view {v} pixel {p}: no outcome within tol (best {best:.3g})"
            via_alt += bad.size
    return worst, via_alt


def flat_grads(grads) -> np.ndarray:
    n = grads.n
    return np.concatenate([t.detach().cpu().numpy().reshape(-1, n) for t in grads.tensors()], 0).astype(np.float64)


def grad_tol(b, rel=GRAD_REL, floor=GRAD_ABS):
    return rel * np.abs(b.grad) + floor + EPS_ACC * b.scale + EPS_T * b.scale_t + b.slack


def grad_report(g_gpu: np.ndarray, b, rel=GRAD_REL, floor=GRAD_ABS):
    """Checks |g_gpu - g| <= rel |g| + floor + EPS_ACC scale + EPS_T scale_t
    + slack and returns statistics, including which widening terms the
    elements outside the strict bar rel |g| + floor needed:
      via_acc / via_t / via_slack: the elements that pass with the strict bar
        plus the accumulation term, then plus the transmittance term, then
        plus the slack (each counted at the first sum that admits them);
      only_acc / only_t / only_slack: the elements that would fail if that
        one term were dropped from the full bar."""
    err = np.abs(g_gpu - b.grad)
    strict = rel * np.abs(b.grad) + floor
    acc, tt, sl = EPS_ACC * b.scale, EPS_T * b.scale_t, b.slack
    tol = grad_tol(b, rel, floor)
    ok = err <= tol
    ratio = err / tol
    s1, s2 = strict + acc, strict + acc + tt
    return {
        "via_acc": int(((err > strict) & (err <= s1)).sum()),
        "via_t": int(((err > s1) & (err <= s2)).sum()),
        "via_slack": int(((err > s2) & ok).sum()),
        "only_acc": int((ok & (err > tol - acc)).sum()),
        "only_t": int((ok & (err > tol - tt)).sum()),
        "only_slack": int((ok & (err > tol - sl)).sum()),
        "max_err_over_tol": float(ratio.max()),
        "p50_err_over_tol": float(np.percentile(ratio, 50)),
        "p99_err_over_tol": float(np.percentile(ratio, 99)),
        "n": int(err.size),
        "fail": int((~ok).sum()),
        "strict_fail": int((err > strict).sum()),
        "max_rel_err_large": float((err / np.maximum(np.abs(b.grad), 1e-30))[np.abs(b.grad) > 1e-2].max()
                                   if (np.abs(b.grad) > 1e-2).any() else 0.0),
        "worst_idx": np.unravel_index(int(np.argmax(err / tol)), err.shape),
    }


def adam_check(oracle, theta0, g0, m0, v0, out_t, out_m, out_v, lr, b1, b2, eps, step):
    """Checks one Adam step of the library against the oracle's FP64 step on
    every element and returns the worst error / bound.  The hyperparameters
    reach the library as FP32 numbers, so the oracle gets the same rounded
    values.  Bounds, with u = 2^-24 and d = theta - theta' (oracle):
      m': 4u (beta1 |m| + (1 - beta1) |g|)    (a product, a fused add)
      v': 4u |v'|                             (a sum of non-negative terms)
      theta': 2u |theta'| + 16u |d| + 4u (|d| / |m'|) (beta1 |m| + (1 - beta1) |g|)
    (the final subtraction, the roundings of the update's own chain, and the
    rounding of m' carried through the update's factor d / m')."""
    f32 = lambda x: float(np.float32(x))
    u = 2.0 ** -24
    th, mo, vo = oracle.adam(theta0, g0, m0, v0, f32(lr), f32(b1), f32(b2), f32(eps), step)
    mg = f32(b1) * np.abs(m0) + (1 - f32(b1)) * np.abs(g0)
    assert (mo != 0).all()
    d = np.abs(np.asarray(theta0, np.float64) - th)
    tol_t = 2 * u * np.abs(th) + 16 * u * d + 4 * u * (d / np.abs(mo)) * mg
    worst = 0.0
    for got, ref, tol, what in ((out_t, th, tol_t, "theta"), (out_m, mo, 4 * u * mg, "m"), (out_v, vo, 4 * u * np.abs(vo), "v")):
        r = np.abs(got - ref) / tol
        worst = max(worst, float(r.max()))
        assert (r <= 1.0).all(), (what, float(r.max()))
    return worst
