"""Pins of the oracle's analytic gradient (differentiable rendering of the
optimized 3DGS parameters, Sec. 3.2.3; loss against the reference views,
Sec. 3.1): torch autograd on the dense brute force, central finite
differences, multi-view linearity and the L1 upstream."""
import numpy as np
import pytest
import torch

from oracle import brute
from paper_2604_02851_amd import scenes as S

F32 = np.float32
NAMES = ("mean", "log_scale", "quat", "opacity_logit", "sh")


def _flat(d, n):
    return np.concatenate([np.asarray(d[k]).reshape(-1, n) for k in NAMES], 0)


@pytest.mark.parametrize("seed,deg,sizes", [(11, 0, [(22, 18)]), (12, 3, [(20, 20), (17, 13)])])
def test_matches_torch_autograd(oracle, seed, deg, sizes):
    w = S.small_workload(seed, 90, 1.0, deg, sizes, dist=2.5)
    bg = (0.1, 0.0, 0.2)
    rng = np.random.default_rng(seed)
    P = w.n_pixels
    G = rng.normal(size=3 * P).astype(F32)
    b = oracle.backward(w.scene, w.cams, G, mode=0, bg=bg)
    ts = brute.to_torch(w.scene)
    off = oracle.pixel_offsets(w.cams)
    total = 0
    for v, cam in enumerate(w.cams):
        img, _, _ = brute.render_torch(ts, deg, cam, bg)
        Gv = torch.tensor(G[3 * off[v]:3 * off[v + 1]].astype(np.float64)).reshape(img.shape)
        total = total + (img * Gv).sum()
    total.backward()
    ref = _flat({k: ts[k].grad.numpy() for k in NAMES}, w.scene.n)
    tol = 1e-9 * (np.abs(ref) + b.scale) + b.slack
    assert np.all(np.abs(b.grad - ref) <= tol + 1e-13)
    assert np.abs(ref).max() > 1.0


def _fd_check(oracle, w, G, bg, idx_list, rel=1e-4):
    """Central differences of L = <G, image> on float32 parameters."""
    b = oracle.backward(w.scene, w.cams, G, mode=0, bg=bg)
    base = oracle.render(w.scene, w.cams, bg=bg)
    checked = 0
    for (name, row, i) in idx_list:
        arr = getattr(w.scene, name)
        a2 = arr.reshape(-1, w.scene.n)
        x0 = float(a2[row, i])
        grads = []
        for h in (1e-3, 5e-4):
            hh = h * max(1.0, abs(x0))
            vals, steps, same = [], [], True
            for sgn in (1, -1):
                sc = w.scene.copy()
                t = getattr(sc, name).reshape(-1, sc.n)
                t[row, i] = F32(x0 + sgn * hh)
                r = oracle.render(sc, w.cams, bg=bg)
                same &= np.array_equal(r.n_contrib, base.n_contrib)
                vals.append(float(np.dot(G.astype(np.float64), r.image)))
                steps.append(float(t[row, i]))
            if not same:
                break
            grads.append((vals[0] - vals[1]) / (steps[0] - steps[1]))
        if len(grads) < 2 or abs(grads[0] - grads[1]) > 1e-3 * max(abs(grads[1]), 1e-3):
            continue            # a decision changed or the function is not smooth here
        row_of = {"mean": 0, "log_scale": 3, "quat": 6, "opacity_logit": 10, "sh": 11}[name] + row
        an = b.grad[row_of, i]
        assert abs(an - grads[1]) <= rel * max(abs(an), 1e-2) + b.slack[row_of, i], (name, row, i, an, grads)
        checked += 1
    return checked


def test_matches_finite_differences(oracle):
    w = S.small_workload(21, 60, 1.0, 3, [(28, 24)], dist=2.5)
    bg = (0.0, 0.0, 0.0)
    G = np.random.default_rng(1).normal(size=3 * w.n_pixels).astype(F32)
    r = oracle.render(w.scene, w.cams, bg=bg)
    pr = oracle.project(w.scene, w.cams)
    vis = np.nonzero(pr.visible[0])[0]
    rng = np.random.default_rng(2)
    picks = []
    for name, rows in (("mean", 3), ("log_scale", 3), ("quat", 4), ("opacity_logit", 1), ("sh", 48)):
        for _ in range(6):
            picks.append((name, int(rng.integers(rows)), int(rng.choice(vis))))
    assert _fd_check(oracle, w, G, bg, picks) >= 20


def test_multi_view_gradients_are_sums(oracle):
    w = S.small_workload(31, 150, 1.0, 2, [(30, 22), (25, 27), (16, 40)])
    G = np.random.default_rng(3).normal(size=3 * w.n_pixels).astype(F32)
    off = oracle.pixel_offsets(w.cams)
    all3 = oracle.backward(w.scene, w.cams, G, mode=0)
    acc = np.zeros_like(all3.grad)
    for v in range(3):
        acc += oracle.backward(w.scene, w.cams[v:v + 1], G[3 * off[v]:3 * off[v + 1]], mode=0).grad
    assert np.allclose(all3.grad, acc, rtol=1e-12, atol=1e-12)


def test_l1_upstream_and_loss(oracle):
    w = S.small_workload(41, 150, 1.0, 1, [(26, 21), (18, 18)])
    tgt = np.concatenate([t.reshape(-1) for t in w.extra["target"]]).astype(F32)
    off = oracle.pixel_offsets(w.cams)
    for loss_mode in (0, 1):
        b1 = oracle.backward(w.scene, w.cams, tgt, mode=1, loss_mode=loss_mode)
        img = b1.image
        wv = np.concatenate([np.full(3 * (off[v + 1] - off[v]), 1.0 if loss_mode == 0 else 1.0 / (3 * (off[v + 1] - off[v])))
                             for v in range(2)])
        G = (np.sign(img - tgt.astype(np.float64)) * wv).astype(F32)
        b0 = oracle.backward(w.scene, w.cams, G, mode=0)
        # (the mean weight 1/(3HW) is rounded to float32 in the mode-0 call)
        rel = 1e-12 if loss_mode == 0 else 1e-7
        assert np.all(np.abs(b1.grad - b0.grad) <= rel * (np.abs(b0.grad) + b0.scale) + 1e-15)
        assert abs(b1.loss - np.sum(wv * np.abs(img - tgt))) < 1e-9 * max(1.0, b1.loss)
