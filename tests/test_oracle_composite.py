"""Pins of the oracle's forward render (front-to-back alpha compositing of
prior 3DGS work, Sec. 3.2.3; the optimizer renders the model from the
reference views, Sec. 3.1): closed forms, invariants and the dense torch
brute force."""
import math

import numpy as np
import pytest
import torch

from oracle import brute
from paper_2604_02851_amd import scenes as S

F32 = np.float32
AMAX = float(F32(0.99))


def _iso(mean, sigma, opac_logit, rgb):
    dc = (np.asarray(rgb, np.float64) - 0.5) * 2 * math.sqrt(math.pi)
    return S.Scene(np.asarray(mean, F32).reshape(3, 1), np.full((3, 1), math.log(sigma), F32),
                   np.array([[1], [0], [0], [0]], F32), np.array([opac_logit], F32),
                   dc.astype(F32).reshape(3, 1), 0)


def _stack(parts):
    return S.Scene(*(np.concatenate([getattr(p, k) for p in parts], axis=-1) for k in
                     ("mean", "log_scale", "quat", "opacity_logit", "sh")), parts[0].sh_degree)


def _closed_form_alpha(sc, i, cam, px, py):
    """On-axis isotropic Gaussian at depth z: Sigma2 = ((f s / z)^2 + 0.3) I."""
    z = float(cam["campos"][2]) - float(sc.mean[2, i])
    s = math.exp(float(sc.log_scale[0, i]))
    var = (float(cam["fx"]) * s / z) ** 2 + float(F32(0.3))
    dx = px + 0.5 - float(cam["cx"])
    dy = py + 0.5 - float(cam["cy"])
    P = -0.5 * (dx * dx + dy * dy) / var
    o = 1.0 / (1.0 + math.exp(-float(sc.opacity_logit[i])))
    a = min(AMAX, o * math.exp(P))
    if P < -4.5 or a < float(F32(1) / F32(255)):
        return 0.0
    return a


def _col(sc, i):
    return np.maximum(0.0, 0.5 + sc.sh[0:3, i].astype(np.float64) / (2 * math.sqrt(math.pi)))


def test_single_gaussian_closed_form(oracle):
    cam = S.look_at((0, 0, 3), 33, 27)
    cams = S.cams_array([cam])
    sc = _iso([0, 0, 0], 0.15, 0.7, [0.9, 0.2, 0.4])
    bg = (0.1, 0.3, 0.6)
    r = oracle.render(sc, cams, bg=bg)
    img = r.image.reshape(3, 27, 33)
    for py in range(27):
        for px in range(33):
            a = _closed_form_alpha(sc, 0, cams[0], px, py)
            exp = _col(sc, 0) * a + (1 - a) * np.asarray(bg)
            assert np.allclose(img[:, py, px], exp, atol=1e-13)
            assert abs(r.T[py * 33 + px] - (1 - a)) < 1e-13
    assert r.n_contrib.max() == 1 and r.n_contrib.sum() > 20


def test_two_depth_separated_gaussians(oracle):
    cams = S.cams_array([S.look_at((0, 0, 3), 31, 31)])
    front = _iso([0, 0, 0.5], 0.03, 0.2, [1, 0, 0])
    back = _iso([0, 0, -0.5], 0.05, 1.5, [0, 0, 1])
    for order in ([front, back], [back, front]):   # input order must not matter
        sc = _stack(order)
        r = oracle.render(sc, cams)
        img = r.image.reshape(3, 31, 31)
        fi, bi = (0, 1) if order[0] is front else (1, 0)
        for py in range(31):
            for px in range(31):
                a1 = _closed_form_alpha(sc, fi, cams[0], px, py)
                a2 = _closed_form_alpha(sc, bi, cams[0], px, py)
                exp = _col(sc, fi) * a1 + _col(sc, bi) * a2 * (1 - a1)
                assert np.allclose(img[:, py, px], exp, atol=1e-13)
                assert abs(r.T[py * 31 + px] - (1 - a1) * (1 - a2)) < 1e-13


def test_stacked_opaque_gaussians_stop_on_fp32_threshold(oracle):
    # Three identical fully opaque Gaussians: (1 - fl32(0.99))^2 falls below
    # fl32(1e-4), so only the first is composited (with decimal constants in
    # FP64 the second one would be).
    cams = S.cams_array([S.look_at((0, 0, 3), 9, 9)])
    sc = _stack([_iso([0, 0, 0], 0.2, 12.0, [0.25, 0.5, 0.75])] * 3)
    r = oracle.render(sc, cams)
    c = 4 * 9 + 4
    assert r.n_contrib[c] == 1
    assert r.T[c] == 1 - AMAX
    assert (1 - AMAX) ** 2 < float(F32(1e-4)) and (1 - 0.99) ** 2 > 1e-4
    assert np.allclose(r.image.reshape(3, 81)[:, c], np.array([0.25, 0.5, 0.75]) * AMAX, atol=1e-6)


def test_transmittance_and_background_invariants(oracle):
    w = S.small_workload(1, 300, 1.0, 3, [(40, 28), (17, 33)])
    r0 = oracle.render(w.scene, w.cams, bg=(0, 0, 0))
    r1 = oracle.render(w.scene, w.cams, bg=(1, 1, 1))
    assert np.all(r0.T <= 1) and np.all(r0.T >= float(F32(1e-4)))
    # the image is affine in the background with slope T_final
    off = oracle.pixel_offsets(w.cams)
    for v in range(2):
        a = r0.image[3 * off[v]:3 * off[v + 1]].reshape(3, -1)
        b = r1.image[3 * off[v]:3 * off[v + 1]].reshape(3, -1)
        assert np.allclose(b - a, r0.T[off[v]:off[v + 1]][None, :], atol=1e-12)
    assert np.array_equal(r0.n_contrib, r1.n_contrib)


def test_permutation_invariance(oracle):
    w = S.small_workload(2, 250, 1.0, 2, [(36, 36)])
    r0 = oracle.render(w.scene, w.cams, bg=(0.2, 0.2, 0.2))
    perm = np.random.default_rng(0).permutation(w.scene.n)
    sc = S.Scene(w.scene.mean[:, perm].copy(), w.scene.log_scale[:, perm].copy(), w.scene.quat[:, perm].copy(),
                 w.scene.opacity_logit[perm].copy(), w.scene.sh[:, perm].copy(), w.scene.sh_degree)
    z = brute.depth_keys(w.scene.mean, w.cams[0])
    assert len(np.unique(z)) == len(z)                     # distinct depths
    r1 = oracle.render(sc, w.cams, bg=(0.2, 0.2, 0.2))
    assert np.array_equal(r0.image, r1.image) and np.array_equal(r0.T, r1.T)


@pytest.mark.parametrize("seed,deg,sizes", [(3, 0, [(24, 20)]), (4, 3, [(19, 23), (16, 16)])])
def test_matches_dense_brute_force(oracle, seed, deg, sizes):
    w = S.small_workload(seed, 120, 1.0, deg, sizes, dist=2.5)
    bg = (0.05, 0.1, 0.15)
    r = oracle.render(w.scene, w.cams, bg=bg)
    off = oracle.pixel_offsets(w.cams)
    ts = brute.to_torch(w.scene, requires_grad=False)
    for v, cam in enumerate(w.cams):
        img, T, n = brute.render_torch(ts, deg, cam, bg)
        H, W = int(cam["height"]), int(cam["width"])
        fl = r.flags[off[v]:off[v + 1]].reshape(H, W) > 0
        mine = r.image[3 * off[v]:3 * off[v + 1]].reshape(3, H, W)
        diff = np.abs(mine - img.numpy()).max(0)
        assert diff[~fl].max() < 1e-12
        assert np.array_equal(r.n_contrib[off[v]:off[v + 1]].reshape(H, W)[~fl], n.numpy()[~fl])
        assert np.allclose(r.T[off[v]:off[v + 1]].reshape(H, W)[~fl], T.numpy()[~fl], atol=1e-12)
    assert r.n_contrib.max() > 3


def test_alternatives_include_primary(oracle):
    w = S.workload(1)
    r = oracle.render(w.scene, w.cams)
    idx = np.nonzero(r.flags)[0]
    assert len(idx) > 0
    xy = np.stack([idx % 128, idx // 128], 1)
    alts = oracle.render_alternatives(w.scene, w.cams, 0, xy)
    img = r.image.reshape(3, -1)
    for q, p in enumerate(idx):
        assert len(alts[q]) >= 2
        assert np.allclose(alts[q][0, :3], img[:, p], atol=0) and alts[q][0, 3] == r.T[p]
