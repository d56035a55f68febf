"""Pins of the oracle's projection stage (EWA splatting of prior 3DGS work,
Sec. 3.2.3): closed forms, invariances, a finite-difference linearisation of
the pinhole camera and library routines (scipy rotations, expit, SH)."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import expit, sph_harm_y

from oracle import brute
from paper_2604_02851_amd import scenes as S

F32 = np.float32


def _one(mean, log_scale, quat, opac=0.0, sh=None, deg=0):
    n = 1
    sh = np.zeros((3 * (deg + 1) ** 2, 1), F32) if sh is None else sh
    return S.Scene(np.asarray(mean, F32).reshape(3, n), np.asarray(log_scale, F32).reshape(3, n),
                   np.asarray(quat, F32).reshape(4, n), np.asarray([opac], F32), np.asarray(sh, F32), deg)


def _scene_of(cols):
    """Stack single-Gaussian scenes."""
    return S.Scene(*(np.concatenate([getattr(c, k) for c in cols], axis=-1) for k in
                     ("mean", "log_scale", "quat", "opacity_logit", "sh")), cols[0].sh_degree)


def test_isotropic_on_axis_closed_form(oracle):
    z0, sigma = 4.0, 0.05
    cams = S.cams_array([S.look_at((0, 0, z0), 96, 64)])
    sc = _one([0, 0, 0], [math.log(sigma)] * 3, [0.3, 0.1, -0.5, 0.8])
    pr = oracle.project(sc, cams)
    u, w, A, B, C, a, b, c = pr.rec[0, 0, :8]
    f = float(cams[0]["fx"])
    s = float(F32(sigma)) if False else math.exp(float(F32(math.log(sigma))))
    expect = (f * s / z0) ** 2 + float(F32(0.3))
    assert pr.visible[0, 0]
    assert abs(A - expect) < 1e-12 * expect and abs(C - expect) < 1e-12 * expect and abs(B) < 1e-12
    assert abs(u - 48.0) < 1e-12 and abs(w - 32.0) < 1e-12
    assert abs(a - 1 / expect) < 1e-12 and abs(c - 1 / expect) < 1e-12 and abs(b) < 1e-12


def test_rotation_about_view_axis_swaps_axes(oracle):
    cams = S.cams_array([S.look_at((0, 0, 5), 64, 64)])
    ls = [math.log(0.2), math.log(0.05), math.log(0.1)]
    q0 = Rotation.from_euler("z", 0.0).as_quat()          # (x, y, z, w)
    q90 = Rotation.from_euler("z", 90, degrees=True).as_quat()
    wxyz = lambda q: [q[3], q[0], q[1], q[2]]
    pr = oracle.project(_scene_of([_one([0, 0, 0], ls, wxyz(q0)), _one([0, 0, 0], ls, wxyz(q90))]), cams)
    A0, B0, C0 = pr.rec[0, 0, 2:5]
    A1, B1, C1 = pr.rec[0, 1, 2:5]
    assert abs(A0 - C1) < 1e-9 * A0 and abs(C0 - A1) < 1e-9 * C0 and abs(B0 + B1) < 1e-9 * max(A0, C0)
    assert abs(A0 - C0) > 1.0                               # genuinely anisotropic


def test_quaternion_sign_and_norm_invariance(oracle):
    rng = np.random.default_rng(3)
    cams = S.cams_array([S.look_at((0.5, 0.2, 4), 80, 60)])
    q = rng.normal(size=4).astype(F32)
    base = dict(mean=[0.1, -0.2, 0.3], log_scale=[-2.0, -2.5, -1.8])
    pr = oracle.project(_scene_of([_one(quat=q, **base), _one(quat=-q, **base), _one(quat=F32(4.0) * q, **base), _one(quat=F32(0.5) * q, **base)]), cams)
    for k in (1, 2, 3):
        assert np.allclose(pr.rec[0, 0, :12], pr.rec[0, k, :12], rtol=1e-12, atol=1e-12)


def _pinhole_linearisation(cam, mean, log_scale, quat, h=1e-6):
    """J_fd L L^T J_fd^T + 0.3 I with L = R(q) diag(e^s) from scipy and the
    camera's own projection differentiated by central differences."""
    Rq = Rotation.from_quat([quat[1], quat[2], quat[3], quat[0]]).as_matrix()
    L = Rq * np.exp(np.asarray(log_scale, np.float64))[None, :]
    mu = np.asarray(mean, np.float64)[:, None]
    cols = []
    for k in range(3):
        lk = L[:, k:k + 1]
        cols.append((brute.pinhole(cam, mu + h * lk) - brute.pinhole(cam, mu - h * lk))[:, 0] / (2 * h))
    Jl = np.stack(cols, 1)
    return Jl @ Jl.T + float(F32(0.3)) * np.eye(2), brute.pinhole(cam, mu)[:, 0]


def test_screen_covariance_matches_linearised_camera(oracle):
    rng = np.random.default_rng(11)
    sc = S.draw_scene(rng, 64, 1.0, 0)
    cams = S.cams_array([S.look_at((1.0, 0.5, 3.5), 160, 120)])
    pr = oracle.project(sc, cams)
    checked = 0
    for i in range(sc.n):
        if not pr.visible[0, i]:
            continue
        x = cams[0]["R"].astype(np.float64).reshape(3, 3) @ sc.mean[:, i].astype(np.float64) + cams[0]["t"]
        if abs(x[0] / x[2]) > 1.3 * 80 / cams[0]["fx"] or abs(x[1] / x[2]) > 1.3 * 60 / cams[0]["fy"]:
            continue                                   # guard band active
        S2, uv = _pinhole_linearisation(cams[0], sc.mean[:, i], sc.log_scale[:, i], sc.quat[:, i].astype(np.float64))
        A, B, C = pr.rec[0, i, 2:5]
        assert np.allclose([A, B, C], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-6, atol=1e-6)
        assert np.allclose(pr.rec[0, i, :2], uv, rtol=0, atol=1e-9)
        a, b, c = pr.rec[0, i, 5:8]
        assert np.allclose(np.array([[a, b], [b, c]]) @ np.array([[A, B], [B, C]]), np.eye(2), atol=1e-9)
        checked += 1
    assert checked > 20


def test_depth_key_is_fp32_expression(oracle):
    rng = np.random.default_rng(5)
    sc = S.draw_scene(rng, 500, 1.0, 0)
    cams = S.cams_array([S.look_at((0.3, -0.4, 3), 64, 64), S.look_at((2, 1, -2), 50, 70)])
    pr = oracle.project(sc, cams)
    for v in range(2):
        z = brute.depth_keys(sc.mean, cams[v])
        vis = pr.visible[v]
        assert np.array_equal(pr.zbits[v][vis], z.view(np.uint32)[vis])
        assert np.all(z[vis] >= F32(0.2))


def test_opacity_and_colour_from_library_routines(oracle):
    rng = np.random.default_rng(6)
    sc = S.draw_scene(rng, 200, 1.0, 3)
    cams = S.cams_array([S.look_at((0.2, 0.1, 3), 64, 64)])
    pr = oracle.project(sc, cams)
    vis = pr.visible[0]
    assert np.allclose(pr.rec[0, vis, 8], expit(sc.opacity_logit.astype(np.float64)[vis]), rtol=1e-14)
    campos = cams[0]["campos"].astype(np.float64)
    for i in np.nonzero(vis)[0][:40]:
        d = sc.mean[:, i].astype(np.float64) - campos
        d /= np.linalg.norm(d)
        th, ph = math.acos(max(-1.0, min(1.0, d[2]))), math.atan2(d[1], d[0])
        Y = []
        for l in range(4):
            for m in range(-l, l + 1):
                c = sph_harm_y(l, abs(m), th, ph)
                Y.append(c.real if m == 0 else math.sqrt(2) * (c.real if m > 0 else c.imag))
        f = sc.sh[:, i].astype(np.float64).reshape(16, 3)
        pre = 0.5 + np.asarray(Y) @ f
        assert np.allclose(pr.rec[0, i, 12:15], pre, atol=1e-12)
        assert np.allclose(pr.rec[0, i, 9:12], np.maximum(pre, 0), atol=1e-12)


def test_non_finite_and_behind_camera_are_culled(oracle):
    cams = S.cams_array([S.look_at((0, 0, 3), 64, 64)])
    good = _one([0, 0, 0], [-3, -3, -3], [1, 0, 0, 0])
    nan = _one([0, np.nan, 0], [-3, -3, -3], [1, 0, 0, 0])
    inf = _one([0, 0, 0], [-3, np.inf, -3], [1, 0, 0, 0])
    behind = _one([0, 0, 3.1], [-3, -3, -3], [1, 0, 0, 0])
    zeroq = _one([0, 0, 0], [-3, -3, -3], [0, 0, 0, 0])
    offscreen = _one([50, 0, 0], [-3, -3, -3], [1, 0, 0, 0])
    pr = oracle.project(_scene_of([good, nan, inf, behind, zeroq, offscreen]), cams)
    assert pr.visible[0].tolist() == [True, False, False, False, False, False]
