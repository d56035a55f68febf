"""Pins of the scene-dynamics oracle (Sec. 3.4: rigid objects follow engine
transforms; DC relighting; Sec. 3.3: appending to the trainable part) against
what geometry fixes: identity transforms change nothing, rigid motion keeps
distances within an object and moves the pivot by the translation, a half
turn about z negates x and y about the pivot, composing two motions equals
one motion by the composed quaternion, the rotation of the composed
quaternion is the product of rotations (the orientation follows the
object), and both agree with the configuration-5 harness's own host update;
relighting scales the DC colour exactly and a unit gain is the identity;
appending places the new Gaussians between the pools."""
import math

import numpy as np

from oracle import oracle as O
from paper_2604_02851_amd import scenes as S

F32 = np.float32


def _scene(n, seed):
    return S.draw_scene(np.random.default_rng(seed), n, 2.0, 2)


def test_identity_and_static():
    sc = _scene(400, 1)
    obj = np.random.default_rng(2).integers(-1, 3, 400)
    ident = [((1, 0, 0, 0), (0.3, -1, 2), (0, 0, 0))] * 3
    m, q = O.object_transform(sc.mean, sc.quat, obj, ident)
    assert np.array_equal(m, sc.mean) and np.array_equal(q, sc.quat)
    moves = [((0.9, 0.1, -0.3, 0.2), (1, 2, 3), (0.5, 0, -1))]
    m, q = O.object_transform(sc.mean, sc.quat, np.full(400, -1), moves)
    assert np.array_equal(m, sc.mean) and np.array_equal(q, sc.quat)
    m, q = O.object_transform(sc.mean, sc.quat, np.full(400, 5), moves)   # unknown object: static
    assert np.array_equal(m, sc.mean) and np.array_equal(q, sc.quat)


def test_rigid_motion_geometry():
    sc = _scene(300, 3)
    obj = np.zeros(300, np.int64)
    q = np.array([0.8, 0.2, -0.5, 0.1])
    p, t = np.array([0.4, -0.2, 1.0]), np.array([1.0, 2.0, -0.5])
    m, _ = O.object_transform(sc.mean, sc.quat, obj, [(q, p, t)])
    a, b = sc.mean.astype(np.float64), m.astype(np.float64)
    d0 = np.linalg.norm(a[:, :, None] - a[:, None, :], axis=0)
    d1 = np.linalg.norm(b[:, :, None] - b[:, None, :], axis=0)
    assert np.allclose(d0, d1, atol=1e-5)                        # distances kept
    mp, _ = O.object_transform(p.reshape(3, 1).astype(F32), sc.quat[:, :1], [0], [(q, p.astype(F32), t)])
    assert np.allclose(mp[:, 0], p + t, atol=1e-6)                 # the pivot moves by t
    half = [((0.0, 0.0, 0.0, 1.0), (1.0, 1.0, 0.0), (0, 0, 0))]    # half turn about z through (1, 1, 0)
    m2, _ = O.object_transform(sc.mean, sc.quat, obj, half)
    assert np.allclose(m2[0], 2.0 - sc.mean[0], atol=1e-6) and np.allclose(m2[1], 2.0 - sc.mean[1], atol=1e-6)
    assert np.array_equal(m2[2], sc.mean[2])


def test_composition_and_orientation():
    rng = np.random.default_rng(4)
    sc = _scene(200, 5)
    obj = np.zeros(200, np.int64)
    qa, qb = rng.normal(size=4), rng.normal(size=4)
    qa, qb = qa / np.linalg.norm(qa), qb / np.linalg.norm(qb)
    ta, tb = rng.normal(size=3), rng.normal(size=3)
    zero = np.zeros(3)
    m1, q1 = O.object_transform(sc.mean, sc.quat, obj, [(qa, zero, ta)])
    m2, q2 = O.object_transform(m1, q1, obj, [(qb, zero, tb)])
    Ra, Rb = O._rot_of_quat(qa), O._rot_of_quat(qb)
    qab = O._hamilton(qb, qa)
    assert np.allclose(O._rot_of_quat(qab), Rb @ Ra, atol=1e-12)   # rotation of a product
    m3, q3 = O.object_transform(sc.mean, sc.quat, obj, [(qab, zero, Rb @ ta + tb)])
    assert np.allclose(m2, m3, atol=2e-5) and np.allclose(q2, q3, atol=2e-6)
    # the Gaussian's covariance axes turn with the object: R(q' quat) = R_obj R(quat)
    for i in range(5):
        Ri = O._rot_of_quat(sc.quat[:, i].astype(np.float64))
        assert np.allclose(O._rot_of_quat(q1[:, i].astype(np.float64)), Ra @ Ri, atol=1e-6)


def test_matches_dynamics_harness():
    rng = np.random.default_rng(6)
    sc = _scene(3000, 7)
    dyn = S.Dynamics(np.random.default_rng(8), sc, n_objects=4, per_object=100)
    moved = sc.copy()
    moves, relit = dyn.step([moved])
    obj = np.full(sc.n, -1)
    transforms = []
    for k, (idx, axis, ang, tr) in enumerate(moves):
        obj[idx] = k
        c = sc.mean[:, idx].astype(np.float64).mean(1)
        transforms.append((np.r_[math.cos(ang / 2), math.sin(ang / 2) * axis], c, tr))
    m, q = O.object_transform(sc.mean, sc.quat, obj, transforms)
    assert np.allclose(m, moved.mean, atol=2e-6) and np.allclose(q, moved.quat, atol=2e-6)
    # the harness's relighting is a per-Gaussian gain on all channels
    gain = np.ones((1, sc.n), F32)
    gain[0, relit] = np.asarray(dyn_gain(moved, sc, relit), F32)
    out = O.relight_dc(sc.sh, gain)
    assert np.allclose(out[:3], moved.sh[:3], atol=1e-5) and np.array_equal(out[3:], sc.sh[3:])


def dyn_gain(moved, sc, relit):
    # the gain the harness drew, recovered from the DC colours it wrote
    c0 = O.SH_C0
    return (c0 * moved.sh[0, relit].astype(np.float64) + 0.5) / (c0 * sc.sh[0, relit].astype(np.float64) + 0.5)


def test_relight_dc_exact_scaling():
    sc = _scene(500, 9)
    rng = np.random.default_rng(10)
    g3 = rng.uniform(0.2, 2.0, (3, 500)).astype(F32)
    g3[:, ::7] = 1.0
    out = O.relight_dc(sc.sh, g3)
    c0 = O.SH_C0
    col0 = c0 * sc.sh[:3].astype(np.float64) + 0.5
    col1 = c0 * out[:3].astype(np.float64) + 0.5
    assert np.allclose(col1, col0 * g3, rtol=0, atol=1e-6)
    assert np.array_equal(out[:3, ::7], sc.sh[:3, ::7])            # unit gain: untouched
    assert np.array_equal(out[3:], sc.sh[3:])                      # higher bands untouched


def test_append_rows_between_pools():
    old = np.arange(2 * 10).reshape(2, 10)
    add = -np.arange(2 * 3).reshape(2, 3) - 1
    out = O.append_rows(old, add, 6)
    assert out.shape == (2, 13)
    for r in range(2):
        expect = [old[r, j] for j in range(6)] + [add[r, j] for j in range(3)] + [old[r, j] for j in range(6, 10)]
        assert out[r].tolist() == expect
    assert np.array_equal(O.append_rows(old, add[:, :0], 4), old)
