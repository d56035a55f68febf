"""Seeded synthetic inputs for the online 3DGS optimize step.

This module only draws random numbers and builds camera poses.  It holds none
of the renderer's or optimizer's arithmetic, so both the HIP path and the CPU
oracle can consume its arrays without sharing any of the method's code.

The paper measures on a custom game-engine scene that is not public (Sec. 4,
evaluation setup); the five workloads below stand in for it.  Their shapes:

  cfg1  1,000 Gaussians, means U[-1,1]^3, SH degree 0, one 128x128 view at
        distance 3.
  cfg2  100k Gaussians, means U[-5,5]^3, SH degree 3, one 800x800 view at
        distance 15.
  cfg3  500k Gaussians (as cfg2), 8 views 1280x720 on a ring of radius 8.
  cfg4  1M Gaussians (as cfg2), 16 views of mixed resolution on a sphere of
        radius U[6,12].
  cfg5  3M Gaussians (as cfg2), 4 views 1920x1080, plus rigid-object motion
        and DC rescaling of the appearance between steps (Sec. 3.4).

Common distributions: log-scales N(-3, 0.5) per axis (second argument is a
standard deviation), rotations uniform unit quaternions (w, x, y, z),
opacity logits N(0, 1), DC appearance such that the degree-0 colour is
U[0,1] per channel, higher SH bands N(0, 0.1).  Cameras look at the origin
with a 60 degree horizontal field of view, OpenCV axes (x right, y down,
z forward), principal point at the image centre.

All parameter arrays are planar float32 ("SoA"): mean[3][N], log_scale[3][N],
quat[4][N], opacity_logit[N], sh[(D+1)^2 * 3][N] with row (k*3 + channel).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 260402851

# Layout of one camera record; mirrors the C struct gs_camera (84 bytes).
CAM_DTYPE = np.dtype([
    ("R", "<f4", (9,)),       # world->camera rotation, row-major
    ("t", "<f4", (3,)),       # world->camera translation
    ("campos", "<f4", (3,)),  # camera centre in world space
    ("fx", "<f4"), ("fy", "<f4"), ("cx", "<f4"), ("cy", "<f4"),
    ("width", "<i4"), ("height", "<i4"),
])
assert CAM_DTYPE.itemsize == 84

RESOLUTIONS_MIXED = ((640, 360), (1280, 720), (1920, 1080))


@dataclass
class Scene:
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity_logit: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.opacity_logit.shape[0])

    def copy(self) -> "Scene":
        return Scene(self.mean.copy(), self.log_scale.copy(), self.quat.copy(),
                     self.opacity_logit.copy(), self.sh.copy(), self.sh_degree)

    def tensors(self):
        """(name, array) in the fixed parameter order."""
        return [("mean", self.mean), ("log_scale", self.log_scale), ("quat", self.quat),
                ("opacity_logit", self.opacity_logit), ("sh", self.sh)]


@dataclass
class Workload:
    name: str
    scene: Scene
    cams: np.ndarray            # CAM_DTYPE records
    tile_size: int = 16
    extra: dict = field(default_factory=dict)

    @property
    def n_pixels(self) -> int:
        return int(sum(int(c["width"]) * int(c["height"]) for c in self.cams))


def sh_coeff_count(degree: int) -> int:
    return (degree + 1) ** 2


def draw_scene(rng: np.random.Generator, n: int, extent: float, sh_degree: int) -> Scene:
    """Draw order: means, log-scales, quats, opacity logits, DC, higher bands."""
    mean = rng.uniform(-extent, extent, size=(3, n))
    log_scale = rng.normal(-3.0, 0.5, size=(3, n))
    q = rng.normal(0.0, 1.0, size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opacity_logit = rng.normal(0.0, 1.0, size=n)
    # DC coefficients spanning the range whose degree-0 colour is U[0,1]:
    # colour = 0.5 + Y00 * dc with Y00 = 1 / (2 sqrt(pi)).
    dc = rng.uniform(-0.5, 0.5, size=(3, n)) * (2.0 * math.sqrt(math.pi))
    nk = sh_coeff_count(sh_degree)
    sh = np.empty((nk * 3, n), dtype=np.float64)
    sh[0:3] = dc
    if nk > 1:
        sh[3:] = rng.normal(0.0, 0.1, size=((nk - 1) * 3, n))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f32(mean), f32(log_scale), f32(q), f32(opacity_logit), f32(sh), sh_degree)


def perturb(rng: np.random.Generator, s: Scene) -> Scene:
    """Perturbed copy used to render targets: additive N(0, sd) per tensor."""
    out = s.copy()
    out.mean += rng.normal(0, 0.05, size=s.mean.shape).astype(np.float32)
    out.log_scale += rng.normal(0, 0.1, size=s.log_scale.shape).astype(np.float32)
    out.quat += rng.normal(0, 0.05, size=s.quat.shape).astype(np.float32)
    out.opacity_logit += rng.normal(0, 0.25, size=s.opacity_logit.shape).astype(np.float32)
    out.sh += rng.normal(0, 0.05, size=s.sh.shape).astype(np.float32)
    return out


def look_at(eye, width: int, height: int, fov_x_deg: float = 60.0, target=(0.0, 0.0, 0.0)):
    """One CAM_DTYPE record for a pinhole camera at `eye` looking at `target`."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.array([0.0, 1.0, 0.0])
    if abs(float(f @ up)) > 0.999:
        up = np.array([0.0, 0.0, 1.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f])
    t = -R @ eye
    focal = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    rec = np.zeros((), dtype=CAM_DTYPE)
    rec["R"] = R.reshape(-1)
    rec["t"] = t
    rec["campos"] = eye
    rec["fx"] = focal
    rec["fy"] = focal
    rec["cx"] = width / 2.0
    rec["cy"] = height / 2.0
    rec["width"] = width
    rec["height"] = height
    return rec


def cams_array(recs) -> np.ndarray:
    return np.ascontiguousarray(np.array(list(recs), dtype=CAM_DTYPE))


def sphere_cams(rng: np.random.Generator, count: int, rmin: float, rmax: float,
                resolutions=RESOLUTIONS_MIXED) -> np.ndarray:
    recs = []
    for _ in range(count):
        d = rng.normal(0.0, 1.0, size=3)
        d /= np.linalg.norm(d)
        r = rng.uniform(rmin, rmax)
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        recs.append(look_at(d * r, w, h))
    return cams_array(recs)


def ring_cams(count: int, radius: float, width: int, height: int) -> np.ndarray:
    recs = []
    for k in range(count):
        a = 2.0 * math.pi * k / count
        recs.append(look_at((radius * math.cos(a), 0.0, radius * math.sin(a)), width, height))
    return cams_array(recs)


def streams(cfg: int, count: int = 8):
    """Independent sub-streams: gaussians, cameras, perturbation, targets,
    finite-difference samples, dynamics, spare, spare."""
    ss = np.random.SeedSequence(SEED_BASE + cfg)
    return [np.random.default_rng(c) for c in ss.spawn(count)]


def workload(cfg: int, n_override: int | None = None) -> Workload:
    """The five configured workloads (optionally with fewer Gaussians)."""
    g, c, p, t, fd, dyn, _, _ = streams(cfg)
    if cfg == 1:
        scene = draw_scene(g, n_override or 1000, 1.0, 0)
        cams = cams_array([look_at((0.0, 0.0, 3.0), 128, 128)])
        target = t.uniform(0.0, 1.0, size=(3, 128, 128)).astype(np.float32)
        return Workload("cfg1", scene, cams, 16, {"target": target, "rng_fd": fd})
    scene = draw_scene(g, n_override or {2: 100_000, 3: 500_000, 4: 1_000_000, 5: 3_000_000}[cfg], 5.0, 3)
    if cfg == 2:
        cams = cams_array([look_at((0.0, 0.0, 15.0), 800, 800)])
    elif cfg == 3:
        cams = ring_cams(8, 8.0, 1280, 720)
    elif cfg == 4:
        cams = sphere_cams(c, 16, 6.0, 12.0)
    elif cfg == 5:
        cams = sphere_cams(c, 4, 6.0, 12.0, resolutions=((1920, 1080),))
    else:
        raise ValueError(cfg)
    extra = {"perturbed": perturb(p, scene), "rng_fd": fd, "rng_dyn": dyn}
    return Workload(f"cfg{cfg}", scene, cams, 16, extra)


def small_workload(seed: int, n: int, extent: float, sh_degree: int, sizes, dist: float = 3.0,
                   tile_size: int = 16) -> Workload:
    """Small scenes for parity tests: ragged image sizes, several views."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    scene = draw_scene(rng, n, extent, sh_degree)
    recs = []
    for k, (w, h) in enumerate(sizes):
        d = rng.normal(0.0, 1.0, size=3)
        d /= np.linalg.norm(d)
        recs.append(look_at(d * dist * rng.uniform(0.9, 1.2), w, h))
    cams = cams_array(recs)
    target = [rng.uniform(0.0, 1.0, size=(3, h, w)).astype(np.float32) for (w, h) in sizes]
    return Workload(f"small{seed}", scene, cams, tile_size,
                    {"target": target, "perturbed": perturb(rng, scene), "rng": rng})


# ---------------------------------------------------------------------------
# Scene dynamics between steps (rigid objects + DC rescale), Sec. 3.4.
# Applied on the host in float32 to the model and the target copy alike.
# ---------------------------------------------------------------------------

def _heading(k: int, views: int, arc: float) -> float:
    """Heading of camera k of a rig spread evenly over `arc` degrees (a full
    turn places the cameras 360/views apart; a partial arc includes both ends)."""
    if arc >= 360.0:
        return 2 * math.pi * k / views
    return math.radians(arc) * (k / (views - 1) if views > 1 else 0.0)


def rig_workload(seed: int, n: int, half: float = 20.0, height: float = 2.0, views: int = 4,
                 size=(320, 180), sh_degree: int = 3, arc: float = 360.0) -> Workload:
    """A wide, flat scene (means uniform in [-half, half] x [-height, height] x
    [-half, half]) seen from a rig of cameras at the origin looking outward at
    headings evenly spaced over `arc` degrees, as around a player in a large
    world: each view sees only part of the model, and with an arc below a
    full turn part of the model is seen by no view (the preculling workload)."""
    rng = np.random.default_rng(np.random.SeedSequence(260402851 + 1000 + seed))
    scene = draw_scene(rng, n, 1.0, sh_degree)
    scene.mean[0] *= np.float32(half)
    scene.mean[1] *= np.float32(height)
    scene.mean[2] *= np.float32(half)
    w, h = size
    recs = [look_at((0.0, 0.0, 0.0), w, h, 60.0,
                    target=(math.cos(_heading(k, views, arc)), 0.0, math.sin(_heading(k, views, arc))))
            for k in range(views)]
    return Workload(f"rig{seed}", scene, cams_array(recs), 16, {"perturbed": perturb(rng, scene)})


def _quat_mul(a, b):
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def _axis_angle_R(axis, ang):
    x, y, z = axis
    c, s = math.cos(ang), math.sin(ang)
    C = 1 - c
    return np.array([[c + x * x * C, x * y * C - z * s, x * z * C + y * s],
                     [y * x * C + z * s, c + y * y * C, y * z * C - x * s],
                     [z * x * C - y * s, z * y * C + x * s, c + z * z * C]])


class Dynamics:
    """20 rigid objects of 7,500 Gaussians each (5% of 3M), nearest to random
    centres; 10% of Gaussians get their DC colour rescaled each step."""

    def __init__(self, rng: np.random.Generator, scene: Scene, n_objects: int = 20,
                 per_object: int | None = None, extent: float = 5.0):
        self.rng = rng
        n = scene.n
        per_object = per_object or max(1, (n * 5 // 100) // n_objects)
        centres = rng.uniform(-extent, extent, size=(n_objects, 3))
        mu = scene.mean.T.astype(np.float64)
        # nearest-centre assignment, then each object keeps its closest members
        d2 = np.stack([((mu - c) ** 2).sum(1) for c in centres], axis=1)
        owner = d2.argmin(1)
        self.members = []
        for k in range(n_objects):
            idx = np.nonzero(owner == k)[0]
            idx = idx[np.argsort(d2[idx, k], kind="stable")[:per_object]]
            self.members.append(np.sort(idx))

    def step(self, scenes):
        """Mutate every Scene in `scenes` identically (float32)."""
        rng = self.rng
        moves = []
        for idx in self.members:
            axis = rng.normal(size=3)
            axis /= np.linalg.norm(axis)
            ang = math.radians(rng.uniform(0.0, 5.0))
            tr = rng.normal(0.0, 0.02, size=3)
            moves.append((idx, axis, ang, tr))
        n = scenes[0].n
        relit = rng.choice(n, size=n // 10, replace=False)
        gain = rng.uniform(0.5, 1.5, size=relit.shape[0])
        y00 = 1.0 / (2.0 * math.sqrt(math.pi))
        for s in scenes:
            for idx, axis, ang, tr in moves:
                R = _axis_angle_R(axis, ang)
                mu = s.mean[:, idx].astype(np.float64)
                c = mu.mean(1, keepdims=True)
                s.mean[:, idx] = (R @ (mu - c) + c + tr[:, None]).astype(np.float32)
                qr = np.array([math.cos(ang / 2)] + list(math.sin(ang / 2) * axis))
                q = s.quat[:, idx].astype(np.float64)
                s.quat[:, idx] = _quat_mul(qr[:, None], q).astype(np.float32)
            dc = s.sh[0:3, relit].astype(np.float64)
            s.sh[0:3, relit] = (((y00 * dc + 0.5) * gain - 0.5) / y00).astype(np.float32)
        return moves, relit
