"""ctypes front end of the FP64 CPU oracle (gsoracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library; inputs are the float32 arrays of the seeded generators.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gsoracle.cpp")
LIB = os.path.join(HERE, "libgsoracle.so")

GROUPS = ("opacity", "sh_dc", "sh_rest", "mean", "log_scale", "quat")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP contraction off, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c++17",
                               "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32, u32, dbl, flt = ctypes.c_int64, ctypes.c_int, ctypes.c_uint32, ctypes.c_double, ctypes.c_float
        params = [P, P, P, P, P, i64, i32]
        L.or_sh_basis.argtypes = [i32, P, P, P]
        L.or_project.argtypes = params + [P, i32, P, P, P, P]
        L.or_tile_lists.argtypes = params + [P, i32, i32, i32, P, i64, P]
        L.or_tile_lists.restype = i64
        L.or_render.argtypes = params + [P, i32, P, i32, i32, P, P, P, P]
        L.or_render_alternatives.argtypes = params + [P, i32, P, P, i32, P, P]
        L.or_backward.argtypes = params + [P, i32, P, P, i32, i32, dbl, P, P, P, P, P, P]
        L.or_adam.argtypes = [P, P, P, P, i64, flt, flt, flt, flt, i32, P, P, P]
        L.or_delta.argtypes = [P, P, P, i64, u32, flt, P]
        L.or_delta.restype = i64
        L.or_codec_encode.argtypes = [P, P, P, i64, u32, P, P, P, P, P, u32, P]
        L.or_codec_encode.restype = i64
        L.or_codec_apply.argtypes = [P, P, i64, P, i64, P, P, P, P, u32]
        L.or_codec_apply.restype = u32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _scene_args(scene):
    arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in
            (scene.mean, scene.log_scale, scene.quat, scene.opacity_logit, scene.sh)]
    return arrs, [_p(a) for a in arrs] + [ctypes.c_int64(scene.n), ctypes.c_int(scene.sh_degree)]


def n_params(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


def sh_basis(deg: int, d):
    d = np.ascontiguousarray(d, dtype=np.float64)
    nk = (deg + 1) ** 2
    Y = np.zeros(16)
    dY = np.zeros(48)
    lib().or_sh_basis(deg, _p(d), _p(Y), _p(dY))
    return Y[:nk], dY[:nk * 3].reshape(nk, 3)


@dataclass
class Projection:
    visible: np.ndarray   # [V, N] bool
    zbits: np.ndarray     # [V, N] uint32
    rec: np.ndarray       # [V, N, 16] u,w,A,B,C,a,b,c,o,r,g,b,pre_r,pre_g,pre_b,z
    rect: np.ndarray      # [V, N, 4] px0,py0,px1,py1


def project(scene, cams) -> Projection:
    cams = np.ascontiguousarray(cams)
    V, N = len(cams), scene.n
    vis = np.zeros(V * N, np.uint8)
    zb = np.zeros(V * N, np.uint32)
    rec = np.zeros(V * N * 16, np.float64)
    rect = np.zeros(V * N * 4, np.int32)
    keep, args = _scene_args(scene)
    lib().or_project(*args, _p(cams), V, _p(vis), _p(zb), _p(rec), _p(rect))
    return Projection(vis.reshape(V, N).astype(bool), zb.reshape(V, N), rec.reshape(V, N, 16), rect.reshape(V, N, 4))


def tile_layout(cams, tile_w: int, tile_h: int):
    tiles = [((int(c["width"]) + tile_w - 1) // tile_w) * ((int(c["height"]) + tile_h - 1) // tile_h) for c in cams]
    base = np.concatenate([[0], np.cumsum(tiles)]).astype(np.int64)
    return base


def tile_lists(scene, cams, tile_w: int, tile_h: int | None = None):
    """(values [K] uint32 = v*N+i, ranges [tiles, 2] uint32)."""
    tile_h = tile_h or tile_w
    cams = np.ascontiguousarray(cams)
    base = tile_layout(cams, tile_w, tile_h)
    ranges = np.zeros(int(base[-1]) * 2, np.uint32)
    keep, args = _scene_args(scene)
    K = lib().or_tile_lists(*args, _p(cams), len(cams), tile_w, tile_h, None, 0, _p(ranges))
    vals = np.zeros(max(K, 1), np.uint32)
    K = lib().or_tile_lists(*args, _p(cams), len(cams), tile_w, tile_h, _p(vals), K, _p(ranges))
    return vals[:K], ranges.reshape(-1, 2)


def pixel_offsets(cams):
    hw = [int(c["width"]) * int(c["height"]) for c in cams]
    return np.concatenate([[0], np.cumsum(hw)]).astype(np.int64)


@dataclass
class Render:
    image: np.ndarray     # [3*P] planar per view (views packed)
    T: np.ndarray         # [P]
    n_contrib: np.ndarray # [P]
    flags: np.ndarray     # [P] near-threshold decisions met

    def view_image(self, cams, v):
        off = pixel_offsets(cams)
        H, W = int(cams[v]["height"]), int(cams[v]["width"])
        return self.image[3 * off[v]: 3 * off[v + 1]].reshape(3, H, W)


def render(scene, cams, bg=(0.0, 0.0, 0.0), rows=None) -> Render:
    cams = np.ascontiguousarray(cams)
    P = int(pixel_offsets(cams)[-1])
    img = np.zeros(3 * P)
    T = np.ones(P)
    nc = np.zeros(P, np.int32)
    fl = np.zeros(P, np.int32)
    bgv = np.asarray(bg, np.float64)
    r0, r1 = (0, 0) if rows is None else rows
    keep, args = _scene_args(scene)
    lib().or_render(*args, _p(cams), len(cams), _p(bgv), r0, r1, _p(img), _p(T), _p(nc), _p(fl))
    return Render(img, T, nc, fl)


def render_alternatives(scene, cams, view: int, pix_xy, bg=(0.0, 0.0, 0.0)):
    """For each (x, y): array [k, 5] of (r, g, b, T, n) over the outcomes of
    the pixel's near-threshold decisions (row 0 is the primary outcome)."""
    cams = np.ascontiguousarray(cams)
    pix = np.ascontiguousarray(np.asarray(pix_xy, np.int32).reshape(-1, 2))
    out = np.zeros(len(pix) * 16 * 5)
    cnt = np.zeros(len(pix), np.int32)
    bgv = np.asarray(bg, np.float64)
    keep, args = _scene_args(scene)
    lib().or_render_alternatives(*args, _p(cams), view, _p(bgv), _p(pix), len(pix), _p(out), _p(cnt))
    out = out.reshape(len(pix), 16, 5)
    return [out[q, :cnt[q]] for q in range(len(pix))]


@dataclass
class Backward:
    grad: np.ndarray      # [nparam, N]
    scale: np.ndarray     # [nparam, N]  |J|^T sum |2D terms|
    slack: np.ndarray     # [nparam, N]  branch / sign-ambiguity allowance
    scale_t: np.ndarray   # [nparam, N]  |J|^T sum |2D terms| * E_p (transmittance condition)
    loss: float
    image: np.ndarray     # primary image [3*P]

    def split(self, arr, sh_degree):
        """Split an [nparam, N] array into the parameter tensors."""
        return {"mean": arr[0:3], "log_scale": arr[3:6], "quat": arr[6:10],
                "opacity_logit": arr[10], "sh": arr[11:]}


def backward(scene, cams, upstream, mode: int, loss_mode: int = 0, bg=(0.0, 0.0, 0.0),
             kink: float = 2e-5) -> Backward:
    """mode 0: `upstream` is dL/dimage; mode 1: L1 against target `upstream`
    (loss_mode 0 = sum over pixels, 1 = mean per view, summed over views)."""
    cams = np.ascontiguousarray(cams)
    npar = n_params(scene.sh_degree)
    N = scene.n
    P = int(pixel_offsets(cams)[-1])
    up = np.ascontiguousarray(upstream, dtype=np.float32).reshape(-1)
    assert up.shape[0] == 3 * P
    g = np.zeros(npar * N)
    s = np.zeros(npar * N)
    k = np.zeros(npar * N)
    t = np.zeros(npar * N)
    loss = np.zeros(1)
    img = np.zeros(3 * P)
    bgv = np.asarray(bg, np.float64)
    keep, args = _scene_args(scene)
    lib().or_backward(*args, _p(cams), len(cams), _p(bgv), _p(up), mode, loss_mode, float(kink),
                      _p(g), _p(s), _p(k), _p(t), _p(loss), _p(img))
    return Backward(g.reshape(npar, N), s.reshape(npar, N), k.reshape(npar, N), t.reshape(npar, N),
                    float(loss[0]), img)


def adam(theta, g, m, v, lr, beta1, beta2, eps, step):
    """One Adam step on float32 arrays; returns FP64 (theta, m, v)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float32).reshape(-1) for a in (theta, g, m, v)]
    n = arrs[0].shape[0]
    to, mo, vo = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().or_adam(*[_p(a) for a in arrs], n, float(lr), float(beta1), float(beta2), float(eps), int(step),
                  _p(to), _p(mo), _p(vo))
    shp = np.shape(theta)
    return to.reshape(shp), mo.reshape(shp), vo.reshape(shp)


def group_arrays(scene):
    """The six streamed attribute groups as ([width][N] float32 views)."""
    n = scene.n
    sh = scene.sh
    return [scene.opacity_logit.reshape(1, n), sh[0:3], sh[3:], scene.mean, scene.log_scale, scene.quat]


def delta_capacity_words(n: int, sh_degree: int, mask: int = 0x3F) -> int:
    widths = [1, 3, 3 * ((sh_degree + 1) ** 2 - 1), 3, 3, 4]
    return 6 + sum(n * (1 + w) for g, w in enumerate(widths) if (mask >> g) & 1)


def delta(cur_scene, base_scene, mask: int = 0x3F, tau: float = 1e-3):
    """Delta extraction; updates `base_scene` in place; returns the words."""
    n = cur_scene.n
    cur = [np.ascontiguousarray(a) for a in group_arrays(cur_scene)]
    base = group_arrays(base_scene)
    for b in base:
        assert b.flags["C_CONTIGUOUS"] or b.size == 0
    widths = np.array([a.shape[0] for a in cur], np.int32)
    cp = (ctypes.c_void_p * 6)(*[a.ctypes.data for a in cur])
    bp = (ctypes.c_void_p * 6)(*[b.ctypes.data for b in base])
    out = np.zeros(delta_capacity_words(n, cur_scene.sh_degree, mask), np.uint32)
    w = lib().or_delta(cp, bp, _p(widths), n, mask, float(np.float32(tau)), _p(out))
    return out[:w]


def codec_row_words(mode: int, bits: int, width: int) -> int:
    if mode == 0:
        return width
    per = 32 // bits
    return (width + per - 1) // per


def codec_capacity_words(n: int, sh_degree: int, codecs, mask: int = 0x3F) -> int:
    widths = [1, 3, 3 * ((sh_degree + 1) ** 2 - 1), 3, 3, 4]
    return 9 + sum(n * (1 + codec_row_words(codecs[g][0], codecs[g][1], widths[g]))
                   for g in range(6) if (mask >> g) & 1)


def _codec_arrays(codecs):
    assert len(codecs) == 6
    modes = np.array([c[0] for c in codecs], np.int32)
    bits = np.array([c[1] for c in codecs], np.int32)
    steps = np.array([c[2] for c in codecs], np.float32)
    los = np.array([c[3] for c in codecs], np.float32)
    taus = np.array([c[4] for c in codecs], np.float32)
    return modes, bits, steps, los, taus


def delta_encode(cur_scene, base_scene, codecs, mask: int = 0x3F, epoch: int = 0):
    """Delta codecs (residual coding for means and scales, quantized updates
    for the other groups, Sec. 3.5; bit widths, steps and rounding are a
    reading, written out in the C source).  codecs: six (mode, bits, step, lo,
    rel_tau) tuples in group order.  Updates `base_scene` in place to what the
    receiver reconstructs; returns the packet words."""
    n = cur_scene.n
    cur = [np.ascontiguousarray(a) for a in group_arrays(cur_scene)]
    base = group_arrays(base_scene)
    for b in base:
        assert b.flags["C_CONTIGUOUS"] or b.size == 0
    widths = np.array([a.shape[0] for a in cur], np.int32)
    modes, bits, steps, los, taus = _codec_arrays(codecs)
    cp = (ctypes.c_void_p * 6)(*[a.ctypes.data for a in cur])
    bp = (ctypes.c_void_p * 6)(*[b.ctypes.data for b in base])
    out = np.zeros(codec_capacity_words(n, cur_scene.sh_degree, codecs, mask), np.uint32)
    w = lib().or_codec_encode(cp, bp, _p(widths), n, mask, _p(modes), _p(bits), _p(steps), _p(los), _p(taus),
                              int(epoch), _p(out))
    return out[:w]


def delta_apply(model_scene, packet, codecs, epoch: int = 0) -> int:
    """Client replay of one packet onto the receiver's model (in place).
    Returns the status bits (1 epoch mismatch, 2 malformed); nothing is
    applied unless the status is 0."""
    n = model_scene.n
    model = group_arrays(model_scene)
    for b in model:
        assert b.flags["C_CONTIGUOUS"] or b.size == 0
    widths = np.array([a.shape[0] for a in model], np.int32)
    modes, bits, steps, los, _ = _codec_arrays(codecs)
    mp = (ctypes.c_void_p * 6)(*[a.ctypes.data for a in model])
    pk = np.ascontiguousarray(packet, np.uint32)
    return int(lib().or_codec_apply(mp, _p(widths), n, _p(pk), pk.size, _p(modes), _p(bits), _p(steps), _p(los),
                                    int(epoch)))


def freeze_partition(rows_all, rows_active, flags, n_active):
    """Gaussian freezing (active and frozen pools): the stable partition that
    moves the active Gaussians flagged for freezing behind the ones that stay
    active, ahead of the previously frozen ones.

    rows_all: list of [r, N] arrays (parameters, baselines, ids) permuted along
    the Gaussian axis; rows_active: list of [r, n_active] arrays (optimizer
    moments) restricted to the Gaussians that stay active.  Returns
    (permuted rows_all, compacted rows_active, new active count, order) where
    order[j] is the old index of the Gaussian now at j."""
    flags = np.asarray(flags).astype(bool)
    assert flags.shape == (n_active,)
    keep = np.nonzero(~flags)[0]
    moved = np.nonzero(flags)[0]
    n = rows_all[0].shape[-1] if rows_all else n_active
    order = np.concatenate([keep, moved, np.arange(n_active, n)]).astype(np.int64)
    out_all = [np.ascontiguousarray(a[..., order]) for a in rows_all]
    out_act = [np.ascontiguousarray(a[..., keep]) for a in rows_active]
    return out_all, out_act, len(keep), order


def cell_of(mean, origin, cell_size, dims):
    """Preculling grid (Sec. 3.3): the cell of each mean, evaluated in FP32 as
    t = (p - origin) / cell_size per axis, cell = cx + dims0 (cy + dims1 cz);
    means outside the grid (or NaN) get the extra index dims0 dims1 dims2."""
    m = np.asarray(mean, np.float32)
    o = np.asarray(origin, np.float32).reshape(3, 1)
    t = (m - o) / np.float32(cell_size)
    d = np.asarray(dims, np.int64).reshape(3, 1)
    inside = np.all((t >= 0) & (t < d.astype(np.float32)), axis=0)
    idx = np.floor(np.where(inside, t, 0)).astype(np.int64)
    c = idx[0] + d[0, 0] * (idx[1] + d[1, 0] * idx[2])
    return np.where(inside, c, int(np.prod(dims))).astype(np.int64)


def cell_order(cells, n_active, n_cells):
    """Grouping the model by preculling cell (Sec. 3.3: Gaussians belong to
    grid cells): within the active prefix and within the frozen suffix
    separately, Gaussians ordered by cell, equal cells in their old order;
    cell values of n_cells or more count as n_cells (outside the grid).

    Written as the rank definition of a stable sort: the new position of
    Gaussian i in its pool [lo, hi) is lo + #{j in pool: key_j < key_i} +
    #{j in pool, j < i: key_j == key_i}.  Returns order, order[k] = old index
    of the Gaussian now at k."""
    key = [min(int(c), int(n_cells)) for c in np.asarray(cells).reshape(-1)]
    n = len(key)
    order = np.empty(n, np.int64)
    for lo, hi in ((0, int(n_active)), (int(n_active), n)):
        for i in range(lo, hi):
            less = sum(1 for j in range(lo, hi) if key[j] < key[i])
            tie = sum(1 for j in range(lo, i) if key[j] == key[i])
            order[lo + less + tie] = i
    return order


# ---- scene dynamics (Sec. 3.4) ------------------------------------------------

def _rot_of_quat(q):
    """3x3 rotation of the unit quaternion (w, x, y, z) = q / |q| (FP64)."""
    q = np.asarray(q, np.float64)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _hamilton(a, b):
    """Quaternion product a b, (w, x, y, z) order; b may be [4, m]."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def object_transform(mean, quat, object_of, transforms):
    """Rigid-object dynamics (Sec. 3.4: Gaussians carry object identifiers and
    follow the engine's object transforms before each optimization).  Each
    object k moves by the rigid motion x -> R_k (x - p_k) + p_k + t_k, given
    as transforms[k] = (q_k (w, x, y, z), p_k pivot, t_k translation) with
    R_k the rotation of q_k / |q_k|; its Gaussians' means follow it and their
    orientations compose as q_k/|q_k| * quat (scales, opacity and colour do
    not change).  object_of[i] < 0 or >= the number of objects: static.
    FP64, rounded once to FP32.  Returns new (mean, quat) arrays."""
    mean = np.asarray(mean, np.float32)
    quat = np.asarray(quat, np.float32)
    out_m, out_q = mean.copy(), quat.copy()
    obj = np.asarray(object_of, np.int64)
    for k, (q, p, t) in enumerate(transforms):
        idx = np.nonzero(obj == k)[0]
        if idx.size == 0:
            continue
        R = _rot_of_quat(q)
        p = np.asarray(p, np.float64).reshape(3, 1)
        t = np.asarray(t, np.float64).reshape(3, 1)
        mu = mean[:, idx].astype(np.float64)
        out_m[:, idx] = (R @ (mu - p) + p + t).astype(np.float32)
        qu = np.asarray(q, np.float64)
        qu = qu / np.linalg.norm(qu)
        out_q[:, idx] = _hamilton(qu, quat[:, idx].astype(np.float64)).astype(np.float32)
    return out_m, out_q


SH_C0 = 1.0 / (2.0 * np.sqrt(np.pi))


def relight_dc(sh, gain):
    """Relighting restricted to the diffuse DC term (Sec. 3.4 combines the
    Gaussians' SH with lighting SH by a rule the paper does not give): the DC
    colour C0 dc + 1/2 of Gaussian i, channel c, is scaled by gain[c or 0, i]
    (gain [1, N] for all channels alike or [3, N]); a gain of exactly 1 leaves
    the coefficient as it is.  FP64, rounded once to FP32.  Returns new sh."""
    sh = np.asarray(sh, np.float32)
    gain = np.asarray(gain, np.float32)
    out = sh.copy()
    for c in range(3):
        g = gain[c if gain.shape[0] == 3 else 0].astype(np.float64)
        dc = sh[c].astype(np.float64)
        new = ((SH_C0 * dc + 0.5) * g - 0.5) / SH_C0
        out[c] = np.where(g == 1.0, sh[c], new.astype(np.float32))
    return out


def append_rows(old, add, n_active):
    """Model expansion (Sec. 3.3: new Gaussians join the trainable part, the
    trainable tensors and the optimizer state are extended): per row, the
    active prefix, then the k new Gaussians, then the frozen suffix.  For
    optimizer moments pass the active rows as `old`, n_active = their count,
    and zeros as `add`."""
    old = np.asarray(old)
    add = np.asarray(add)
    return np.concatenate([old[..., :n_active], add, old[..., n_active:]], axis=-1)

