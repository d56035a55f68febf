"""Dense brute-force reference renderer in torch FP64 (tiny scenes only).

TEST INFRASTRUCTURE ONLY.  A second, structurally different statement of the
same definition the oracle implements, used to pin the oracle:
  * every pixel is tested against every Gaussian (no rectangles, no rows),
  * depth order comes from an explicit numpy lexsort,
  * the backward pass is torch autograd, not a hand-written adjoint.
Projection uses the camera's pinhole model and scipy's rotation routine.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from scipy.spatial.transform import Rotation

F32 = np.float32
ALPHA_MAX = float(F32(0.99))
ALPHA_MIN = float(F32(1.0) / F32(255.0))
T_MIN = float(F32(1e-4))
DILATION = float(F32(0.3))
GUARD = float(F32(1.3))
NEAR = F32(0.2)


def depth_keys(mean: np.ndarray, cam) -> np.ndarray:
    """FP32 camera-space depth, each operation rounded (numpy float32)."""
    R = cam["R"].astype(F32)
    t2 = F32(cam["t"][2])
    z = (R[6] * mean[0] + R[7] * mean[1]) + R[8] * mean[2]
    return (z + t2).astype(F32)


def sh_basis_torch(deg: int, d: torch.Tensor) -> torch.Tensor:
    """Real SH with the (-1)^m sign, from scipy's complex harmonics' closed
    forms re-derived as polynomials of the unit direction."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    s = 1.0 / math.sqrt(math.pi)
    out = [torch.full_like(x, 0.5 * s)]
    if deg >= 1:
        c = math.sqrt(3.0) / 2.0 * s
        out += [-c * y, c * z, -c * x]
    if deg >= 2:
        a, b, c = math.sqrt(15) / 2 * s, math.sqrt(5) / 4 * s, math.sqrt(15) / 4 * s
        out += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z, c * (x * x - y * y)]
    if deg >= 3:
        a = math.sqrt(35 / 2) / 4 * s
        b = math.sqrt(105) / 2 * s
        c = math.sqrt(21 / 2) / 4 * s
        e = math.sqrt(7) / 4 * s
        f = math.sqrt(105) / 4 * s
        out += [-a * y * (3 * x * x - y * y), b * x * y * z, -c * y * (4 * z * z - x * x - y * y),
                e * z * (2 * z * z - 3 * x * x - 3 * y * y), -c * x * (4 * z * z - x * x - y * y),
                f * z * (x * x - y * y), -a * x * (x * x - 3 * y * y)]
    return torch.stack(out, dim=-1)


def to_torch(scene, requires_grad=True):
    ts = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=requires_grad) for k, v in scene.tensors()}
    return ts


FIELDS = ("u", "w", "a", "b", "c", "o", "r", "g", "bl")   # screen-space quantities per splat


def project_torch(ts: dict, sh_degree: int, cam):
    """Differentiable projection of every Gaussian into one view (FP64).
    Returns (fields, keep, order): fields maps each name of FIELDS to an [N]
    tensor (projected mean u, w; conic [[a, b], [b, c]]; opacity o; colour
    r, g, bl after the clamp at 0), keep the numpy mask of Gaussians that
    pass the near plane and have a positive screen determinant, order the
    depth order (FP32 depth bits, then index)."""
    W_img, H_img = int(cam["width"]), int(cam["height"])
    Rw = torch.tensor(cam["R"].astype(np.float64).reshape(3, 3))
    tw = torch.tensor(cam["t"].astype(np.float64))
    fx, fy, cx, cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    mean = ts["mean"]                      # [3, N]
    N = mean.shape[1]
    mean_np = ts["mean"].detach().numpy().astype(F32)
    z32 = depth_keys(mean_np, cam)
    order = np.lexsort((np.arange(N), z32.view(np.uint32)))
    keep = z32 >= NEAR

    x = Rw @ mean + tw[:, None]            # camera space [3, N]
    # covariance: Sigma = L L^T with L = R(q) diag(exp(s))
    q = ts["quat"]
    qn = q / q.norm(dim=0, keepdim=True)
    # rotation matrices through scipy for the values, rebuilt differentiably
    w_, x_, y_, z_ = qn
    Rq = torch.stack([
        torch.stack([1 - 2 * (y_ * y_ + z_ * z_), 2 * (x_ * y_ - w_ * z_), 2 * (x_ * z_ + w_ * y_)]),
        torch.stack([2 * (x_ * y_ + w_ * z_), 1 - 2 * (x_ * x_ + z_ * z_), 2 * (y_ * z_ - w_ * x_)]),
        torch.stack([2 * (x_ * z_ - w_ * y_), 2 * (y_ * z_ + w_ * x_), 1 - 2 * (x_ * x_ + y_ * y_)]),
    ])                                     # [3, 3, N]
    ref = Rotation.from_quat(torch.stack([x_, y_, z_, w_], 1).detach().numpy()).as_matrix()
    assert np.allclose(ref, Rq.detach().permute(2, 0, 1).numpy(), atol=1e-12), "quaternion convention"
    L = Rq * torch.exp(ts["log_scale"])[None, :, :]
    Sig = torch.einsum("ikn,jkn->ijn", L, L)
    M = torch.einsum("ab,bcn,dc->adn", Rw, Sig, Rw)
    limx = GUARD * (0.5 * W_img) / fx
    limy = GUARD * (0.5 * H_img) / fy
    txz = torch.clamp(x[0] / x[2], -limx, limx)
    tyz = torch.clamp(x[1] / x[2], -limy, limy)
    zeros = torch.zeros_like(x[2])
    J = torch.stack([torch.stack([fx / x[2], zeros, -fx * txz / x[2]]),
                     torch.stack([zeros, fy / x[2], -fy * tyz / x[2]])])   # [2, 3, N]
    S2 = torch.einsum("ikn,kln,jln->ijn", J, M, J)
    A = S2[0, 0] + DILATION
    B = S2[0, 1]
    C = S2[1, 1] + DILATION
    det = A * C - B * B
    keep = keep & (det.detach().numpy() > 0)
    campos = torch.tensor(cam["campos"].astype(np.float64))
    dv = mean - campos[:, None]
    d = (dv / dv.norm(dim=0, keepdim=True)).T          # [N, 3]
    Y = sh_basis_torch(sh_degree, d)                    # [N, K]
    nk = (sh_degree + 1) ** 2
    sh = ts["sh"].reshape(nk, 3, N)
    col = torch.clamp(torch.einsum("nk,kcn->cn", Y, sh) + 0.5, min=0.0)  # [3, N]
    fields = {"u": fx * x[0] / x[2] + cx, "w": fy * x[1] / x[2] + cy, "a": C / det, "b": -B / det, "c": A / det,
              "o": torch.sigmoid(ts["opacity_logit"]), "r": col[0], "g": col[1], "bl": col[2]}
    return fields, keep, order


def _per_gaussian(v, N):
    a = np.asarray(v, np.float64)
    return np.broadcast_to(a, (N,)) if a.ndim == 0 else a


def composite_torch(fields: dict, keep, order, H_img: int, W_img: int, bg=(0.0, 0.0, 0.0), cutoff=-4.5,
                    alpha_min=ALPHA_MIN, t_min=T_MIN, clamp_at=ALPHA_MAX, stats: bool = False):
    """Front-to-back compositing of every pixel against every Gaussian in
    depth order (FP64, differentiable in the fields).  The thresholds may be
    scalars or per-Gaussian arrays, so that a test can force the outcome of
    one Gaussian's decision: the ellipse test P >= cutoff, the skip test
    alpha >= alpha_min, the stop test T (1 - alpha) < t_min and the clamp
    o e^P >= clamp_at (a clamped alpha is ALPHA_MAX).  Returns (image [3,H,W],
    T [H,W], n [H,W]) and, with stats, also E [H,W] = sum over the composited
    splats of 1 / (1 - alpha)."""
    N = fields["u"].shape[0]
    cut, amin, tmin, camp = (_per_gaussian(v, N) for v in (cutoff, alpha_min, t_min, clamp_at))
    py, px = torch.meshgrid(torch.arange(H_img, dtype=torch.float64), torch.arange(W_img, dtype=torch.float64),
                            indexing="ij")
    px = px.reshape(-1) + 0.5
    py = py.reshape(-1) + 0.5
    npx = px.shape[0]
    T = torch.ones(npx, dtype=torch.float64)
    Cacc = torch.zeros(3, npx, dtype=torch.float64)
    done = torch.zeros(npx, dtype=torch.bool)
    ncon = torch.zeros(npx, dtype=torch.int64)
    E = torch.zeros(npx, dtype=torch.float64)
    u, v, ca, cb, cc, o = (fields[k] for k in ("u", "w", "a", "b", "c", "o"))
    col = torch.stack([fields["r"], fields["g"], fields["bl"]])
    for i in order:
        if not keep[i]:
            continue
        dx = px - u[i]
        dy = py - v[i]
        P = -0.5 * (ca[i] * dx * dx + cc[i] * dy * dy) - cb[i] * dx * dy
        oG = o[i] * torch.exp(P)
        clamped = oG.detach() >= camp[i]
        alpha = torch.where(clamped, torch.full_like(oG, ALPHA_MAX), oG)
        ok = (P.detach() >= cut[i]) & (alpha.detach() >= amin[i]) & ~done
        Tn = T * (1 - alpha)
        stop = ok & (Tn.detach() < tmin[i])
        take = ok & ~stop
        done = done | stop
        w = torch.where(take, alpha * T, torch.zeros_like(T))
        Cacc = Cacc + col[:, i:i + 1] * w[None, :]
        T = torch.where(take, Tn, T)
        ncon = ncon + take.long()
        E = E + torch.where(take, 1.0 / (1.0 - alpha.detach()), torch.zeros_like(E))
    bgt = torch.tensor(bg, dtype=torch.float64)[:, None]
    img = Cacc + T[None, :] * bgt
    out = (img.reshape(3, H_img, W_img), T.reshape(H_img, W_img), ncon.reshape(H_img, W_img))
    return out + (E.reshape(H_img, W_img),) if stats else out


def render_torch(ts: dict, sh_degree: int, cam, bg=(0.0, 0.0, 0.0), **thresholds):
    """Returns (image [3,H,W], T [H,W], n [H,W]) in FP64 with autograd;
    keyword thresholds as in composite_torch."""
    fields, keep, order = project_torch(ts, sh_degree, cam)
    return composite_torch(fields, keep, order, int(cam["height"]), int(cam["width"]), bg, **thresholds)


def pinhole(cam, p: np.ndarray) -> np.ndarray:
    """Project world points [3, M] with the camera's pinhole model (FP64)."""
    R = cam["R"].astype(np.float64).reshape(3, 3)
    t = cam["t"].astype(np.float64)
    x = R @ p + t[:, None]
    return np.stack([cam["fx"] * x[0] / x[2] + cam["cx"], cam["fy"] * x[1] / x[2] + cam["cy"]])
