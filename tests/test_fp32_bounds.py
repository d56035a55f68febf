"""Pin of the FP32 transmittance allowance used by the gradient parity bar.

The GPU composites in FP32 and its adjoint rebuilds each transmittance from
the final one by dividing by (1 - alpha) with the hardware reciprocal
(front-to-back compositing of prior 3DGS work, Sec. 3.2.3, walked back to
front).  The gradient bar allows EPS_T * scale_t, i.e. a relative error of
EPS_T * E_p on the transmittance of every composited splat, where
E_p = sum over the pixel's composited splats of 1 / (1 - alpha) in FP64.

This test emulates that arithmetic in numpy float32 on synthetic pixels
(per-splat conic, offset and opacity drawn to cover clamped alphas, deep
lists and powers near the 3-sigma cut-off): the power and exponential in
FP32 from FP32-rounded inputs, a one-unit error on every hardware exp2 and
reciprocal result (the accuracy the ISA documents for them), the forward
product T (1 - alpha) and the backward chain T * rcp(1 - alpha), each
operation rounded.  It compares every rebuilt transmittance with the FP64
one and requires the error to stay within the allowance; the measured worst
ratio is printed."""
import numpy as np

from gpu_util import EPS_T

F32 = np.float32
U = 2.0 ** -24
AMAX32, AMIN32, TMIN32 = F32(0.99), F32(1) / F32(255), F32(1e-4)
LOG2E32 = F32(1.4426950408889634)


def _ulp_noise(x: np.ndarray, rng) -> np.ndarray:
    """x moved by -1, 0 or +1 unit in the last place (float32)."""
    k = rng.integers(-1, 2, size=x.shape)
    up = np.nextafter(x, F32(np.inf))
    dn = np.nextafter(x, F32(-np.inf))
    return np.where(k > 0, up, np.where(k < 0, dn, x)).astype(F32)


def _pixel(rng, n, kind):
    """One pixel's splat list: conic (a, b, c) with a positive determinant,
    offsets (dx, dy) and opacity."""
    a = rng.uniform(0.02, 2.0, n)
    c = rng.uniform(0.02, 2.0, n)
    b = rng.uniform(-0.9, 0.9, n) * np.sqrt(a * c)
    if kind == "clamped":        # near-opaque splats close to their centres
        q = rng.uniform(0.0, 0.02, n)
        o = rng.uniform(0.98, 0.99999, n)
    elif kind == "cutoff":       # powers close to -4.5 with large opacities
        q = rng.uniform(8.0, 9.0, n)
        o = rng.uniform(0.4, 0.99999, n)
    else:                        # deep lists of faint splats
        q = rng.uniform(0.0, 9.0, n)
        o = rng.uniform(0.0, 0.2, n)
    # offsets with the quadratic form q = a dx^2 + 2 b dx dy + c dy^2
    ang = rng.uniform(0, 2 * np.pi, n)
    ex, ey = np.cos(ang), np.sin(ang)
    form = a * ex * ex + 2 * b * ex * ey + c * ey * ey
    r = np.sqrt(q / form)
    return a, b, c, r * ex, r * ey, o


def _walk(rng, a, b, c, dx, dy, o):
    """(FP64 T before each composited splat, FP32 forward T before it, FP32
    rebuilt T, FP64 E_p), or None when the two sides decide differently."""
    P64 = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
    a32, b32, c32, dx32, dy32 = (x.astype(F32) for x in (a, b, c, dx, dy))
    P32 = F32(-0.5) * (a32 * dx32 * dx32 + c32 * dy32 * dy32) - b32 * dx32 * dy32
    G32 = _ulp_noise(np.exp2(P32 * LOG2E32).astype(F32), rng)
    o32 = _ulp_noise(o.astype(F32), rng)
    oG32 = (o32 * G32).astype(F32)
    al32 = np.where(oG32 >= AMAX32, AMAX32, oG32)
    oG64 = o * np.exp(P64)
    al64 = np.where(oG64 >= float(AMAX32), float(AMAX32), oG64)
    T64, T32 = 1.0, F32(1.0)
    taken = []
    for j in range(len(a)):
        s64 = P64[j] < -4.5 or al64[j] < float(AMIN32)
        s32 = P32[j] < F32(-4.5) or al32[j] < AMIN32
        if s64 != s32:
            return None
        if s64:
            continue
        n64 = T64 * (1.0 - al64[j])
        n32 = F32(T32 * F32(F32(1.0) - al32[j]))
        if (n64 < float(TMIN32)) != (n32 < TMIN32):
            return None
        if n64 < float(TMIN32):
            break
        taken.append((j, T64, T32))
        T64, T32 = n64, n32
    if not taken:
        return None
    # adjoint: rebuild T before each splat from the final one
    Tb = T32
    rebuilt = []
    for j, t64, t32 in reversed(taken):
        one_m = F32(F32(1.0) - al32[j])
        Tb = F32(Tb * _ulp_noise(np.array([F32(1.0) / one_m]), rng)[0])
        rebuilt.append((t64, t32, Tb))
    E = sum(1.0 / (1.0 - al64[j]) for j, _, _ in taken)
    return rebuilt, E


def test_rebuilt_transmittance_within_allowance():
    rng = np.random.default_rng(2604)
    worst_fwd = worst_bwd = 0.0
    pixels = 0
    for kind, n, count in (("clamped", 3, 3000), ("cutoff", 60, 1500), ("faint", 400, 600), ("mixed", 120, 1500)):
        for _ in range(count):
            if kind == "mixed":
                parts = [_pixel(rng, n // 3, k) for k in ("clamped", "cutoff", "faint")]
                arr = [np.concatenate(x) for x in zip(*parts)]
                perm = rng.permutation(len(arr[0]))
                args = [x[perm] for x in arr]
            else:
                args = _pixel(rng, n, kind)
            res = _walk(rng, *args)
            if res is None:
                continue
            rebuilt, E = res
            pixels += 1
            for t64, t32, tb in rebuilt:
                worst_fwd = max(worst_fwd, abs(float(t32) - t64) / t64 / (U * E))
                worst_bwd = max(worst_bwd, abs(float(tb) - t64) / t64 / (U * E))
    print(f"pixels {pixels}: worst forward T error {worst_fwd:.2f} u E_p, rebuilt {worst_bwd:.2f} u E_p "
          f"(allowance {EPS_T / U:.0f} u E_p)")
    assert pixels > 5000
    assert worst_bwd <= EPS_T / U and worst_fwd <= EPS_T / U
