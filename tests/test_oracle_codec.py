"""Pins of the delta codecs and client replay (Sec. 3.5: residual coding of
means and scales relative to the last transmitted state, quantized updates of
the other attributes, receiver-side replay, transmission epochs).

The oracle's reading (bit widths, steps, rounding) is pinned against a
packet worked out by hand, the closed-loop property (the receiver's model
equals the sender's baseline bit for bit after every packet), the
quantization error bounds, the raw mode's agreement with the plain delta
rule, and the receiver's rejection of stale or malformed packets."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2604_02851_amd import scenes as S

F32 = np.float32


def _scene(n, deg, rng, scale=1.0):
    return S.draw_scene(rng, n, scale, deg)


def _copy(sc):
    return sc.copy()


def _equal(a, b):
    return all(np.array_equal(x.view(np.uint32), y.view(np.uint32)) for (_, x), (_, y) in zip(a.tensors(), b.tensors()))


RAW = (0, 32, 1.0, 0.0, 0.0)


def test_hand_worked_packet():
    # two Gaussians, degree 0; opacity quantized (8 bits, lo -2, step 1/2),
    # means residual-coded (8 bits, step 1/4); mask = opacity | mean = 0b1001
    rng = np.random.default_rng(1)
    cur = _scene(2, 0, rng)
    base = _copy(cur)
    cur.opacity_logit[:] = F32([0.3, 1.0])
    base.opacity_logit[:] = F32([0.2, -0.6])
    cur.mean[:, 0] = F32([1.3, 0.0, -0.9])
    base.mean[:, 0] = F32([1.0, 0.0, 0.0])
    cur.mean[:, 1] = F32([5.0, 5.1, 4.95])
    base.mean[:, 1] = F32([5.0, 5.0, 5.0])
    codecs = [(2, 8, 0.5, -2.0, 0.0), RAW, RAW, (1, 8, 0.25, 0.0, 0.0), RAW, RAW]
    receiver = _copy(base)
    pk = O.delta_encode(cur, base, codecs, mask=0b1001, epoch=7)
    # opacity: q(0.3) = rint(4.6) = 5 vs q(0.2) = rint(4.4) = 4 -> sent;
    #          q(1.0) = 6 vs q(-0.6) = rint(2.8) = 3 -> sent; one 8-bit code per word
    # mean 0:  residual (0.3, 0, -0.9) / (1/4) = (1.2, 0, -3.6) -> codes (1, 0, -4) -> sent,
    #          packed 0x01 | 0x00 << 8 | 0xFC << 16
    # mean 1:  residual (0, ~0.1, ~-0.05) * 4 rounds to (0, 0, 0) -> not sent
    expect = [7, 0b1001, 2, 0, 0, 1, 0, 0, 15, 0, 1, 5, 6, 0, 0x00FC0001]
    assert pk.tolist() == expect
    assert base.opacity_logit.tolist() == [0.5, 1.0]                  # -2 + 5/2, -2 + 6/2
    assert base.mean[:, 0].tolist() == [1.25, 0.0, -1.0]
    assert base.mean[:, 1].tolist() == [5.0, 5.0, 5.0]
    # a receiver in another epoch rejects it and keeps its model
    stale = _copy(receiver)
    assert O.delta_apply(stale, pk, codecs, epoch=6) == 1
    assert _equal(stale, receiver)
    assert O.delta_apply(receiver, pk, codecs, epoch=7) == 0
    assert _equal(receiver, base)


DEFAULT = [(2, 16, 2.0 ** -12, -8.0, 0.0), (2, 16, 2.0 ** -13, -4.0, 0.0), (2, 8, 2.0 ** -7, -1.0, 0.0),
           (1, 16, 2.0 ** -12, 0.0, 0.0), (1, 16, 2.0 ** -10, 0.0, 0.0), (2, 16, 2.0 ** -14, -2.0, 0.0)]


@pytest.mark.parametrize("codecs", [DEFAULT, [(1, 8, 1e-2, 0.0, 0.0)] * 6, [(2, 8, 0.01, -1.5, 0.0)] * 6,
                                    [RAW[:4] + (1e-3,)] * 6])
def test_closed_loop_receiver_tracks_sender(codecs):
    rng = np.random.default_rng(2)
    cur = _scene(300, 2, rng)
    base = _copy(cur)
    receiver = _copy(cur)
    epoch = 3
    for frame in range(12):
        for _, a in cur.tensors():                     # the model drifts
            a += (0.02 * rng.normal(size=a.shape)).astype(F32)
        mask = 0b000011 if frame % 3 else 0b111111     # a schedule: some groups every frame, all every third
        if frame == 7:                                 # snapshot: baselines := current, epoch + 1
            base, receiver, epoch = _copy(cur), _copy(cur), epoch + 1
            continue
        pk = O.delta_encode(cur, base, codecs, mask=mask, epoch=epoch)
        assert pk[8] == pk.size
        assert O.delta_apply(receiver, pk, codecs, epoch=epoch) == 0
        assert _equal(receiver, base), frame


def test_error_bounds():
    rng = np.random.default_rng(3)
    n = 2000
    cur = _scene(n, 1, rng)
    base = _copy(cur)
    for _, a in cur.tensors():
        a += (0.05 * rng.normal(size=a.shape)).astype(F32)
    codecs = [(2, 16, 2.0 ** -12, -8.0, 0.0), (2, 16, 2.0 ** -13, -4.0, 0.0), (2, 8, 2.0 ** -7, -1.0, 0.0),
              (1, 16, 2.0 ** -12, 0.0, 0.0), (1, 16, 2.0 ** -10, 0.0, 0.0), (2, 16, 2.0 ** -14, -2.0, 0.0)]
    before = [b.copy() for b in O.group_arrays(base)]
    O.delta_encode(cur, base, codecs)
    for g, (c, b, b0) in enumerate(zip(O.group_arrays(cur), O.group_arrays(base), before)):
        mode, bits, step, lo, _ = codecs[g]
        c64, b64 = c.astype(np.float64), b.astype(np.float64)
        sp = lambda x: np.spacing(np.abs(x).astype(F32)).astype(np.float64)
        if mode == 1:
            # residuals within the code range: the reconstruction is within half a step
            # plus the FP32 roundings of the residual and of the addition (the steps
            # are powers of two, so the scalings are exact)
            slack = step / 2 + sp(c64 - b0.astype(np.float64)) + sp(b64)
            assert np.all(np.abs(c64 - b64) <= slack), g
        else:
            hi = lo + ((1 << bits) - 1) * step
            sent = np.any(b != b0, axis=0)
            inside = (c64 >= lo) & (c64 <= hi)
            slack = step / 2 + sp(c64 - lo) + sp(b64)      # roundings of (x - lo) and of lo + k step
            ok = np.abs(c64 - b64) <= slack
            assert np.all(ok[:, sent] | ~inside[:, sent]), g
            # every reconstructed value sits on the grid lo + k step
            k = (b64[:, sent] - lo) / step
            assert np.allclose(k, np.rint(k), atol=1e-3), g


def test_clamped_residual_converges():
    rng = np.random.default_rng(4)
    cur = _scene(5, 0, rng)
    base = _copy(cur)
    cur.mean[0, :] += F32(10.0)                            # far beyond one 8-bit packet (127 steps of 1/64)
    codecs = [RAW, RAW, RAW, (1, 8, 1.0 / 64, 0.0, 0.0), RAW, RAW]
    moves = []
    for _ in range(8):
        prev = base.mean[0].copy()
        pk = O.delta_encode(cur, base, codecs, mask=1 << 3)
        moves.append((base.mean[0] - prev).astype(np.float64))
        if pk[5] == 0:
            break
    assert np.allclose(moves[0], 127 / 64)                 # the clamp moves by the largest code
    assert np.all(np.abs(cur.mean[0].astype(np.float64) - base.mean[0]) <= 1 / 128 + 1e-5)


def test_raw_mode_matches_plain_delta_rule():
    rng = np.random.default_rng(5)
    cur = _scene(500, 3, rng)
    b1, b2 = _copy(cur), _copy(cur)
    for _, a in cur.tensors():
        a += (rng.random(a.shape) < 0.1) * F32(0.5)
    tau = 1e-3
    plain = O.delta(cur, b1, 0x3F, tau)
    coded = O.delta_encode(cur, b2, [(0, 32, 1.0, 0.0, tau)] * 6, 0x3F, epoch=0)
    assert np.array_equal(plain[:6], coded[2:8])
    assert np.array_equal(plain[6:], coded[9:])
    assert _equal(b1, b2)


def test_malformed_packets_are_rejected_whole():
    rng = np.random.default_rng(6)
    cur = _scene(50, 1, rng)
    base = _copy(cur)
    for _, a in cur.tensors():
        a += F32(0.3)
    pk = O.delta_encode(cur, base, DEFAULT, 0x3F, epoch=1)
    ref = _copy(base)
    cases = {}
    cases["short"] = pk[:8]
    t = pk.copy(); t[1] |= 1 << 6; cases["mask bits"] = t
    t = pk.copy(); t[9] = 50; cases["index out of range"] = t
    t = pk.copy(); t[10] = t[9]; cases["not ascending"] = t
    t = pk.copy(); t[8] += 1; cases["total"] = t
    cases["truncated"] = pk[:-1]
    t = O.delta_encode(cur, _copy(ref), DEFAULT, 0b1, epoch=1)
    t[3] = 1; cases["rows in unmasked group"] = t
    for name, bad in cases.items():
        model = _copy(ref)
        model_before = _copy(model)
        st = O.delta_apply(model, bad, DEFAULT, epoch=1)
        assert st & 2, name
        assert _equal(model, model_before), name
