"""GPU parity of the HIP path against the FP64 oracle, stage by stage and end
to end, through the C ABI.  Bars: tile lists, depth keys, rectangles and
delta buffers bit-exact; images within 1e-5 per channel (or one outcome of a
near-threshold decision); gradients within 1e-4 relative + 1e-6 absolute,
widened by the FP32 accumulation allowance and the oracle's decision slack."""
import numpy as np
import pytest
import torch

from gpu_util import (IMG_TOL, adam_check, compare_images, flat_grads, grad_report, renderer_for, seg_np)
from paper_2604_02851_amd import scenes as S
from paper_2604_02851_amd.native import DeviceParams

pytestmark = pytest.mark.gpu
F32 = np.float32


def small(seed=101, n=2000, deg=3, sizes=((100, 75), (64, 64), (37, 53)), dist=3.0, extent=1.0):
    return S.small_workload(seed, n, extent, deg, list(sizes), dist=dist)


def _up(w, seed=0):
    return np.random.default_rng(seed).normal(size=3 * w.n_pixels).astype(F32)


def test_project_keys_rects_and_records(oracle):
    w = small()
    V, N = len(w.cams), w.scene.n
    r = renderer_for(w)
    P = DeviceParams.from_scene(w.scene)
    r.ctx.project(P, r.dev_cams, 0, V, r.ws)
    cnt = seg_np(r, "count", np.uint32).reshape(V, N)
    depth = seg_np(r, "depth", np.uint32).reshape(V, N)
    rect = seg_np(r, "rect", np.uint16).reshape(V, N, 4).astype(np.int64)
    rec = seg_np(r, "record", np.float32).reshape(V, N, 12).astype(np.float64)
    pr = oracle.project(w.scene, w.cams)
    vis = pr.visible
    assert vis.sum() > 1000
    assert np.array_equal(cnt > 0, vis)
    assert np.array_equal(depth[vis], pr.zbits[vis])
    assert np.array_equal(rect[vis], (pr.rect[vis] // 16).astype(np.int64))
    tiles = (rect[..., 2] - rect[..., 0] + 1) * (rect[..., 3] - rect[..., 1] + 1)
    assert np.array_equal(cnt[vis], tiles[vis])
    u = rec[..., 0] + rec[..., 2]
    v_ = rec[..., 1] + rec[..., 3]
    assert np.abs(u - pr.rec[..., 0])[vis].max() < 1e-9 * 2048
    assert np.abs(v_ - pr.rec[..., 1])[vis].max() < 1e-9 * 2048
    a, rr, s = rec[..., 4], rec[..., 5], rec[..., 6]
    qa, qb, qc = a, rr * a, s + rr * rr * a
    for mine, ref in ((qa, pr.rec[..., 5]), (qb, pr.rec[..., 6]), (qc, pr.rec[..., 7])):
        scale = np.maximum(np.abs(pr.rec[..., 5]), np.abs(pr.rec[..., 7]))
        assert (np.abs(mine - ref) / scale)[vis].max() < 1e-6
    assert (np.abs(rec[..., 7] - pr.rec[..., 8]) / pr.rec[..., 8])[vis].max() < 1e-6
    assert np.abs(rec[..., 8:11] - pr.rec[..., 9:12])[vis].max() < 1e-5


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 16), (32, 32)])
def test_tile_lists_bit_exact(oracle, tile):
    w = small(seed=102)
    r = renderer_for(w, tile=tile)
    P = DeviceParams.from_scene(w.scene)
    r.forward(P)
    c = r.counters()
    vals_o, ranges_o = oracle.tile_lists(w.scene, w.cams, tile[0], tile[1])
    assert c.overflow == 0 and c.keys == len(vals_o)
    vals = seg_np(r, "sorted_values", np.uint32)[:c.keys]
    assert np.array_equal(vals, vals_o)
    ranges = seg_np(r, "ranges", np.uint32).reshape(-1, 2)
    assert np.array_equal(ranges, ranges_o)


def test_tile_lists_with_pairs_spanning_sort_chunks_bit_exact(oracle):
    # a few Gaussians as large as the view at 8x8 tiles: one (view, Gaussian)
    # pair then emits more keys than one chunk of the tile sort holds (4096),
    # so its keys straddle several chunks written by different workgroups
    w = small(seed=131, n=1500, sizes=((1280, 720), (200, 120)))
    w.scene.log_scale[:, :8] = 0.0
    r = renderer_for(w, tile=(8, 8), cap=1 << 20)   # about 615k keys
    P = DeviceParams.from_scene(w.scene)
    r.forward(P)
    c = r.counters()
    cnt = seg_np(r, "count", np.uint32)
    assert cnt.max() > 3 * 4096
    vals_o, ranges_o = oracle.tile_lists(w.scene, w.cams, 8, 8)
    assert c.overflow == 0 and c.keys == len(vals_o)
    vals = seg_np(r, "sorted_values", np.uint32)[:c.keys]
    assert np.array_equal(vals, vals_o)
    ranges = seg_np(r, "ranges", np.uint32).reshape(-1, 2)
    assert np.array_equal(ranges, ranges_o)


@pytest.mark.parametrize("sizes", [((192, 160),), ((192, 160), (64, 48))])
def test_tile_lists_with_narrow_first_digit_bit_exact(oracle, sizes):
    # 480 (9 bits) or 528 (10 bits) tiles at 8x8: the tile sort's first pass
    # takes 1 or 2 bits, so the digit counts of the emission see tile rows
    # that wrap the digit range many times, and large Gaussians make pairs
    # of hundreds of keys that straddle sort chunks
    w = small(seed=137, n=1500, sizes=sizes)
    w.scene.log_scale[:, :40] = -0.5
    r = renderer_for(w, tile=(8, 8), cap=1 << 20)
    P = DeviceParams.from_scene(w.scene)
    r.forward(P)
    c = r.counters()
    cnt = seg_np(r, "count", np.uint32)
    assert cnt.max() >= 100 and c.keys > 2 * 4096
    vals_o, ranges_o = oracle.tile_lists(w.scene, w.cams, 8, 8)
    assert c.overflow == 0 and c.keys == len(vals_o)
    vals = seg_np(r, "sorted_values", np.uint32)[:c.keys]
    assert np.array_equal(vals, vals_o)
    ranges = seg_np(r, "ranges", np.uint32).reshape(-1, 2)
    assert np.array_equal(ranges, ranges_o)


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.3, 0.5, 0.1)])
def test_composite_matches_oracle(oracle, bg):
    w = small(seed=103)
    r = renderer_for(w, bg=bg)
    P = DeviceParams.from_scene(w.scene)
    img, T, nc = r.forward(P)
    torch.cuda.synchronize()
    ref = oracle.render(w.scene, w.cams, bg=bg)
    worst, via_alt = compare_images(oracle, w, img.cpu().numpy(), bg, ref=ref)
    print(f"max clean-pixel error {worst:.3g}, pixels matched through an alternative outcome {via_alt}")
    clean = ref.flags == 0
    assert np.abs(T.cpu().numpy() - ref.T)[clean].max() <= IMG_TOL
    assert np.array_equal(nc.cpu().numpy()[clean], ref.n_contrib[clean])
    assert ref.n_contrib.max() > 20


# (tile, pixels per thread, wave sub-tile width); every built variant
VARIANTS = [((8, 8), 1, 8), ((16, 8), 1, 16), ((16, 8), 2, 16), ((16, 16), 1, 16), ((16, 16), 2, 16),
            ((16, 16), 4, 16), ((32, 16), 1, 32), ((32, 16), 2, 32), ((32, 16), 4, 32), ((32, 16), 2, 16),
            ((32, 16), 4, 16), ((32, 32), 1, 32), ((32, 32), 2, 32), ((32, 32), 4, 32), ((32, 32), 2, 16),
            ((32, 32), 4, 16)]


def test_tile_batch_and_thread_shape_invariance_bit_identical():
    w = small(seed=104)
    P = DeviceParams.from_scene(w.scene)
    base = None
    for tile, ppt, sw in VARIANTS:
        for batch, schedule in [(32, 0), (64, 1), (128, 2), (64, 3)]:
            r = renderer_for(w, tile=tile, batch=batch, ppt=ppt, wave_w=sw, schedule=schedule)
            img, T, nc = r.forward(P)
            cur = (img.cpu().numpy(), T.cpu().numpy(), nc.cpu().numpy())
            if base is None:
                base = cur
            else:
                for a, b in zip(base, cur):
                    assert np.array_equal(a, b), (tile, batch, ppt, sw, schedule)


def test_unbuilt_launch_shape_is_refused():
    from paper_2604_02851_amd.native import GsError
    w = small(seed=104)
    for kw in (dict(tile=(32, 32), ppt=8), dict(tile=(16, 16), ppt=4, wave_w=8), dict(tile=(16, 16), schedule=4)):
        with pytest.raises(GsError):
            renderer_for(w, **kw)


@pytest.mark.parametrize("tile,ppt,sw,schedule", [((16, 16), 4, 16, 0), ((32, 32), 2, 32, 1), ((32, 16), 4, 32, 0),
                                                   ((16, 8), 2, 16, 1), ((32, 32), 4, 16, 0), ((32, 16), 2, 16, 1),
                                                   ((32, 32), 4, 16, 2), ((16, 16), 2, 16, 3), ((8, 8), 1, 8, 3)])
def test_backward_variants_match_oracle(oracle, tile, ppt, sw, schedule):
    w = small(seed=110, n=1200, sizes=((70, 50), (33, 64)))
    r = renderer_for(w, tile=tile, ppt=ppt, wave_w=sw, schedule=schedule)
    P = DeviceParams.from_scene(w.scene)
    G = _up(w, 3)
    r.forward(P)
    grads = DeviceParams.zeros_like(P)
    r.backward(P, torch.from_numpy(G).cuda(), 0, grads)
    torch.cuda.synchronize()
    b = oracle.backward(w.scene, w.cams, G, mode=0)
    rep = grad_report(flat_grads(grads), b)
    print(tile, ppt, sw, schedule, rep)
    assert rep["fail"] == 0


def test_backward_matches_oracle_gradient(oracle):
    w = small(seed=105, n=1500, sizes=((80, 60), (48, 64)))
    r = renderer_for(w)
    P = DeviceParams.from_scene(w.scene)
    G = _up(w, 1)
    r.forward(P)
    grads = DeviceParams.zeros_like(P)
    r.backward(P, torch.from_numpy(G).cuda(), 0, grads)
    torch.cuda.synchronize()
    b = oracle.backward(w.scene, w.cams, G, mode=0)
    rep = grad_report(flat_grads(grads), b)
    print(rep)
    assert rep["fail"] == 0
    assert rep["max_rel_err_large"] < 1e-3


def test_l1_backward_and_loss_match_oracle(oracle):
    w = small(seed=106, n=1500, sizes=((72, 72), (50, 30)))
    tgt = np.concatenate([t.reshape(-1) for t in w.extra["target"]]).astype(F32)
    for loss_mode in (0, 1):
        r = renderer_for(w, loss_mode=loss_mode)
        P = DeviceParams.from_scene(w.scene)
        r.forward(P)
        grads = DeviceParams.zeros_like(P)
        loss = torch.zeros(1, device="cuda")
        r.backward(P, torch.from_numpy(tgt).cuda(), 1, grads, loss=loss)
        torch.cuda.synchronize()
        b = oracle.backward(w.scene, w.cams, tgt, mode=1, loss_mode=loss_mode)
        rep = grad_report(flat_grads(grads), b)
        print(loss_mode, rep)
        assert rep["fail"] == 0
        assert abs(loss.item() - b.loss) <= 1e-5 * b.loss


@pytest.mark.parametrize("schedule", [0, 3])
def test_batched_equals_plain(oracle, schedule):
    """One launch per stage for all views against one view per launch (for
    the persistent schedules: a work queue drained and reset per launch)."""
    w = small(seed=107, n=1500)
    P = DeviceParams.from_scene(w.scene)
    G = torch.from_numpy(_up(w, 2)).cuda()
    r = renderer_for(w, schedule=schedule)
    img_b = r.forward(P)[0].clone()
    g_b = DeviceParams.zeros_like(P)
    r.backward(P, G, 0, g_b)
    g_p = DeviceParams.zeros_like(P)
    img_p = torch.zeros_like(img_b)
    for v in range(r.n_views):
        r.forward(P, v, 1)
        r.backward(P, G, 0, g_p, v, 1, accumulate=1 if v else 0)
        img_p += 0  # images of view v land at their own offsets
    img_p = r.images.clone()
    torch.cuda.synchronize()
    assert torch.equal(img_b, img_p)
    b = oracle.backward(w.scene, w.cams, G.cpu().numpy(), mode=0)
    for g in (g_b, g_p):
        assert grad_report(flat_grads(g), b)["fail"] == 0


def test_config1_forward_backward(oracle):
    w = S.workload(1)
    tgt = w.extra["target"].reshape(-1)
    r = renderer_for(w)
    P = DeviceParams.from_scene(w.scene)
    img = r.forward(P)[0]
    grads = DeviceParams.zeros_like(P)
    loss = torch.zeros(1, device="cuda")
    r.backward(P, torch.from_numpy(tgt).cuda(), 1, grads, loss=loss)
    torch.cuda.synchronize()
    compare_images(oracle, w, img.cpu().numpy())
    b = oracle.backward(w.scene, w.cams, tgt, mode=1)
    rep = grad_report(flat_grads(grads), b)
    print(rep)
    assert rep["fail"] == 0


def test_empty_and_non_finite(oracle):
    w = small(seed=108, n=500, sizes=((40, 30),))
    sc = w.scene.copy()
    sc.mean[2, :] = 50.0          # everything behind or far: nothing visible from some cameras
    sc.mean[:, :] = np.asarray(w.cams[0]["campos"], F32)[:, None]   # at the camera centre: culled by near
    r = renderer_for(S.Workload("e", sc, w.cams), bg=(0.2, 0.4, 0.6))
    P = DeviceParams.from_scene(sc)
    img, T, nc = r.forward(P)
    torch.cuda.synchronize()
    assert r.counters().visible == 0 and r.counters().keys == 0
    assert np.allclose(img.view(3, -1).cpu().numpy(), np.array([0.2, 0.4, 0.6], F32)[:, None])
    assert torch.all(T == 1) and torch.all(nc == 0)
    # non-finite parameters are culled and do not poison other pixels
    sc2 = w.scene.copy()
    sc2.mean[0, :50] = np.nan
    sc2.log_scale[1, 50:60] = np.inf
    sc2.sh[5, 60:70] = np.nan
    r2 = renderer_for(S.Workload("nf", sc2, w.cams))
    P2 = DeviceParams.from_scene(sc2)
    img2 = r2.forward(P2)[0]
    G = torch.ones_like(img2)
    grads = DeviceParams.zeros_like(P2)
    r2.backward(P2, G, 0, grads)
    torch.cuda.synchronize()
    assert torch.isfinite(img2).all()
    assert all(torch.isfinite(t).all() for t in grads.tensors())
    compare_images(oracle, S.Workload("nf", sc2, w.cams), img2.cpu().numpy())


def test_key_capacity_overflow_is_reported_and_recoverable(oracle):
    from paper_2604_02851_amd.native import GS_ERR_CAPACITY, GsError
    w = small(seed=109, n=1000)
    P = DeviceParams.from_scene(w.scene)
    r = renderer_for(w, cap=64)
    r.forward(P)
    c = r.counters()
    assert c.overflow == 1 and c.overflow_any == 1 and c.keys > 64 and c.key_capacity == 64
    # the read marks the context: rendering is refused until a new plan
    with pytest.raises(GsError) as e:
        r.forward(P)
    assert e.value.status == GS_ERR_CAPACITY
    r.replan(c.keys)
    img = r.forward(P)[0]
    c = r.counters()
    assert c.overflow == 0 and c.overflow_any == 0
    compare_images(oracle, w, img.cpu().numpy())


def test_capacity_error_is_sticky_across_graph_replays():
    """An overflow in one replayed step is still reported after later steps
    that fit, and from then on replays fail with GS_ERR_CAPACITY until the
    renderer is re-planned and the step captured again."""
    from paper_2604_02851_amd.native import GS_ERR_CAPACITY, GsError
    from paper_2604_02851_amd.renderer import Optimizer
    w = small(seed=110, n=2000)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        P = DeviceParams.from_scene(w.scene)
        r = renderer_for(w, loss_mode=1)
        r.fit_capacity(P)
        tgt = r.forward(DeviceParams.from_scene(w.extra["perturbed"]))[0].clone()
        opt = Optimizer(r, P, tgt, stream=s)
        opt.capture()
        opt.replay()
        assert opt.check_capacity().overflow_any == 0
        fit = r.key_capacity
        P.log_scale.add_(1.5)        # in place: the captured graph stays valid, the splats grow
        opt.replay()                 # overflows (keys beyond the capacity are dropped)
        P.log_scale.sub_(1.5)
        opt.replay()                 # fits again
        s.synchronize()
        c = r.counters()
        assert c.overflow == 0 and c.overflow_any == 1 and c.keys <= fit
        for call in (opt.replay, opt.step, lambda: r.forward(P)):
            with pytest.raises(GsError) as e:
                call()
            assert e.value.status == GS_ERR_CAPACITY
        big = DeviceParams(*[t.clone() for t in P.tensors()], P.sh_degree)
        big.log_scale.add_(1.5)
        r.fit_capacity(big)          # re-plans for the larger need
        assert r.key_capacity > fit
        opt.invalidate()
        opt.capture()
        opt.replay()
        assert opt.check_capacity().overflow_any == 0


def test_adam_matches_oracle(oracle):
    rng = np.random.default_rng(5)
    sc = S.draw_scene(rng, 3001, 2.0, 3)
    P = DeviceParams.from_scene(sc)
    mk = lambda scale: DeviceParams(*[torch.from_numpy((rng.normal(size=t.shape) * scale).astype(F32)).cuda()
                                      for t in P.tensors()], 3)
    g = mk(1.0)
    m = mk(0.1)
    v = DeviceParams(*[torch.from_numpy(np.abs(rng.normal(size=t.shape)).astype(F32)).cuda()
                       for t in P.tensors()], 3)
    theta0 = [t.cpu().numpy().copy() for t in P.tensors()]
    m0 = [t.cpu().numpy().copy() for t in m.tensors()]
    v0 = [t.cpu().numpy().copy() for t in v.tensors()]
    g0 = [t.cpu().numpy().copy() for t in g.tensors()]
    step = torch.tensor([4], dtype=torch.int32, device="cuda")
    lr = (1e-3, 5e-3, 1e-3, 5e-2, 5e-3, 2.5e-3)
    from paper_2604_02851_amd.native import Context
    ctx = Context(0)
    ctx.adam_step(P, g, m, v, step, lr, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    assert step.item() == 5
    out_t, out_m, out_v = ([t.cpu().numpy() for t in d.tensors()] for d in (P, m, v))
    groups = [(0, slice(None), lr[0]), (1, slice(None), lr[1]), (2, slice(None), lr[2]), (3, slice(None), lr[3]),
              (4, slice(0, 3), lr[4]), (4, slice(3, None), lr[5])]
    for ti, sl, l in groups:
        adam_check(oracle, theta0[ti][sl], g0[ti][sl], m0[ti][sl], v0[ti][sl], out_t[ti][sl], out_m[ti][sl],
                   out_v[ti][sl], l, 0.9, 0.999, 1e-8, 5)


def test_delta_bit_exact(oracle):
    rng = np.random.default_rng(6)
    base = S.draw_scene(rng, 5003, 5.0, 3)
    cur = base.copy()
    for name, a in cur.tensors():
        a2 = a.reshape(-1, cur.n)
        mask = rng.uniform(size=a2.shape) < 0.05
        a2[mask] *= F32(1) + rng.uniform(-3e-3, 3e-3, size=mask.sum()).astype(F32)
    cur.opacity_logit[:3] = 0.0
    base.opacity_logit[:3] = 0.0
    cur.opacity_logit[3] = 1e-30
    base.opacity_logit[3] = 0.0
    from paper_2604_02851_amd import native as N
    w = S.Workload("d", cur, S.cams_array([S.look_at((0, 0, 10), 16, 16)]))
    r = renderer_for(w)
    Pc, Pb = DeviceParams.from_scene(cur), DeviceParams.from_scene(base)
    for mask in (0x3F, 0b000011, 0b111000):
        b_or = base.copy()
        Pb = DeviceParams.from_scene(base)
        out = torch.zeros(N.delta_capacity_words(cur.n, 3, mask), dtype=torch.int32, device="cuda")
        r.ctx.delta_extract(Pc, Pb, mask, 1e-3, out, r.ws)
        torch.cuda.synchronize()
        ref = oracle.delta(cur, b_or, mask=mask, tau=1e-3)
        got = out.cpu().numpy().view(np.uint32)[:len(ref)]
        assert np.array_equal(got, ref), mask
        for (_, a), (_, b) in zip(Pb.to_scene().tensors(), b_or.tensors()):
            assert np.array_equal(a, b)
        # idempotent: a second extraction is empty
        out.zero_()
        r.ctx.delta_extract(Pc, Pb, mask, 1e-3, out, r.ws)
        torch.cuda.synchronize()
        assert not out[:6].any()
    # snapshot reset: baseline := current, epoch + 1
    Pb = DeviceParams.from_scene(base)
    epoch = torch.zeros(1, dtype=torch.int32, device="cuda")
    r.ctx.delta_reset_baseline(Pc, Pb, epoch)
    torch.cuda.synchronize()
    assert epoch.item() == 1
    for a, b in zip(Pb.tensors(), Pc.tensors()):
        assert torch.equal(a, b)
