"""Parity at the configured sizes, through the C ABI in the benchmark's launch
configuration: cfg2 in full (autograd Function, oracle gradient and FP64
finite differences), cfg3 / cfg4 / cfg5 on sampled rows of every view, a full
gradient check on two views of cfg3, cfg4 tile lists of three 640x360 views
and of a 1920x1080 view bit-exact inside the 16-view batched call, the
16-view batched cfg4 backward against the oracle's gradient of the views it
is given gradients on (three 640x360 views; a 1920x1080 and a 1280x720
view), the four-view cfg5 backward against the oracle on one 1080p view,
Adam over the whole cfg4 model on every element, cfg5 delta extraction
bit-exact at 3M Gaussians after scene dynamics and a GPU step, and graph
replay against eager steps."""
import numpy as np
import pytest
import torch

from gpu_util import EPS_ACC, EPS_T, adam_check, compare_images, flat_grads, grad_report, seg_np
from paper_2604_02851_amd import scenes as S
from paper_2604_02851_amd.native import DeviceParams
from paper_2604_02851_amd.renderer import GaussianRasterize, Optimizer, Renderer

pytestmark = pytest.mark.gpu
F32 = np.float32
BENCH_SHAPE = dict(tile=(32, 32), batch_depth=128, pixels_per_thread=4, wave_w=16, schedule=0)


def _renderer(w, loss_mode=0, **kw):
    opts = dict(BENCH_SHAPE)
    opts.update(kw)
    r = Renderer(w.cams, w.scene.n, w.scene.sh_degree, loss_mode=loss_mode, **opts)
    return r


def _rows_check(oracle, w, img, rows_per_view=8, bg=(0.0, 0.0, 0.0)):
    """Compares rows sampled from the middle and the edges of every view."""
    off = oracle.pixel_offsets(w.cams)
    checked = 0
    for v, cam in enumerate(w.cams):
        H, W = int(cam["height"]), int(cam["width"])
        for r0 in (0, H // 2 - rows_per_view // 2, H - rows_per_view):
            sub = w.cams[v:v + 1].copy()
            ref = oracle.render(w.scene, sub, bg=bg, rows=(r0, r0 + rows_per_view))
            mine = img[3 * off[v]:3 * off[v + 1]].reshape(3, H, W)[:, r0:r0 + rows_per_view].astype(np.float64)
            theirs = ref.image.reshape(3, H, W)[:, r0:r0 + rows_per_view]
            fl = ref.flags.reshape(H, W)[r0:r0 + rows_per_view] > 0
            d = np.abs(mine - theirs).max(0)
            assert d[~fl].max() <= 1e-5, (v, r0, d[~fl].max())
            if (d[fl] > 1e-5).any():
                ys, xs = np.nonzero((d > 1e-5) & fl)
                alts = oracle.render_alternatives(w.scene, sub, 0, np.stack([xs, ys + r0], 1), bg=bg)
                for q in range(len(xs)):
                    best = np.abs(alts[q][:, :3] - mine[:, ys[q], xs[q]][None, :]).max(1).min()
                    assert best <= 1e-5
            checked += W * rows_per_view
    return checked


def test_config2_full_autograd_oracle_and_fd(oracle):
    w = S.workload(2)
    pert = w.extra["perturbed"]
    tgt = oracle.render(pert, w.cams).image.astype(F32)          # target: oracle render of the perturbed copy
    r = _renderer(w)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda().requires_grad_(True) for _, a in w.scene.tensors()]
    img = GaussianRasterize.apply(*dev, r)
    loss = (img - torch.from_numpy(tgt).cuda()).abs().sum()
    loss.backward()
    torch.cuda.synchronize()
    # image: every pixel
    compare_images(oracle, w, img.detach().cpu().numpy())
    # gradient: oracle analytic gradient of the same sum-L1 loss
    b = oracle.backward(w.scene, w.cams, tgt, mode=1, loss_mode=0)
    g = np.concatenate([t.grad.cpu().numpy().reshape(-1, w.scene.n) for t in dev], 0).astype(np.float64)
    rep = grad_report(g, b)
    print("cfg2 gradient", rep)
    assert rep["fail"] == 0
    assert abs(loss.item() - b.loss) <= 1e-5 * b.loss
    # FP64 central differences of the oracle on 64 parameters, stratified
    # over the groups, among Gaussians composited into at least one pixel
    pr = oracle.project(w.scene, w.cams)
    ref = oracle.render(w.scene, w.cams)
    rng = w.extra["rng_fd"]
    vis = np.nonzero(pr.visible[0])[0]
    groups = [("mean", 0, 3), ("log_scale", 3, 3), ("quat", 6, 4), ("opacity_logit", 10, 1), ("sh", 11, 48)]
    picks = []
    for name, row0, rows in groups:
        for _ in range(13 if name != "opacity_logit" else 12):
            picks.append((name, row0, int(rng.integers(rows)), int(rng.choice(vis))))
    H = int(w.cams[0]["height"])
    ok = 0
    for name, row0, row, i in picks:
        y0, y1 = int(pr.rect[0, i, 1]) - 3, int(pr.rect[0, i, 3]) + 4
        y0, y1 = max(0, y0), min(H, y1)
        base_band = oracle.render(w.scene, w.cams, rows=(y0, y1))
        x0 = float(getattr(w.scene, name).reshape(-1, w.scene.n)[row, i])
        est = []
        for hrel in (1e-3, 5e-4):
            h = hrel * max(1.0, abs(x0))
            vals, steps, same = [], [], True
            for sgn in (1, -1):
                sc = w.scene.copy()
                t = getattr(sc, name).reshape(-1, sc.n)
                t[row, i] = F32(x0 + sgn * h)
                rb = oracle.render(sc, w.cams, rows=(y0, y1))
                same &= np.array_equal(rb.n_contrib, base_band.n_contrib)
                band = rb.image.reshape(3, H, -1)[:, y0:y1]
                vals.append(float(np.abs(band - tgt.reshape(3, H, -1)[:, y0:y1]).sum()))
                steps.append(float(t[row, i]))
            if not same:
                break
            est.append((vals[0] - vals[1]) / (steps[0] - steps[1]))
        if len(est) < 2 or abs(est[0] - est[1]) > 1e-3 * max(abs(est[1]), 1e-2):
            continue          # a discrete decision or an L1 kink lies within the step
        gpu = g[row0 + row, i]
        tol = 1e-4 * max(abs(est[1]), abs(gpu)) + 1e-6 + EPS_ACC * b.scale[row0 + row, i] + \
            EPS_T * b.scale_t[row0 + row, i] + b.slack[row0 + row, i] + abs(est[0] - est[1])
        assert abs(gpu - est[1]) <= tol, (name, row, i, gpu, est)
        ok += 1
    print("cfg2 FD samples checked:", ok, "of", len(picks))
    assert ok >= 40


def test_config3_sampled_rows_and_two_view_gradient(oracle):
    w = S.workload(3)
    r = _renderer(w)
    r.fit_capacity(DeviceParams.from_scene(w.scene))
    P = DeviceParams.from_scene(w.scene)
    img = r.forward(P)[0]
    torch.cuda.synchronize()
    n = _rows_check(oracle, w, img.cpu().numpy())
    print("cfg3 pixels checked", n)
    # gradient of views 0-1 (the same kernels, a two-view call) against the oracle
    G = np.random.default_rng(3).normal(size=3 * w.n_pixels).astype(F32)
    r.forward(P, 0, 2)
    grads = DeviceParams.zeros_like(P)
    r.backward(P, torch.from_numpy(G).cuda(), 0, grads, 0, 2)
    torch.cuda.synchronize()
    off = oracle.pixel_offsets(w.cams)
    b = oracle.backward(w.scene, w.cams[0:2], G[:3 * off[2]], mode=0)
    rep = grad_report(flat_grads(grads), b)
    print("cfg3 two-view gradient", rep)
    assert rep["fail"] == 0


def test_config4_sampled_rows(oracle):
    w = S.workload(4)
    P = DeviceParams.from_scene(w.scene)
    r = _renderer(w, loss_mode=1)
    r.fit_capacity(P)
    img = r.forward(P)[0]
    torch.cuda.synchronize()
    n = _rows_check(oracle, w, img.cpu().numpy(), rows_per_view=4)
    print("cfg4 pixels checked", n)


def test_config5_sampled_rows(oracle):
    """The 3M-Gaussian model over four 1920x1080 views (the densest overlap
    of the workloads) in the benchmark's launch shape: rows from the top,
    middle and bottom of every view against the oracle."""
    w = S.workload(5)
    P = DeviceParams.from_scene(w.scene)
    r = _renderer(w)
    r.fit_capacity(P)
    img = r.forward(P)[0]
    torch.cuda.synchronize()
    assert r.counters().overflow == 0
    n = _rows_check(oracle, w, img.cpu().numpy(), rows_per_view=4)
    print("cfg5 pixels checked", n)


def test_config4_tile_lists_three_views(oracle):
    """Tile lists of the 16-view batched cfg4 call (60M keys, 32x32 tiles)
    bit-exact for views 3-5: they are the contiguous run of the global tile
    range that belongs to those views, so they equal the oracle's lists of
    the three views alone, with view indices shifted by 3 and list positions
    by the start of the run."""
    w = S.workload(4)
    P = DeviceParams.from_scene(w.scene)
    r = _renderer(w)
    r.fit_capacity(P)
    r.forward(P)
    c = r.counters()
    assert c.overflow == 0 and c.keys > 50_000_000
    tw, th = BENCH_SHAPE["tile"]
    vals_o, ranges_o = oracle.tile_lists(w.scene, w.cams[3:6], tw, th)
    base = oracle.tile_layout(w.cams, tw, th)
    t0, t1 = int(base[3]), int(base[6])
    ranges = seg_np(r, "ranges", np.uint32).reshape(-1, 2)[t0:t1].astype(np.int64)
    assert ranges.shape == ranges_o.shape
    empty_o = ranges_o[:, 0] == ranges_o[:, 1]
    assert np.array_equal(ranges[:, 0] == ranges[:, 1], empty_o)
    assert (~empty_o).any()
    off = int(ranges[~empty_o, 0].min())
    assert np.array_equal(ranges[~empty_o] - off, ranges_o[~empty_o].astype(np.int64))
    vals = seg_np(r, "sorted_values", np.uint32)[off:off + len(vals_o)]
    n = w.scene.n
    assert np.array_equal(vals, vals_o + np.uint32(3 * n))
    print("cfg4 tile lists of views 3-5:", len(vals_o), "keys of", c.keys)
    # the closest 1920x1080 view (11) inside the same call
    vals_o, ranges_o = oracle.tile_lists(w.scene, w.cams[11:12], tw, th)
    t0, t1 = int(base[11]), int(base[12])
    ranges = seg_np(r, "ranges", np.uint32).reshape(-1, 2)[t0:t1].astype(np.int64)
    empty_o = ranges_o[:, 0] == ranges_o[:, 1]
    assert np.array_equal(ranges[:, 0] == ranges[:, 1], empty_o)
    off = int(ranges[~empty_o, 0].min())
    assert np.array_equal(ranges[~empty_o] - off, ranges_o[~empty_o].astype(np.int64))
    vals = seg_np(r, "sorted_values", np.uint32)[off:off + len(vals_o)]
    assert np.array_equal(vals, vals_o + np.uint32(11 * n))
    print("cfg4 tile lists of view 11 (1080p):", len(vals_o), "keys of", c.keys)


def _batched_gradient_check(oracle, w, views, seed, label):
    """The batched backward over every view of `w` (the call the benchmark
    step makes), with an upstream gradient that is zero outside `views`:
    every other view then adds exact zeros, so the whole gradient must equal
    the oracle's gradient over those views alone."""
    P = DeviceParams.from_scene(w.scene)
    r = _renderer(w)
    r.fit_capacity(P)
    off = oracle.pixel_offsets(w.cams)
    G = np.zeros(3 * w.n_pixels, F32)
    rng = np.random.default_rng(seed)
    for v in views:
        lo, hi = 3 * int(off[v]), 3 * int(off[v + 1])
        G[lo:hi] = rng.normal(size=hi - lo).astype(F32)
    r.forward(P)
    grads = DeviceParams.zeros_like(P)
    r.backward(P, torch.from_numpy(G).cuda(), 0, grads)
    torch.cuda.synchronize()
    assert r.counters().overflow_any == 0
    sub = np.ascontiguousarray(w.cams[list(views)])
    Gs = np.concatenate([G[3 * int(off[v]):3 * int(off[v + 1])] for v in views])
    b = oracle.backward(w.scene, sub, Gs, mode=0)
    rep = grad_report(flat_grads(grads), b)
    print(label, rep)
    assert rep["fail"] == 0
    return rep


def test_config4_batched_gradient_three_views(oracle):
    """Views 3-5 (640x360 each) of the 16-view batched cfg4 backward."""
    w = S.workload(4)
    assert list(w.cams["width"][3:6]) == [640] * 3 and list(w.cams["height"][3:6]) == [360] * 3
    _batched_gradient_check(oracle, w, (3, 4, 5), 44, "cfg4 batched gradient (views 3-5 nonzero)")


def test_config4_batched_gradient_1080p_and_720p(oracle):
    """The closest 1920x1080 view (11, radius 6.9) and the closest 1280x720
    view (7, radius 6.5) of the 16-view batched cfg4 backward: the largest
    splats of the workload and the deepest lists."""
    w = S.workload(4)
    assert (int(w.cams["width"][11]), int(w.cams["height"][11])) == (1920, 1080)
    assert (int(w.cams["width"][7]), int(w.cams["height"][7])) == (1280, 720)
    _batched_gradient_check(oracle, w, (7, 11), 45, "cfg4 batched gradient (views 7 and 11 nonzero)")


def test_config5_batched_gradient_1080p(oracle):
    """The 3M-Gaussian four-view 1080p call with the upstream gradient on its
    closest view (2, radius 6.3): the densest overlap of the workloads."""
    w = S.workload(5)
    assert all(int(c["width"]) == 1920 and int(c["height"]) == 1080 for c in w.cams)
    _batched_gradient_check(oracle, w, (2,), 46, "cfg5 batched gradient (view 2 nonzero)")


def test_config4_adam_every_element(oracle):
    """Adam over the whole 1M-Gaussian SH-degree-3 model (59M scalars, the
    launch of the benchmark step) at its first step, where the bias
    corrections are largest, against the oracle on every element of the
    parameters and both moments, within the bounds derived from the FP32
    update (at step 1, 1 - beta2 turns the FP32 rounding of 0.999 into a
    relative change of 1.3e-5, so both sides take the same FP32 values)."""
    from paper_2604_02851_amd.native import Context
    w = S.workload(4)
    assert w.scene.n == 1_000_000 and w.scene.sh_degree == 3
    rng = np.random.default_rng(46)
    P = DeviceParams.from_scene(w.scene)
    mk = lambda f: DeviceParams(*[torch.from_numpy(f(t.shape)).cuda() for t in P.tensors()], 3)
    g = mk(lambda sh: rng.normal(size=sh).astype(F32))
    m = mk(lambda sh: (0.1 * rng.normal(size=sh)).astype(F32))
    v = mk(lambda sh: np.abs(rng.normal(size=sh)).astype(F32))
    host = lambda d: [t.cpu().numpy().copy() for t in d.tensors()]
    theta0, g0, m0, v0 = host(P), host(g), host(m), host(v)
    step = torch.tensor([0], dtype=torch.int32, device="cuda")
    lr = (1e-3, 5e-3, 1e-3, 5e-2, 5e-3, 2.5e-3)
    Context(0).adam_step(P, g, m, v, step, lr, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    assert step.item() == 1
    out_t, out_m, out_v = host(P), host(m), host(v)
    groups = [(0, slice(None), lr[0]), (1, slice(None), lr[1]), (2, slice(None), lr[2]), (3, slice(None), lr[3]),
              (4, slice(0, 3), lr[4]), (4, slice(3, None), lr[5])]
    worst = 0.0
    for ti, sl, l in groups:
        worst = max(worst, adam_check(oracle, theta0[ti][sl], g0[ti][sl], m0[ti][sl], v0[ti][sl], out_t[ti][sl],
                                      out_m[ti][sl], out_v[ti][sl], l, 0.9, 0.999, 1e-8, 1))
    print("cfg4 Adam: worst error / bound", worst)


def test_config5_delta_after_dynamics_and_step(oracle):
    from paper_2604_02851_amd import native as N
    w = S.workload(5)
    pert = w.extra["perturbed"]
    dyn = S.Dynamics(w.extra["rng_dyn"], w.scene)
    P = DeviceParams.from_scene(w.scene)
    r = _renderer(w, loss_mode=1)
    r.fit_capacity(P)
    tgt = r.forward(DeviceParams.from_scene(pert))[0].clone()
    base = P.clone()                                   # last transmitted state
    opt = Optimizer(r, P, tgt)
    opt.enable_delta(base, 0x3F, 1e-3)
    # one step on the initial scene (baseline == current before it)
    host = w.scene.copy()
    dyn.step([host, pert])                             # the engine moves objects and relights
    for dst, (_, src) in zip(P.tensors(), host.tensors()):
        dst.copy_(torch.from_numpy(src))
    before_base = base.to_scene()
    opt.step()
    torch.cuda.synchronize()
    assert r.counters().overflow == 0
    cur = P.to_scene()
    ref = oracle.delta(cur, before_base, mask=0x3F, tau=1e-3)
    got = opt.delta["out"].cpu().numpy().view(np.uint32)[:len(ref)]
    print("cfg5 delta rows per group", ref[:6].tolist())
    assert np.array_equal(got, ref)
    for a, b2 in zip(base.to_scene().tensors(), before_base.tensors()):
        assert np.array_equal(a[1], b2[1])


@pytest.mark.parametrize("schedule", [0, 3])
def test_graph_replay_matches_eager(oracle, schedule):
    """Graph replays of the batched step against eager steps (schedule 3: the
    persistent compositing kernels, whose work queue must be empty again at
    the end of every replayed launch)."""
    w = S.small_workload(301, 3000, 1.0, 3, [(96, 64), (64, 96), (50, 50)], dist=3.0)
    pert = w.extra["perturbed"]
    shape = dict(BENCH_SHAPE, schedule=schedule)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        r1 = Renderer(w.cams, w.scene.n, 3, loss_mode=1, **shape)
        tgt = r1.forward(DeviceParams.from_scene(pert))[0].clone()
        Pe = DeviceParams.from_scene(w.scene)
        Pg = DeviceParams.from_scene(w.scene)
        r1.fit_capacity(Pe)
        r2 = Renderer(w.cams, w.scene.n, 3, loss_mode=1, key_capacity=r1.key_capacity, **shape)
        eager = Optimizer(r1, Pe, tgt, stream=s)
        graph = Optimizer(r2, Pg, tgt, stream=s)
        graph.capture()
        for k in range(3):
            eager.step()
            graph.replay()
            s.synchronize()
            if k == 0:
                # same inputs, same kernels: the forward pass is bit-identical;
                # the loss is summed with atomics, so only up to rounding
                assert torch.equal(r1.images, r2.images)
                assert abs(eager.loss.item() - graph.loss.item()) <= 1e-6 * eager.loss.item()
            else:
                # gradients are summed with atomics in arbitrary order, so later
                # steps agree to rounding (Adam turns a sign flip of a
                # near-zero gradient into +-lr, hence the fraction test)
                assert abs(eager.loss.item() - graph.loss.item()) <= 1e-3 * eager.loss.item()
        for a, b in zip(Pe.tensors(), Pg.tensors()):
            close = (a - b).abs() <= 1e-5 + 1e-4 * a.abs()
            assert close.float().mean().item() > 0.99
        assert eager.step_count.item() == 3 and graph.step_count.item() == 3
        # stale arguments are refused
        graph.targets = tgt.clone()
        graph.invalidate()
        from paper_2604_02851_amd.native import GsError, GS_ERR_STALE
        with pytest.raises(GsError) as e:
            graph.replay()
        assert e.value.status == GS_ERR_STALE


def test_device_hparams_change_without_recapture():
    """The captured step reads Adam's hyper-parameters from device memory:
    after set_hparams with zero learning rates a replay leaves every
    parameter bit-identical (and still advances the step counter), and
    after restoring them a replay moves the model again, with no
    recapture and no GS_ERR_STALE."""
    from paper_2604_02851_amd.renderer import DEFAULT_LR
    w = S.small_workload(302, 3000, 1.0, 3, [(96, 64), (50, 50)], dist=3.0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        r = Renderer(w.cams, w.scene.n, 3, loss_mode=1, **BENCH_SHAPE)
        tgt = r.forward(DeviceParams.from_scene(w.extra["perturbed"]))[0].clone()
        P = DeviceParams.from_scene(w.scene)
        r.fit_capacity(P)
        opt = Optimizer(r, P, tgt, stream=s)
        opt.capture()
        opt.replay()
        s.synchronize()
        before = [t.clone() for t in P.tensors()]
        opt.set_hparams(lr=(0.0,) * 6)
        opt.replay()
        s.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(before, P.tensors()))
        assert opt.step_count.item() == 2
        opt.set_hparams(lr=DEFAULT_LR)
        opt.replay()
        s.synchronize()
        assert opt.step_count.item() == 3
        moved = sum(int((a != b).sum().item()) for a, b in zip(before, P.tensors()))
        assert moved > 0.5 * sum(t.numel() for t in before)
