"""Gaussian freezing (Sec. 3.3: an active pool that is optimised and a frozen
pool that is only rendered) through the C ABI: the adjoint restricted to the
active prefix equals the oracle gradient's columns for those Gaussians (the
frozen ones still shape every pixel), Adam leaves frozen Gaussians untouched,
gs_freeze's partition is bit-exact against the oracle's, and the batched step
with a frozen pool replays from a graph like the eager step."""
import numpy as np
import pytest
import torch

from gpu_util import adam_check, compare_images, flat_grads, grad_report, renderer_for
from paper_2604_02851_amd import scenes as S
from paper_2604_02851_amd.native import DeviceParams

pytestmark = pytest.mark.gpu
F32 = np.float32


def _cols(b, na):
    from oracle.oracle import Backward
    return Backward(b.grad[:, :na], b.scale[:, :na], b.slack[:, :na], b.scale_t[:, :na], b.loss, b.image)


def test_adjoint_of_active_pool_matches_oracle_columns(oracle):
    w = S.small_workload(120, 1500, 1.0, 3, [(80, 60), (48, 64)], dist=3.0)
    r = renderer_for(w, tile=(32, 32), batch=128, ppt=4, wave_w=16)
    P = DeviceParams.from_scene(w.scene)
    G = np.random.default_rng(7).normal(size=3 * w.n_pixels).astype(F32)
    b = oracle.backward(w.scene, w.cams, G, mode=0)
    for na in (1500, 900, 1, 0):
        r.forward(P)
        grads = DeviceParams.zeros(na, 3)
        r.backward(P, torch.from_numpy(G).cuda(), 0, grads)
        torch.cuda.synchronize()
        if na == 0:
            continue
        rep = grad_report(flat_grads(grads), _cols(b, na))
        print("active", na, rep)
        assert rep["fail"] == 0


def test_adam_updates_only_the_active_prefix(oracle):
    rng = np.random.default_rng(9)
    sc = S.draw_scene(rng, 3001, 2.0, 3)
    P = DeviceParams.from_scene(sc)
    na = 1777
    rows = [t.reshape(-1, sc.n).shape[0] for t in P.tensors()]
    mk = lambda f: DeviceParams(*[torch.from_numpy(f((r_, na)).astype(F32).reshape(t.shape[:-1] + (na,))).cuda()
                                  for r_, t in zip(rows, P.tensors())], 3)
    g = mk(lambda s: rng.normal(size=s))
    m = mk(lambda s: 0.1 * rng.normal(size=s))
    v = mk(lambda s: np.abs(rng.normal(size=s)))
    theta0 = [t.cpu().numpy().reshape(-1, sc.n).copy() for t in P.tensors()]
    g0, m0, v0 = ([t.cpu().numpy().reshape(-1, na).copy() for t in x.tensors()] for x in (g, m, v))
    step = torch.tensor([2], dtype=torch.int32, device="cuda")
    lr = (1e-3, 5e-3, 1e-3, 5e-2, 5e-3, 2.5e-3)
    from paper_2604_02851_amd.native import Context
    Context(0).adam_step(P, g, m, v, step, lr, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    out = [t.cpu().numpy().reshape(-1, sc.n) for t in P.tensors()]
    out_m, out_v = ([t.cpu().numpy().reshape(-1, na) for t in x.tensors()] for x in (m, v))
    groups = [(0, slice(None), lr[0]), (1, slice(None), lr[1]), (2, slice(None), lr[2]), (3, slice(None), lr[3]),
              (4, slice(0, 3), lr[4]), (4, slice(3, None), lr[5])]
    for ti, sl, l in groups:
        adam_check(oracle, theta0[ti][sl][:, :na], g0[ti][sl], m0[ti][sl], v0[ti][sl], out[ti][sl][:, :na],
                   out_m[ti][sl], out_v[ti][sl], l, 0.9, 0.999, 1e-8, 3)
        assert np.array_equal(out[ti][sl][:, na:], theta0[ti][sl][:, na:])   # frozen: untouched


def _rows(dp, n):
    return [t.detach().cpu().numpy().reshape(-1, n).copy() for t in dp.tensors()]


@pytest.mark.parametrize("n,na,frac", [(2000, 1300, 0.35), (2001, 2001, 0.5), (777, 500, 0.0), (640, 300, 1.0)])
def test_freeze_partition_bit_exact(oracle, n, na, frac):
    w = S.small_workload(130, n, 1.0, 3, [(64, 48)], dist=3.0)
    r = renderer_for(w)
    rng = np.random.default_rng(n + na)
    P = DeviceParams.from_scene(w.scene)
    base = DeviceParams(*[t + 0.5 for t in P.tensors()], 3)
    rows = [t.reshape(-1, n).shape[0] for t in P.tensors()]
    mk = lambda: DeviceParams(*[torch.from_numpy(rng.normal(size=(r_, na)).astype(F32).reshape(t.shape[:-1] + (na,)))
                                .cuda() for r_, t in zip(rows, P.tensors())], 3)
    m, v = mk(), mk()
    ids = torch.arange(n, dtype=torch.int32, device="cuda")
    flags_np = (rng.random(na) < frac).astype(np.uint8)
    flags = torch.from_numpy(flags_np).cuda()
    p0, b0, m0, v0 = _rows(P, n), _rows(base, n), _rows(m, na), _rows(v, na)
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    r.ctx.freeze(P, m, v, flags, r.ws, out, ids=ids, baseline=base)
    torch.cuda.synchronize()
    na2 = int(out.item())
    all_rows = p0 + b0 + [np.arange(n, dtype=np.uint32)[None]]
    exp_all, exp_act, na_ref, order = oracle.freeze_partition(all_rows, m0 + v0, flags_np, na)
    assert na2 == na_ref
    got_all = _rows(P, n) + _rows(base, n) + [ids.cpu().numpy().view(np.uint32)[None]]
    for a, e in zip(got_all, exp_all):
        assert np.array_equal(a, e)
    if na2 > 0:
        got_act = _rows(m.narrowed(na2), na2) + _rows(v.narrowed(na2), na2)
        for a, e in zip(got_act, exp_act):
            assert np.array_equal(a, e)


def test_step_with_frozen_pool_graph_and_migration(oracle):
    from paper_2604_02851_amd.native import GS_ERR_STALE, GsError
    from paper_2604_02851_amd.renderer import Optimizer, Renderer
    w = S.small_workload(303, 3000, 1.0, 3, [(96, 64), (64, 96), (50, 50)], dist=3.0)
    shape = dict(tile=(32, 32), batch_depth=128, pixels_per_thread=4, wave_w=16)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        r1 = Renderer(w.cams, w.scene.n, 3, loss_mode=1, **shape)
        tgt = r1.forward(DeviceParams.from_scene(w.extra["perturbed"]))[0].clone()
        Pe, Pg = DeviceParams.from_scene(w.scene), DeviceParams.from_scene(w.scene)
        r1.fit_capacity(Pe)
        r2 = Renderer(w.cams, w.scene.n, 3, loss_mode=1, key_capacity=r1.key_capacity, **shape)
        na = 2000
        eager = Optimizer(r1, Pe, tgt, stream=s, n_active=na)
        graph = Optimizer(r2, Pg, tgt, stream=s, n_active=na)
        frozen0 = _rows(Pe, 3000)
        graph.capture()
        for _ in range(2):
            eager.step()
            graph.replay()
        s.synchronize()
        for a, b, f in zip(_rows(Pe, 3000), _rows(Pg, 3000), frozen0):
            assert np.array_equal(a[:, na:], f[:, na:]) and np.array_equal(b[:, na:], f[:, na:])
            assert not np.array_equal(a[:, :na], f[:, :na])
            close = np.abs(a - b) <= 1e-5 + 1e-4 * np.abs(a)
            assert close.mean() > 0.99
        # migrate every third active Gaussian into the frozen pool
        flags = (torch.arange(na, device="cuda") % 3 == 0).to(torch.uint8)
        assert eager.freeze(flags) == graph.freeze(flags) == na - (na + 2) // 3
        with pytest.raises(GsError) as e:
            graph.replay()
        assert e.value.status == GS_ERR_STALE
        graph.capture()
        eager.step()
        graph.replay()
        s.synchronize()
        assert abs(eager.loss.item() - graph.loss.item()) <= 1e-3 * eager.loss.item()
        # the permuted model renders like the oracle's render of it
        img = r1.forward(Pe)[0].clone()
        s.synchronize()
        compare_images(oracle, S.Workload("permuted", Pe.to_scene(), w.cams, 16, {}), img.cpu().numpy())
