"""Grouping the model by preculling cell (Sec. 3.3) through the C ABI: the
in-place reorder is bit-exact against the oracle's order for parameters,
baseline, ids, cell indices and moments (pools kept apart, out-of-range
cells last, sizes spanning several sort chunks and several digit passes);
after grouping a rig scene, its cells are contiguous and the reordered
model renders like the oracle's render of it; an optimizer grouped between
steps keeps replaying its captured graph like the eager step."""
import numpy as np
import pytest
import torch

from gpu_util import compare_images, renderer_for
from paper_2604_02851_amd import scenes as S
from paper_2604_02851_amd.native import DeviceParams
from paper_2604_02851_amd.renderer import Optimizer, Renderer

pytestmark = pytest.mark.gpu
F32 = np.float32
GRID = dict(origin=(-20.0, -2.0, -20.0), cell_size=2.5, dims=(16, 2, 16))
SHAPE = dict(tile=(32, 32), batch_depth=128, pixels_per_thread=4, wave_w=16)


def _rows(dp, n):
    return [t.detach().cpu().numpy().reshape(-1, n).copy() for t in dp.tensors()]


@pytest.mark.parametrize("n,na,n_cells,moments", [(5000, 3000, 37, True), (4097, 4097, 300, False),
                                                  (1, 1, 1, True), (70001, 41234, 700, True),
                                                  (9000, 0, 1 << 20, True)])
def test_sort_cells_bit_exact(oracle, n, na, n_cells, moments):
    w = S.small_workload(140, n, 1.0, 3, [(64, 48)], dist=3.0)
    r = renderer_for(w)
    rng = np.random.default_rng(n + na + n_cells)
    P = DeviceParams.from_scene(w.scene)
    base = DeviceParams(*[t + 0.5 for t in P.tensors()], 3)
    rows = [t.reshape(-1, n).shape[0] for t in P.tensors()]
    mk = lambda: DeviceParams(*[torch.from_numpy(rng.normal(size=(r_, na)).astype(F32).reshape(t.shape[:-1] + (na,)))
                                .cuda() for r_, t in zip(rows, P.tensors())], 3)
    m, v = (mk(), mk()) if moments else (None, None)
    ids = torch.arange(n, dtype=torch.int32, device="cuda")
    # cells, with some indices beyond the grid (sorted as the outside cell)
    cells_np = rng.integers(0, n_cells + max(2, n_cells // 8), n).astype(np.uint32)
    cells_np[rng.random(n) < 0.05] = 0xFFFFFFFF
    cells = torch.from_numpy(cells_np.view(np.int32)).cuda()
    p0, b0 = _rows(P, n), _rows(base, n)
    mv0 = (_rows(m, na) + _rows(v, na)) if moments and na > 0 else []
    r.ctx.sort_cells(P, cells, n_cells, r.ws, m=m, v=v, ids=ids, baseline=base)
    torch.cuda.synchronize()
    order = oracle.cell_order(cells_np, na if moments else n, n_cells)
    for a, e in zip(_rows(P, n) + _rows(base, n), p0 + b0):
        assert np.array_equal(a, e[:, order])
    assert np.array_equal(ids.cpu().numpy(), order.astype(np.int32))
    assert np.array_equal(cells.cpu().numpy().view(np.uint32), cells_np[order])
    if mv0:
        for a, e in zip(_rows(m, na) + _rows(v, na), mv0):
            assert np.array_equal(a, e[:, order[:na]])


def test_grouped_rig_scene_renders_like_oracle(oracle):
    w = S.rig_workload(4, 6000, views=3, size=(160, 96))
    r = Renderer(w.cams, w.scene.n, 3, **SHAPE)
    P = DeviceParams.from_scene(w.scene)
    r.enable_precull(P, **GRID)
    r.sort_cells(P)
    torch.cuda.synchronize()
    cells = r.cell_of.cpu().numpy().astype(np.int64)
    assert np.all(np.diff(cells) >= 0)
    sc = P.to_scene()
    assert np.array_equal(cells, oracle.cell_of(sc.mean, GRID["origin"], GRID["cell_size"], GRID["dims"]))
    # the same set of Gaussians, regrouped
    key = lambda s: np.lexsort(s.mean)
    assert np.array_equal(sc.mean[:, key(sc)], w.scene.mean[:, key(w.scene)])
    r.update_precull(P)
    r.fit_capacity(P)
    img = r.forward(P)[0].clone()
    torch.cuda.synchronize()
    compare_images(oracle, S.Workload("grouped", sc, w.cams, 16, {}), img.cpu().numpy())


def test_grouping_between_steps_keeps_graph_valid():
    w = S.rig_workload(5, 5000, views=3, size=(160, 96))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        r1 = Renderer(w.cams, w.scene.n, 3, loss_mode=1, **SHAPE)
        tgt = r1.forward(DeviceParams.from_scene(w.extra["perturbed"]))[0].clone()
        Pe, Pg = DeviceParams.from_scene(w.scene), DeviceParams.from_scene(w.scene)
        r1.fit_capacity(Pe)
        r2 = Renderer(w.cams, w.scene.n, 3, loss_mode=1, key_capacity=r1.key_capacity, **SHAPE)
        for r, P in ((r1, Pe), (r2, Pg)):
            r.enable_precull(P, **GRID)
        eager = Optimizer(r1, Pe, tgt, stream=s, n_active=4000)
        graph = Optimizer(r2, Pg, tgt, stream=s, n_active=4000)
        eager.ids = torch.arange(5000, dtype=torch.int32, device="cuda")
        graph.ids = torch.arange(5000, dtype=torch.int32, device="cuda")
        graph.capture()
        eager.step()
        graph.replay()
        eager.sort_cells()
        graph.sort_cells()
        for _ in range(2):
            eager.step()
            graph.replay()
        s.synchronize()
        assert torch.equal(eager.ids, graph.ids)
        assert not torch.equal(eager.ids, torch.arange(5000, dtype=torch.int32, device="cuda"))
        assert sorted(eager.ids[:4000].tolist()) == list(range(4000))   # the active pool stays the active pool
        for a, b in zip(_rows(Pe, 5000), _rows(Pg, 5000)):
            close = np.abs(a - b) <= 1e-5 + 1e-4 * np.abs(a)
            assert close.mean() > 0.99
        assert abs(eager.loss.item() - graph.loss.item()) <= 1e-3 * eager.loss.item()
