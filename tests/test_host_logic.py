"""Host-side logic of the Python binding that needs no GPU: the guard that
keeps a rasterizer backward from using another forward's state, the key
capacity fitting (grow on a short or overflowed capacity, never shrink below
a need already seen), and the autotuner's search over launch shapes."""
from types import SimpleNamespace

import pytest
import torch

from paper_2604_02851_amd import native as N
from paper_2604_02851_amd.renderer import (TUNE_BATCHES, TUNE_SCHEDULES, TUNE_SHAPES, GaussianRasterize, Renderer,
                                           tune_search)


def test_rasterize_backward_refuses_state_of_a_later_forward():
    r = SimpleNamespace(forward_count=3)
    ctx = SimpleNamespace(renderer=r, forward_id=2, saved_tensors=(torch.zeros(3),), params=None)
    with pytest.raises(RuntimeError, match="another forward"):
        GaussianRasterize.backward(ctx, torch.zeros(3))


class _FakeCtx:
    """Stands in for the library context: each build 'needs' the next count of
    `needs`; a build over the capacity reports an overflow."""

    def __init__(self, needs, cap):
        self.needs, self.cap, self.keys = list(needs), cap, 0
        self.plans = []

    def project(self, *a, **k):
        pass

    def build_tile_lists(self, *a, **k):
        self.keys = self.needs.pop(0)

    def read_counters(self, ws):
        over = 1 if self.keys > self.cap else 0
        return N.GsCounters(0, self.keys, self.cap, over, over)


def _renderer(needs, cap):
    r = Renderer.__new__(Renderer)
    r.ctx = _FakeCtx(needs, cap)
    r.cams = [None, None]                   # two views
    r.key_capacity, r.max_need, r.forward_count, r.capacity_exceeded = cap, 0, 0, False
    r.dev_cams, r.ws = None, None

    def replan(c):
        r.ctx.plans.append(c)
        r.key_capacity = r.ctx.cap = c
        r.capacity_exceeded = False
    r.replan = replan
    return r


def test_fit_capacity_grows_and_never_drops_below_a_seen_need():
    r = _renderer([5000, 1000], 2048)
    assert r.fit_capacity(None) == 5000            # overflow: grows
    assert r.key_capacity >= 5000 and r.ctx.plans
    cap = r.key_capacity
    assert r.fit_capacity(None) == 1000            # a smaller model: the capacity keeps the larger need
    assert r.key_capacity == cap


def test_fit_capacity_replans_at_once_after_an_overflowing_view():
    r = _renderer([100, 9000, 50], 1024)
    assert r.fit_capacity(None, per_view=True) == 9000
    # re-planned right after the overflowing view, before the next one ran
    assert r.ctx.plans[0] >= 9000 and r.key_capacity >= 9000


def test_tune_search_finds_a_separable_optimum_and_times_each_shape_once():
    """With a cost that is a sum of per-dimension costs, the coordinate
    search must land on the product of the per-dimension optima, visit every
    built shape, batch depth and schedule, and time no candidate twice."""
    shape_cost = {s: 1.0 + 0.1 * k for k, s in enumerate(TUNE_SHAPES)}
    best_shape = TUNE_SHAPES[7]
    shape_cost[best_shape] = 0.5
    batch_cost = {32: 0.3, 64: 0.2, 128: 0.0, 256: 0.4}
    sched_cost = {0: 0.2, 1: 0.3, 2: 0.1, 3: 0.0}
    seen = []

    def cost(c):
        seen.append(c)
        tile, batch, ppt, sw, sched = c
        return shape_cost[(tile, ppt, sw)] + batch_cost[batch] + sched_cost[sched]

    best, times = tune_search(cost)
    assert best == (best_shape[0], 128, best_shape[1], best_shape[2], 3)
    assert len(seen) == len(set(seen)) == len(times)
    assert {(c[0], c[2], c[3]) for c in seen} == set(TUNE_SHAPES)
    assert {c[1] for c in seen} == set(TUNE_BATCHES)
    assert {c[4] for c in seen} == set(TUNE_SCHEDULES)
    assert times[best] == min(times.values())


def test_tune_search_rechecks_runners_up_with_the_chosen_batch_and_schedule():
    """A shape that loses at the starting batch depth but wins at the chosen
    one is found by the re-check of the runners-up."""
    a, b = TUNE_SHAPES[3], TUNE_SHAPES[5]

    def cost(c):
        tile, batch, ppt, sw, sched = c
        s = (tile, ppt, sw)
        if s == a:
            return 1.0 if batch == 64 else 0.9
        if s == b:
            return 1.1 if batch == 64 else 0.5
        return 2.0

    best, _ = tune_search(cost)
    assert (best[0], best[2], best[3]) == b
