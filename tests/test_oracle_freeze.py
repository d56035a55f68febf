"""Pins of the freezing partition (Sec. 3.3: active and frozen pools) against
its plain properties: a permutation of the Gaussian axis that is stable within
each class, leaves the previously frozen tail in place, and compacts the
moments of the Gaussians that stay active; idempotent for empty flags."""
import numpy as np

from oracle import oracle as O


def _case(seed, n=37, na=23):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(5, n)).astype(np.float32)
    ids = np.arange(n, dtype=np.uint32)[None]
    m = rng.normal(size=(5, na)).astype(np.float32)
    flags = rng.random(na) < 0.4
    return p, ids, m, flags, n, na


def test_partition_is_stable_and_keeps_frozen_tail():
    p, ids, m, flags, n, na = _case(1)
    (p2, ids2), (m2,), na2, order = O.freeze_partition([p, ids], [m], flags, na)
    assert na2 == int((~flags).sum())
    # a permutation of 0..n-1
    assert sorted(order.tolist()) == list(range(n))
    # stays-active first, in order; then newly frozen in order; then the old tail
    assert order[:na2].tolist() == [i for i in range(na) if not flags[i]]
    assert order[na2:na].tolist() == [i for i in range(na) if flags[i]]
    assert order[na:].tolist() == list(range(na, n))
    # columns travel whole
    assert np.array_equal(p2, p[:, order]) and np.array_equal(ids2[0], order.astype(np.uint32))
    # moments of the Gaussians that stay active, compacted in order
    assert np.array_equal(m2, m[:, ~flags])


def test_partition_special_cases():
    p, ids, m, flags, n, na = _case(2)
    none = np.zeros(na, bool)
    (p2,), (m2,), na2, order = O.freeze_partition([p], [m], none, na)
    assert na2 == na and np.array_equal(p2, p) and np.array_equal(m2, m)
    allf = np.ones(na, bool)
    (p3,), (m3,), na3, order3 = O.freeze_partition([p], [m], allf, na)
    assert na3 == 0 and m3.shape == (5, 0) and np.array_equal(p3, p)
    # two partitions compose: freezing A then B equals freezing A|B in one go
    # when B only flags Gaussians that were active after A
    rng = np.random.default_rng(3)
    fa = rng.random(na) < 0.3
    (pa,), (ma,), naa, oa = O.freeze_partition([p], [m], fa, na)
    fb = rng.random(naa) < 0.5
    (pb,), (mb,), nab, ob = O.freeze_partition([pa], [ma], fb, naa)
    assert nab == naa - int(fb.sum())
    assert np.array_equal(mb, m[:, ~fa][:, ~fb])
    assert sorted(oa[ob].tolist()) == list(range(n))
