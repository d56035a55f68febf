"""Pins of the cell grouping order (Sec. 3.3: Gaussians assigned to grid
cells) against Python's own stable sort and against its plain properties: a
permutation that keeps the active and frozen pools in place, orders each pool
by cell with ties in old order, and sends out-of-range cells to the end."""
import numpy as np

from oracle import oracle as O


def _stable(cells, na, n_cells):
    key = [min(int(c), n_cells) for c in cells]
    n = len(key)
    act = sorted(range(na), key=lambda i: key[i])
    frz = sorted(range(na, n), key=lambda i: key[i])
    return np.array(act + frz, np.int64)


def test_matches_library_stable_sort():
    rng = np.random.default_rng(11)
    for n, na, n_cells in ((1, 1, 1), (1, 0, 3), (40, 40, 5), (57, 20, 7), (64, 0, 9), (33, 17, 1)):
        cells = rng.integers(0, n_cells + 3, n)   # some values beyond n_cells: the outside cell
        order = O.cell_order(cells, na, n_cells)
        assert np.array_equal(order, _stable(cells, na, n_cells)), (n, na, n_cells)


def test_properties():
    rng = np.random.default_rng(12)
    n, na, n_cells = 90, 50, 6
    cells = rng.integers(0, n_cells + 2, n)
    order = O.cell_order(cells, na, n_cells)
    assert sorted(order.tolist()) == list(range(n))
    assert set(order[:na].tolist()) == set(range(na))          # pools stay in place
    key = np.minimum(cells, n_cells)[order]
    for lo, hi in ((0, na), (na, n)):
        k, o = key[lo:hi], order[lo:hi]
        assert np.all(np.diff(k) >= 0)                         # grouped by cell
        same = np.diff(k) == 0
        assert np.all(np.diff(o)[same] > 0)                    # ties keep their order
    # already grouped: the identity
    srt = np.sort(rng.integers(0, n_cells, 30))
    assert np.array_equal(O.cell_order(srt, 30, n_cells), np.arange(30))
    # applying the order to the keys a second time changes nothing
    again = O.cell_order(np.asarray(cells)[order], na, n_cells)
    assert np.array_equal(again, np.arange(n))
