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


def test_cell_of_hand_computed():
    """The cell of a point (Sec. 3.3 preculling grid) worked out by hand on a
    grid of 4 x 3 x 2 cells of edge 0.5 from (-1, -2, -3): index
    cx + 4 (cy + 3 cz); outside the grid (or not a number) the extra index 24.
    A cell's lower faces belong to it, its upper faces to the next cell."""
    nan, inf = float("nan"), float("inf")
    cases = [
        ((-1.0, -2.0, -3.0), 0),            # the origin corner
        ((-0.5, -2.0, -3.0), 1),            # on the face between cells 0 and 1
        ((-0.75, -1.25, -2.25), 16),        # t = (0.5, 1.5, 1.5): (0, 1, 1)
        ((0.75, -0.75, -2.25), 23),         # t = (3.5, 2.5, 1.5): the last cell
        ((0.9, -0.6, -2.1), 23),            # inside the last cell, near its far corner
        ((-0.99, -1.99, -2.99), 0),         # negative coordinates, inside cell 0
        ((1.0, -2.0, -3.0), 24),            # t_x = 4 = dims_x: the upper face of the grid
        ((-1.25, -2.0, -3.0), 24),          # below the origin in x
        ((-1.0, -0.5, -3.0), 24),           # t_y = 3 = dims_y
        ((-1.0, -2.0, -2.0), 24),           # t_z = 2 = dims_z
        ((-1.0, -2.0, -3.25), 24),          # below the origin in z
        # x = 1 - 2^-24: x + 1 = 2 - 2^-24 rounds to 2 in FP32 (ties to even), so
        # t_x = 4 and the point lies outside, although it is inside in exact arithmetic
        ((float(np.float32(1.0) - np.float32(2.0 ** -24)), -2.0, -3.0), 24),
        ((0.9999, -2.0, -3.0), 3),          # the same face approached from inside
        ((nan, 0.0, 0.0), 24),
        ((0.0, nan, -3.0), 24),
        ((inf, -2.0, -3.0), 24),
        ((-inf, -2.0, -3.0), 24),
    ]
    pts = np.array([p for p, _ in cases], np.float32).T
    got = O.cell_of(pts, (-1.0, -2.0, -3.0), 0.5, (4, 3, 2))
    assert got.tolist() == [c for _, c in cases]
