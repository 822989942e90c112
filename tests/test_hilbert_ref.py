"""CPU pin of the numpy Hilbert index used by the target-order GPU test: on a
full grid of cells, consecutive Hilbert indices are face neighbours (one unit
step along one axis), which is what makes the curve a Hilbert curve; and the
index is a bijection."""
import numpy as np

from hilbert_ref import hilbert_from_morton


def _morton(q):
    k = np.zeros(len(q), np.uint64)
    for b in range(21):
        for i in range(3):
            k |= ((q[:, i] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + 2 - i)
    return k


def test_hilbert_unit_steps_on_full_grids():
    for level in (1, 2, 3):
        s = 1 << level
        g = np.array([(x, y, z) for x in range(s) for y in range(s) for z in range(s)], np.uint64)
        h = hilbert_from_morton(_morton(g << np.uint64(21 - level)))
        assert len(np.unique(h)) == len(g)
        o = np.argsort(h)
        steps = np.abs(np.diff(g[o].astype(np.int64), axis=0)).sum(1)
        assert (steps == 1).all(), level
        assert tuple(g[o][0]) == (0, 0, 0)


def test_hilbert_cells_are_contiguous_ranges():
    """Every cell of a coarser level is one contiguous range of the index."""
    g = np.random.default_rng(5).integers(0, 1 << 21, size=(20000, 3)).astype(np.uint64)
    h = hilbert_from_morton(_morton(g))
    o = np.argsort(h)
    for level in (1, 2, 4, 6):
        cell = (g[o] >> np.uint64(21 - level))
        cid = (cell[:, 0] << np.uint64(2 * level)) | (cell[:, 1] << np.uint64(level)) | cell[:, 2]
        changes = np.count_nonzero(np.diff(cid.astype(np.int64)))
        assert changes == len(np.unique(cid)) - 1, level
