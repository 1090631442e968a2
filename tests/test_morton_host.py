"""Host checks of the tiled Morton cell order (no GPU): the key of a cell is
a bijection from the grid into the padded key range, the cells of one 8^d tile
take one contiguous key block, and the curve inside a tile is the Morton
curve (consecutive keys differ by one cell along some axis within aligned
2^k blocks)."""
import itertools

import numpy as np

from _parity import tiled_morton_key


def _all_cells(nc):
    g = np.meshgrid(*[np.arange(n) for n in nc], indexing="ij")
    return [a.ravel() for a in g]


def test_bijection_and_padded_range():
    for dim, nc in ((2, (13, 9, 1)), (3, (11, 7, 10)), (3, (16, 8, 8))):
        cx, cy, cz = _all_cells(nc)
        k = tiled_morton_key(cx, cy, cz, nc, dim)
        tiles = ((nc[0] + 7) // 8) * ((nc[1] + 7) // 8) * ((nc[2] + 7) // 8 if dim == 3 else 1)
        assert len(np.unique(k)) == len(k)
        assert k.min() >= 0 and k.max() < tiles * 8 ** dim


def test_tiles_are_contiguous_blocks():
    nc, dim = (20, 12, 9), 3
    cx, cy, cz = _all_cells(nc)
    k = tiled_morton_key(cx, cy, cz, nc, dim)
    tile_of_cell = (cx // 8) + 3 * ((cy // 8) + 2 * (cz // 8))
    assert np.array_equal(k >> 9, tile_of_cell)


def test_morton_curve_inside_a_tile():
    # in a full tile the first 2^(d j) keys cover the aligned 2^j block at the origin
    for dim in (2, 3):
        nc = (8, 8, 8 if dim == 3 else 1)
        cx, cy, cz = _all_cells(nc)
        k = tiled_morton_key(cx, cy, cz, nc, dim)
        for j in (1, 2, 3):
            sel = k < 2 ** (dim * j)
            assert cx[sel].max() == 2 ** j - 1 and cy[sel].max() == 2 ** j - 1
            if dim == 3:
                assert cz[sel].max() == 2 ** j - 1
        # key 1 is the +x neighbour of key 0, key 2 the +y one
        order = np.argsort(k)
        assert (cx[order[1]], cy[order[1]]) == (1, 0) and (cx[order[2]], cy[order[2]]) == (0, 1)
