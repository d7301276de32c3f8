"""The traversal plan (host logic, CPU): every tile's order is a permutation
of its rectangle; batch zigzag (Sec. 2.3) and the Hilbert curve (Sec. 5.4)
are continuous paths (consecutive points are grid neighbours); the Morton
order (Sec. 5.4) sorts the points by their interleaved coordinate bits,
computed here independently; batch zigzag visits each band of height b
column by column in alternating directions."""
import numpy as np
import pytest

P = pytest.importorskip("paper_2606_26785_amd")


def _rects(nx, ny, tx, ty):
    for jy in range(ty):
        y0, y1 = ny * jy // ty, ny * (jy + 1) // ty
        for jx in range(tx):
            x0, x1 = nx * jx // tx, nx * (jx + 1) // tx
            yield x0, x1, y0, y1


@pytest.mark.parametrize("traversal", [0, 1, 2])
@pytest.mark.parametrize("nx,ny,tx,ty,b", [(16, 16, 1, 1, 4), (37, 23, 3, 2, 5), (9, 1, 2, 1, 3), (1, 7, 1, 1, 2)])
def test_tiles_are_permutations(traversal, nx, ny, tx, ty, b):
    tiles = P.debug_order(nx, ny, tx, ty, b, traversal)
    allp = np.concatenate(tiles)
    assert np.array_equal(np.sort(allp), np.arange(nx * ny))
    for o, (x0, x1, y0, y1) in zip(tiles, _rects(nx, ny, tx, ty)):
        i, j = o % nx, o // nx
        assert (i >= x0).all() and (i < x1).all() and (j >= y0).all() and (j < y1).all()
        assert o.size == (x1 - x0) * (y1 - y0)


@pytest.mark.parametrize("traversal,side", [(0, 16), (1, 16), (1, 32), (0, 13)])
def test_continuous_paths(traversal, side):
    b = 4
    (o,) = P.debug_order(side, side, 1, 1, b, traversal)
    i, j = o % side, o // side
    step = np.abs(np.diff(i)) + np.abs(np.diff(j))
    if traversal == 0:
        # continuous inside each band of height b; a band change moves to
        # the next band in the same column
        same_band = (j[1:] // b) == (j[:-1] // b)
        assert (step[same_band] == 1).all()
        assert (np.diff(i)[~same_band] == 0).all()
    else:
        assert (step == 1).all()


def test_hilbert_starts_and_ends_on_the_bottom_edge():
    (o,) = P.debug_order(8, 8, 1, 1, 1, 1)
    i, j = o % 8, o // 8
    assert (i[0], j[0]) == (0, 0)
    assert j[-1] == 0 and i[-1] == 7


def test_morton_order():
    nx, ny = 12, 9
    (o,) = P.debug_order(nx, ny, 1, 1, 1, 2)
    i, j = o % nx, o // nx

    def key(x, y):
        k = 0
        for bit in range(8):
            k |= ((x >> bit) & 1) << (2 * bit)
            k |= ((y >> bit) & 1) << (2 * bit + 1)
        return k
    keys = np.array([key(int(a), int(c)) for a, c in zip(i, j)])
    assert (np.diff(keys) > 0).all()


def test_batch_zigzag_bands():
    nx, ny, b = 6, 7, 3
    (o,) = P.debug_order(nx, ny, 1, 1, b, 0)
    i, j = o % nx, o // nx
    # band k covers rows [k b, min((k + 1) b, ny)), visited left to right for
    # even k and right to left for odd k, a vertical snake in each column
    pos = 0
    for k, y0 in enumerate(range(0, ny, b)):
        h = min(b, ny - y0)
        cols = range(nx) if k % 2 == 0 else range(nx - 1, -1, -1)
        for c, x in enumerate(cols):
            ys = list(range(y0, y0 + h)) if c % 2 == 0 else list(range(y0 + h - 1, y0 - 1, -1))
            assert list(i[pos:pos + h]) == [x] * h
            assert list(j[pos:pos + h]) == ys
            pos += h
    assert pos == nx * ny


def test_bad_arguments():
    with pytest.raises(P.PSError):
        P.debug_order(4, 4, 1, 1, 1, 3)
    with pytest.raises(P.PSError):
        P.debug_order(4, 4, 5, 1, 1, 0)
