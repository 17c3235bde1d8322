"""Pins of the oracle's patch assembly (Sec. 2.5 overlap blending at known
positions, with the tiles brought to a common constant phase first).

* Tiles cut from one field and given arbitrary constant phases: the
  synchronisation returns those phases (up to the common one) and the blend
  returns the field exactly wherever a tile covers it, for any ramp width.
* One tile alone is returned unchanged; uncovered canvas stays zero.
* The ramp's closed form at its ends and middle.
* Across an overlap as wide as the ramp, the two ramps sum to one and the
  canvas is the stated convex combination.
"""

import numpy as np
import pytest

from oracle import assemble as oa


def _field(shape, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 1.0, shape) * np.exp(1j * rng.uniform(-np.pi, np.pi, shape))


def _cut(field, n, stride, rows, cols):
    pos, tiles = [], []
    for i in range(rows):
        for j in range(cols):
            y, x = i * stride, j * stride
            pos.append((y, x))
            tiles.append(field[y:y + n, x:x + n])
    return np.array(tiles), np.array(pos)


@pytest.mark.parametrize("width", [1.0, 4.0, 12.0])
def test_cut_tiles_reassemble_exactly(width):
    n, stride, rows, cols = 32, 24, 3, 4
    field = _field(((rows - 1) * stride + n, (cols - 1) * stride + n))
    tiles, pos = _cut(field, n, stride, rows, cols)
    rng = np.random.default_rng(1)
    phases = rng.uniform(-np.pi, np.pi, len(tiles))
    shifted = tiles * np.exp(1j * phases)[:, None, None]
    theta = oa.synchronise_phases(oa.overlap_matrix(shifted, pos))
    d = np.angle(np.exp(1j * (theta - (phases - phases[0]))))
    assert np.abs(d).max() < 1e-12
    out = oa.blend(shifted, pos, theta, field.shape, width)
    ref = field * np.exp(1j * phases[0])
    assert np.abs(out - ref).max() < 1e-12


def test_separate_groups_synchronise_on_their_own():
    """Two 2 x 2 groups far apart: each group's phases come back relative to
    its own first tile."""
    n, stride = 16, 12
    field = _field((100, 100), seed=8)
    pos = np.array([[0, 0], [0, stride], [stride, 0], [stride, stride],
                    [60, 60], [60, 60 + stride], [60 + stride, 60], [60 + stride, 60 + stride]])
    tiles = np.stack([field[y:y + n, x:x + n] for y, x in pos])
    phases = np.random.default_rng(2).uniform(-np.pi, np.pi, len(pos))
    theta = oa.synchronise_phases(oa.overlap_matrix(tiles * np.exp(1j * phases)[:, None, None], pos))
    for g in (range(0, 4), range(4, 8)):
        g = list(g)
        d = np.angle(np.exp(1j * (theta[g] - (phases[g] - phases[g[0]]))))
        assert np.abs(d).max() < 1e-12
    assert theta[0] == 0 and theta[4] == 0


def test_single_tile_and_uncovered_canvas():
    n = 16
    tile = _field((n, n), seed=3)[None]
    out = oa.blend(tile, np.array([[5, 7]]), np.zeros(1), (30, 40), 4.0)
    assert np.abs(out[5:5 + n, 7:7 + n] - tile[0]).max() < 1e-15
    mask = np.ones((30, 40), bool)
    mask[5:5 + n, 7:7 + n] = False
    assert np.all(out[mask] == 0)


def test_ramp_closed_form():
    r = oa.ramp(16, 4.0)
    assert r[0] == pytest.approx(0.125) and r[1] == pytest.approx(0.375)
    assert r[3] == pytest.approx(0.875) and r[4] == 1.0 and r[11] == 1.0
    assert r[15] == pytest.approx(0.125)


def test_overlap_weights_partition_unity():
    """Two 16 px tiles side by side with an 8 px overlap and ramp width 8:
    across the overlap the two ramps sum to 1, so at tile-0 column 12 (tile-1
    column 4) the canvas is 3.5/8 of tile 0 plus 4.5/8 of tile 1."""
    n = 16
    a = _field((n, n), seed=5)
    b = _field((n, n), seed=6)
    out = oa.blend(np.stack([a, b]), np.array([[0, 0], [0, 8]]), np.zeros(2), (n, 24), 8.0)
    r = oa.ramp(n, 8.0)
    assert np.allclose(r[8:] + r[:8], 1.0)
    y = 8
    assert out[y, 12] == pytest.approx(3.5 / 8 * a[y, 12] + 4.5 / 8 * b[y, 4], rel=1e-14)
