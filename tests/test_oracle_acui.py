"""Pins of the ACUI grid oracle (Eq. 13): closed-form counts, the grid's
symmetry and spacing, and the covering property that the index range
+-([M / 2d] + 1) gives (the outermost points lie beyond the cuboid's faces,
the next ones inside), checked against values worked out by hand."""
import numpy as np
import pytest

from oracle import acui as A


def test_hand_worked_case():
    # S = 2, M = 256, d = 8: [256 / 16] + 1 = 17, so n in -17..17 and the
    # spacing is 2 * 8 / 256 = 1/16 on every axis (35^3 = 42 875 points)
    assert A.half_extent(256, 8) == 17
    assert A.count((2, 2, 2), (256, 256, 256), 8) == 42875
    p = A.points((2, 2, 2), (256, 256, 256), 8)
    assert p.shape == (42875, 3) and p.dtype == np.float32
    assert p[0].tolist() == [-17 / 16] * 3 and p[-1].tolist() == [17 / 16] * 3
    # n3 fastest: the second point moves only along the third axis
    assert p[1].tolist() == [-17 / 16, -17 / 16, -16 / 16]
    assert p[35].tolist() == [-17 / 16, -16 / 16, -17 / 16]


def test_non_integer_interval_and_anisotropic_box():
    # M / 2d = 100 / 7 = 14.28 -> 15; 60 / 7 = 8.57 -> 9; 30 / 7 = 4.29 -> 5
    size, grid, d = (3.0, 1.5, 0.75), (100, 60, 30), 3.5
    assert [A.half_extent(m, d) for m in grid] == [15, 9, 5]
    p = A.points(size, grid, d).astype(np.float64)
    assert len(p) == 31 * 19 * 11 == A.count(size, grid, d)
    for ax, (s, m, k) in enumerate(zip(size, grid, (15, 9, 5))):
        vals = np.unique(p[:, ax])
        assert len(vals) == 2 * k + 1
        np.testing.assert_allclose(np.diff(vals), s * d / m, rtol=1e-6)
        assert abs(vals[0] + vals[-1]) < 1e-7          # symmetric about the origin
        assert np.any(vals == 0.0)                      # the centre is a sample
        # covering: the last sample lies beyond the face, the one before inside
        assert vals[-1] > s / 2 and vals[-2] <= s / 2 + 1e-7


def test_interval_wider_than_grid():
    # d > M / 2: [M / 2d] = 0, so the grid is the centre and one step each way
    p = A.points((1, 1, 1), (4, 4, 4), 3.0)
    assert len(p) == 27
    np.testing.assert_array_equal(np.unique(p[:, 0]), np.float32([-0.75, 0.0, 0.75]))


@pytest.mark.parametrize("grid,d", [((256, 256, 256), 8), ((64, 96, 32), 2.5), ((7, 9, 11), 1.0)])
def test_every_point_once_and_set_is_symmetric(grid, d):
    p = A.points((2.0, 1.0, 0.5), grid, d)
    assert len({tuple(x) for x in p.tolist()}) == len(p)
    fwd = {tuple(x) for x in p.tolist()}
    assert all((-a, -b, -c) in fwd for a, b, c in p.tolist())
