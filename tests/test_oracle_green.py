"""Pins of the oracle's Green's function."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import green
from oracle.physics import EPS0


@pytest.mark.parametrize("a,b,c", [(0.5, 0.5, 0.5), (0.5, 0.5, 1.0), (0.3, 0.7, 1.1)])
def test_box_integral_against_cubature(a, b, c):
    num = integrate.tplquad(lambda z, y, x: 1.0 / math.sqrt(x * x + y * y + z * z),
                            0, a, 0, b, 0, c, epsabs=1e-13, epsrel=1e-12)[0]
    assert green.box_integral_inv_r(a, b, c) == pytest.approx(num, rel=1e-11)


def test_unit_cube_mean_inverse_distance():
    # potential at the centre of a uniformly charged unit cube, in units of
    # charge / (4 pi eps0 side): 2.38007736...
    assert green.mean_inv_r_cell(1.0, 1.0, 1.0) == pytest.approx(2.3800773639795, rel=1e-12)
    assert green.mean_inv_r_cell(2.0, 2.0, 2.0) == pytest.approx(2.3800773639795 / 2, rel=1e-12)


def test_offsets_even_and_coulomb():
    n, h, g0 = (4, 5, 3), (1e-4, 2e-4, 3e-4), 2.0
    G = green.green_offsets(n, h, g0)
    assert G.shape == (9, 11, 7)
    np.testing.assert_array_equal(G, G[::-1, :, :])
    np.testing.assert_array_equal(G, G[:, ::-1, :])
    np.testing.assert_array_equal(G, G[:, :, ::-1])
    # offset (1, -2, 3): rest-frame distance stretches z by gamma0
    r = math.sqrt((1 * h[0]) ** 2 + (2 * h[1]) ** 2 + (g0 * 3 * h[2]) ** 2)
    assert G[4 + 1, 5 - 2, 3 + 3] == pytest.approx(1 / (4 * math.pi * EPS0 * r), rel=1e-15)
    # self term: cell-averaged, finite, larger than any neighbour
    assert G[4, 5, 3] == pytest.approx(
        green.mean_inv_r_cell(h[0], h[1], g0 * h[2]) / (4 * math.pi * EPS0), rel=1e-15)
    # for a cubic rest-frame cell the self term is 2.38 times the nearest neighbour
    Gc = green.green_offsets((2, 2, 2), (1e-4, 1e-4, 0.5e-4), 2.0)
    assert Gc[2, 2, 2] / Gc[3, 2, 2] == pytest.approx(2.3800773639795, rel=1e-12)
