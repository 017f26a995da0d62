"""Open-boundary point Green's function on the PIC grid.

The paper solves the 2D Poisson equation inside a conducting pipe with a sine
expansion (Sec. 4). The 3D open-boundary instance built here uses the
rest-frame Coulomb potential of a point charge: a node charge Q at offset
o = (ox, oy, oz) (in grid cells) produces

    phi = Q G(o),   G(o) = 1 / (4 pi eps0 sqrt((ox hx)^2 + (oy hy)^2 + (gamma0 oz hz)^2))

because lab-frame lengths along z are gamma0 times longer in the beam rest
frame. At o = 0 the point kernel is singular; the reading used here replaces
it by the mean of 1/r over the rest-frame cell hx * hy * (gamma0 hz) centred
on the node, evaluated with the closed-form antiderivative of 1/r.

Pins: tests/test_oracle_green.py (self term against numerical cubature of
1/r; 2.3800773640 / h for a cube; evenness; Coulomb values at offsets).
"""
from __future__ import annotations

import math

import numpy as np

from .physics import EPS0


def _antiderivative(x: float, y: float, z: float) -> float:
    """F with d^3F/dx dy dz = 1/r, vanishing terms dropped where a coordinate is 0."""
    r = math.sqrt(x * x + y * y + z * z)
    t = 0.0
    if y > 0 and z > 0:
        t += y * z * math.log(x + r)
    if x > 0 and z > 0:
        t += x * z * math.log(y + r)
    if x > 0 and y > 0:
        t += x * y * math.log(z + r)
    if x > 0:
        t -= 0.5 * x * x * math.atan(y * z / (x * r))
    if y > 0:
        t -= 0.5 * y * y * math.atan(x * z / (y * r))
    if z > 0:
        t -= 0.5 * z * z * math.atan(x * y / (z * r))
    return t


def box_integral_inv_r(a: float, b: float, c: float) -> float:
    """Integral of 1/r over [0,a] x [0,b] x [0,c] (inclusion-exclusion over corners)."""
    s = 0.0
    for x, sx in ((a, 1), (0.0, -1)):
        for y, sy in ((b, 1), (0.0, -1)):
            for z, sz in ((c, 1), (0.0, -1)):
                s += sx * sy * sz * _antiderivative(x, y, z)
    return s


def mean_inv_r_cell(hx: float, hy: float, hz: float) -> float:
    """Mean of 1/r over the box [-hx/2,hx/2] x [-hy/2,hy/2] x [-hz/2,hz/2]."""
    octant = box_integral_inv_r(0.5 * hx, 0.5 * hy, 0.5 * hz)
    return 8.0 * octant / (hx * hy * hz)


def self_term(h, gamma0: float) -> float:
    """G(0): (1/4 pi eps0) <1/r> over the rest-frame cell."""
    hx, hy, hz = h
    return mean_inv_r_cell(hx, hy, gamma0 * hz) / (4.0 * math.pi * EPS0)


def green_offsets(n, h, gamma0: float) -> np.ndarray:
    """G on all offsets -n_d..n_d per dimension, shape (2nx+1, 2ny+1, 2nz+1).

    Array index m along a dimension holds offset m - n_d.
    """
    nx, ny, nz = n
    hx, hy, hz = h
    ox = np.arange(-nx, nx + 1, dtype=np.float64)[:, None, None] * hx
    oy = np.arange(-ny, ny + 1, dtype=np.float64)[None, :, None] * hy
    oz = np.arange(-nz, nz + 1, dtype=np.float64)[None, None, :] * (gamma0 * hz)
    r = np.sqrt(ox * ox + oy * oy + oz * oz)
    with np.errstate(divide="ignore"):
        G = 1.0 / (4.0 * math.pi * EPS0 * r)
    G[nx, ny, nz] = self_term(h, gamma0)
    return G
