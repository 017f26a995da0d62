"""Pins of the kick units: the oracle's rest-frame kick against the lab-frame
Lorentz force of a uniformly moving point charge.

A source charge moving with the reference velocity v0 along z has, at equal
lab time, the field E = q gamma r / (4 pi eps0 (x^2 + y^2 + gamma^2 z^2)^(3/2))
and B = v x E / c^2 (the textbook field of a uniformly moving charge). A test
particle moving with v0 feels F = q (E + v x B); dividing by p0 v0 gives the
change of the normalised momenta per unit path length. The oracle's
coefficients times the rest-frame Coulomb field at the rest-frame offset
(x, y, gamma z) must agree.
"""
import math

import numpy as np
import pytest

from oracle import physics
from oracle.physics import C_LIGHT, E_CHARGE, EPS0


@pytest.mark.parametrize("T", [1e9, 5e7, 2e10])
def test_kick_coefficients_match_lab_frame_lorentz_force(T):
    rest = physics.PROTON_REST_EV
    g, b = physics.gamma_beta(T, rest)
    kperp, kpar = physics.kick_coefficients(T, rest, 1.0)
    q = E_CHARGE
    qs = 3e-15
    for off in ([1e-3, 2e-3, 0.5e-3], [-2e-3, 0.1e-3, -1e-3]):
        x, y, z = off
        den = (x * x + y * y + g * g * z * z) ** 1.5
        E_lab = qs * g * np.array([x, y, z]) / (4 * math.pi * EPS0 * den)
        v = np.array([0, 0, b * C_LIGHT])
        B_lab = np.cross(v, E_lab) / C_LIGHT ** 2
        F = q * (E_lab + np.cross(v, B_lab))
        m = rest * E_CHARGE / C_LIGHT ** 2
        p0 = g * m * b * C_LIGHT
        dpds = F / (p0 * b * C_LIGHT)
        rr = np.array([x, y, g * z])
        E_rest = qs * rr / (4 * math.pi * EPS0 * np.linalg.norm(rr) ** 3)
        assert kperp * E_rest[0] == pytest.approx(dpds[0], rel=1e-12)
        assert kperp * E_rest[1] == pytest.approx(dpds[1], rel=1e-12)
        assert kpar * E_rest[2] == pytest.approx(dpds[2], rel=1e-12)


def test_long_beam_limit_gives_paper_perveance():
    # Inside a long uniform round beam of radius a and current I, the
    # rest-frame field is E = lambda_rest r / (2 pi eps0 a^2) with
    # lambda_rest = I / (beta0 c gamma0). The kick per unit length must be
    # K r / a^2 with the generalised perveance of Sec. 4,
    # K = q I / (2 pi eps0 p0 v0^2 gamma0^2).
    T, rest, I, a, r = 1e9, physics.PROTON_REST_EV, 100.0, 1e-3, 0.4e-3
    g, b = physics.gamma_beta(T, rest)
    kperp, _ = physics.kick_coefficients(T, rest, 1.0)
    lam = I / (b * C_LIGHT * g)
    E = lam * r / (2 * math.pi * EPS0 * a * a)
    m = rest * E_CHARGE / C_LIGHT ** 2
    p0 = g * m * b * C_LIGHT
    v0 = b * C_LIGHT
    K = E_CHARGE * I / (2 * math.pi * EPS0 * p0 * v0 ** 2 * g ** 2)
    assert kperp * E == pytest.approx(K * r / a ** 2, rel=1e-12)
