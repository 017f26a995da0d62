"""Physical constants, beam kinematics and space-charge kick coefficients.

The paper's kick (Sec. 4, the space-charge map that leaves r fixed and moves
p by -tau dH2/dr, with H2 = K phi / 2 and the 2D perveance K) is written for a
2D beam whose potential units do not close. This oracle uses the 3D reading:
the potential is the rest-frame electrostatic potential of the macroparticle
charges, the transverse lab force is q E_rest_perp / gamma0 and the
longitudinal one q E_rest_par; dividing the force by p0 v0 gives the change of
the normalised momenta per unit path length s:

  d(px/p0)/ds = q E_x^r / (m c^2 beta0^2 gamma0^2)
  d(delta)/ds = q E_z^r / (m c^2 beta0^2 gamma0)

For a long uniform beam this reproduces the paper's generalised perveance
K = q I / (2 pi eps0 p0 v0^2 gamma0^2) exactly (x'' = K x / a^2 inside a round
beam of radius a).

Pins: tests/test_oracle_physics.py (the coefficients against the lab-frame
Lorentz force of a uniformly moving point charge computed from its
Lorentz-transformed E and B fields; the long-beam limit against K).
"""
from __future__ import annotations

import math

E_CHARGE = 1.602176634e-19      # C
C_LIGHT = 299792458.0           # m/s
EPS0 = 8.8541878128e-12         # F/m
PROTON_REST_EV = 938.27208816e6  # eV


def gamma_beta(kinetic_eV: float, rest_eV: float):
    gamma0 = 1.0 + kinetic_eV / rest_eV
    beta0 = math.sqrt(1.0 - 1.0 / (gamma0 * gamma0))
    return gamma0, beta0


def kick_coefficients(kinetic_eV: float, rest_eV: float, charge_e: float):
    """(kappa_perp, kappa_par) in 1/V: Delta(p/p0) = tau * kappa * E_rest."""
    gamma0, beta0 = gamma_beta(kinetic_eV, rest_eV)
    # q / (m c^2) with q = charge_e * e and m c^2 = rest_eV * e
    q_over_mc2 = charge_e / rest_eV
    kperp = q_over_mc2 / (beta0 * beta0 * gamma0 * gamma0)
    kpar = q_over_mc2 / (beta0 * beta0 * gamma0)
    return kperp, kpar
