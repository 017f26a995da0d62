"""Lattice elements, step sizes and half-step external maps (Sec. 4).

The external Hamiltonian H1 = p^2/2 + q psi(r) is integrated exactly over half
a step. For a drift (psi = 0) that is x += (tau/2) px. For a hard-edge
quadrupole of normalised strength k the focusing plane uses the cos/sin map
and the defocusing plane the cosh/sinh map given in Sec. 4. In the dual form
of the map, Dk carries the strength's derivatives and Dtau = L / n_steps the
length's (Sec. 4, the AD form of the quadrupole map).

Readings of points the paper leaves open:
  * k > 0 focuses x and defocuses y; k < 0 the reverse. The y plane sees -k.
  * The number of steps per element is a fixed integer, so dtau/dL = 1/n.
  * The paper's maps are 2D. The longitudinal coordinate z (lab-frame
    distance from the bunch centre) slips as dz/ds = delta / gamma0^2 in every
    element; delta is unchanged by the external maps.
  * For |k| (tau/2)^2 < 1e-8 the trigonometric forms are replaced by their
    Taylor series in u = k (tau/2)^2 up to u^3, which covers both signs.

Pins: tests/test_oracle_lattice.py (zero-current tracking equals the product
of closed-form element matrices; derivatives against complex-step
differentiation of those closed forms; det = 1; series branch against the
trigonometric branch).
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

from .dual import Dual

DRIFT = 0
QUAD = 1
SERIES_THRESHOLD = 1e-8

Map2 = Tuple[Tuple[Dual, Dual], Tuple[Dual, Dual]]


@dataclasses.dataclass
class ElementMap:
    tau: Dual        # full step length L / n_steps
    ax: Map2         # half-step map of (x, px)
    ay: Map2         # half-step map of (y, py)
    slip: Dual       # z += slip * delta per half step, slip = (tau/2) / gamma0^2


def element_strengths(kind: int, L_fixed: float, k_fixed: float, L_param: int,
                      k_param: int, params: Sequence[float], seed: np.ndarray):
    """Element length and strength as duals.

    A parameter-bound quantity takes the parameter's value and its seed row
    (the derivative of that parameter with respect to each tangent); a fixed
    one has zero derivatives.
    """
    n = seed.shape[1]
    L = (Dual.seeded(params[L_param], seed[L_param]) if L_param >= 0
         else Dual.const(L_fixed, n))
    if kind == QUAD:
        k = (Dual.seeded(params[k_param], seed[k_param]) if k_param >= 0
             else Dual.const(k_fixed, n))
    else:
        k = Dual.const(0.0, n)
    return L, k


def plane_map(kk: Dual, s: Dual) -> Map2:
    """Exact map of a plane with signed focusing strength kk over length s."""
    u = kk * s * s
    if abs(float(u.v)) < SERIES_THRESHOLD:
        c = 1.0 - u * 0.5 + u * u * (1.0 / 24.0) - u * u * u * (1.0 / 720.0)
        sn = s * (1.0 - u * (1.0 / 6.0) + u * u * (1.0 / 120.0) - u * u * u * (1.0 / 5040.0))
        return ((c, sn), (-(kk * sn), c))
    if kk.v > 0:
        r = kk.sqrt()
        th = r * s
        return ((th.cos(), th.sin() / r), (-(r * th.sin()), th.cos()))
    r = (-kk).sqrt()
    th = r * s
    return ((th.cosh(), th.sinh() / r), (r * th.sinh(), th.cosh()))


def element_map(kind: int, L: Dual, k: Dual, n_steps: int, gamma0: float) -> ElementMap:
    tau = L / float(n_steps)
    s = tau * 0.5
    one = Dual.const(1.0, L.n)
    zero = Dual.const(0.0, L.n)
    if kind == DRIFT:
        ax = ((one, s), (zero, one))
        ay = ax
    elif kind == QUAD:
        ax = plane_map(k, s)
        ay = plane_map(-k, s)
    else:
        raise ValueError(f"unknown element kind {kind}")
    slip = s * (1.0 / (gamma0 * gamma0))
    return ElementMap(tau=tau, ax=ax, ay=ay, slip=slip)


def build_maps(lat, params: Sequence[float], seed: np.ndarray, gamma0: float) -> List[ElementMap]:
    """One ElementMap per element of the period (shared by all periods)."""
    maps = []
    for e in range(len(lat.kind)):
        L, k = element_strengths(lat.kind[e], lat.L[e], lat.k[e], lat.L_param[e],
                                 lat.k_param[e], params, seed)
        maps.append(element_map(lat.kind[e], L, k, lat.n_steps[e], gamma0))
    return maps


def schedule(lat) -> List[int]:
    """Element index of every step, periods repeated in order."""
    out = []
    for _ in range(lat.n_periods):
        for e in range(len(lat.kind)):
            out.extend([e] * int(lat.n_steps[e]))
    return out
