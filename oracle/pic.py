"""Forward-mode differentiable 3D PIC space-charge step (Sec. 4), plain FP64.

One step of the second-order split-operator integrator (Sec. 4, the map
M(tau) = M1(tau/2) M2(tau) M1(tau/2)) with every particle coordinate, grid
charge, potential and field value a dual number:

  1. M1(tau/2): half-step external map of the current element;
  2. deposit: cloud-in-cell (trilinear) charge of every macroparticle on the
     nodes of a fixed box; value and every derivative channel deposited;
  3. solve: open-boundary potential phi(i) = sum_j Q(j) G(i - j) on the nodes
     and one ghost ring around them, each channel solved independently
     (Sec. 4 solves the derivative arrays of D rho as well as its value);
  4. field: central finite differences of phi (Sec. 4); the z component is
     the rest-frame field, -(1/gamma0) d phi / d z_lab;
  5. gather with the deposit's CIC weights, then the space-charge kick
     p <- p + tau kappa E (Sec. 4, map M2, in the units of physics.py);
  6. M1(tau/2) again.

Emittances follow Sec. 4: eps = sqrt(<x^2><px^2> - <x px>^2) with raw
(uncentred) 1/N sums over all particles, as dual numbers.

Readings of points the paper leaves open (all listed in the design notes):
  * grid: n nodes per dimension at lo + i h, h = (hi - lo)/(n - 1), fixed per
    run and never differentiated; a particle is inside iff
    0 <= (u - lo)/h < n - 1 in every dimension, its cell is floor((u-lo)/h);
    a particle outside gets no deposit and no kick and is counted;
  * node charges are charges (C), not densities; the potential is
    sum_j Q_j G(i - j) with G from green.py;
  * the potential is needed on node indices -1..n per dimension so that the
    central difference is defined on every node; those ghost values are
    exact aperiodic sums, not boundary conditions.

The convolution is evaluated with scipy.signal.fftconvolve of the node
charges with G tabulated on every offset -n..n (a library routine for the
plain aperiodic sum), then sliced to targets -1..n.

This module is test infrastructure: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it; the HIP library never does.

Pins: tests/test_oracle_pic.py (brute-force convolution on tiny grids, charge
conservation, zero total space-charge momentum for value and every
derivative, zero self-force, mirror symmetry, pairwise Coulomb fields of
sparse beams); tests/test_oracle_kick.py (the kick as the step applies it:
one whole step of sparse charges and of a Gaussian bunch against the
lab-frame Lorentz force of the moving charges, which fixes the coefficient of
each momentum, the full step tau, the sign and the step-size tangent; the
centred emittance against numpy's covariance determinant, shift invariance
and the raw form of a zero-mean beam); tests/test_oracle_lattice.py
(zero-current closed forms); tests/test_oracle_fd.py (central finite
differences of the full run).
"""
from __future__ import annotations

import dataclasses
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.fft
from scipy import signal

from . import green, lattice, physics
from .dual import Dual

COORDS = ("x", "px", "y", "py", "z", "d")

# Threads given to the library FFTs inside the convolution (the rest of the
# oracle is single-threaded numpy).
FFT_WORKERS = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 1


@dataclasses.dataclass
class Grid:
    n: tuple
    lo: np.ndarray
    hi: np.ndarray

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        self.lo = np.asarray(self.lo, dtype=np.float64)
        self.hi = np.asarray(self.hi, dtype=np.float64)

    @property
    def h(self) -> np.ndarray:
        return (self.hi - self.lo) / (np.asarray(self.n, dtype=np.float64) - 1.0)


@dataclasses.dataclass
class CIC:
    """Cell indices and dual weights of the inside particles (sel)."""
    sel: np.ndarray
    idx: tuple            # (ix, iy, iz) of the lower corner, inside particles only
    w: tuple              # ((wx0, wx1), (wy0, wy1), (wz0, wz1)) duals
    n_outside: int


# ---------------------------------------------------------------------------
# particle state
# ---------------------------------------------------------------------------
def initial_state(xi: np.ndarray, sigma: Sequence[float], sigma_seed: Optional[np.ndarray],
                  ntan: int) -> Dict[str, Dual]:
    """zeta_j = sigma_j xi_j; sigma_j is a dual whose derivatives are its seed row."""
    st = {}
    for j, name in enumerate(COORDS):
        row = sigma_seed[j] if sigma_seed is not None else np.zeros(ntan)
        s = Dual.seeded(sigma[j], row)
        st[name] = s * xi[:, j]
    return st


def state_array(st: Dict[str, Dual]) -> np.ndarray:
    """(N, 6, 1+ntan) array in coordinate order x, px, y, py, z, delta."""
    return np.stack([st[c].a for c in COORDS], axis=1)


def half_map(st: Dict[str, Dual], em: lattice.ElementMap) -> None:
    """Apply M1(tau/2) of one element in place."""
    (a, b), (c, d) = em.ax
    x, px = st["x"], st["px"]
    st["x"], st["px"] = a * x + b * px, c * x + d * px
    (a, b), (c, d) = em.ay
    y, py = st["y"], st["py"]
    st["y"], st["py"] = a * y + b * py, c * y + d * py
    st["z"] = st["z"] + em.slip * st["d"]


# ---------------------------------------------------------------------------
# deposit / solve / field / gather
# ---------------------------------------------------------------------------
def cic_weights(st: Dict[str, Dual], grid: Grid) -> CIC:
    h = grid.h
    idx, frac = [], []
    inside = np.ones(st["x"].v.shape, dtype=bool)
    for dim, name in enumerate(("x", "y", "z")):
        u = st[name]
        s = (u.v - grid.lo[dim]) / h[dim]
        inside &= (s >= 0.0) & (s < grid.n[dim] - 1)
        idx.append(s)
    sel = np.nonzero(inside)[0]
    w = []
    cells = []
    for dim, name in enumerate(("x", "y", "z")):
        u = st[name][sel]
        i = np.floor(idx[dim][sel])
        f = (u - grid.lo[dim]) / h[dim] - i
        cells.append(i.astype(np.int64))
        w.append((1.0 - f, f))
    return CIC(sel=sel, idx=tuple(cells), w=tuple(w), n_outside=int((~inside).sum()))


def deposit(cic: CIC, grid: Grid, q_macro: float, ntan: int) -> np.ndarray:
    """Node charges rho[ix, iy, iz, channel] (C), channel 0 the value."""
    rho = np.zeros(grid.n + (1 + ntan,))
    ix, iy, iz = cic.idx
    (wx0, wx1), (wy0, wy1), (wz0, wz1) = cic.w
    for a, wx in ((0, wx0), (1, wx1)):
        for b, wy in ((0, wy0), (1, wy1)):
            for c, wz in ((0, wz0), (1, wz1)):
                w = wx * wy * wz
                np.add.at(rho, (ix + a, iy + b, iz + c), (w * q_macro).a)
    return rho


def solve(rho: np.ndarray, G: np.ndarray) -> np.ndarray:
    """phi on node indices -1..n per dimension: phi[i+1] = sum_j rho[j] G(i - j)."""
    nx, ny, nz = rho.shape[:3]
    with scipy.fft.set_workers(FFT_WORKERS):
        # every channel is convolved with the same G (axis 3 is broadcast)
        full = signal.fftconvolve(rho, G[..., None], mode="full", axes=(0, 1, 2))
    return np.ascontiguousarray(full[nx - 1:2 * nx + 1, ny - 1:2 * ny + 1, nz - 1:2 * nz + 1])


def field(phi: np.ndarray, grid: Grid, gamma0: float) -> np.ndarray:
    """Rest-frame field E[comp, ix, iy, iz, channel] on the n^3 nodes."""
    hx, hy, hz = grid.h
    c = slice(1, -1)
    ex = -(phi[2:, c, c] - phi[:-2, c, c]) / (2.0 * hx)
    ey = -(phi[c, 2:, c] - phi[c, :-2, c]) / (2.0 * hy)
    ez = -(phi[c, c, 2:] - phi[c, c, :-2]) / (2.0 * hz * gamma0)
    return np.stack([ex, ey, ez], axis=0)


def gather(E: np.ndarray, cic: CIC) -> List[Dual]:
    """Field at the inside particles: sum over the 8 corners of w * E_node (duals)."""
    ix, iy, iz = cic.idx
    (wx0, wx1), (wy0, wy1), (wz0, wz1) = cic.w
    out = [None, None, None]
    for a, wx in ((0, wx0), (1, wx1)):
        for b, wy in ((0, wy0), (1, wy1)):
            for c, wz in ((0, wz0), (1, wz1)):
                w = wx * wy * wz
                for comp in range(3):
                    e_node = Dual(E[comp, ix + a, iy + b, iz + c])
                    t = w * e_node
                    out[comp] = t if out[comp] is None else out[comp] + t
    return out


def kick(st: Dict[str, Dual], cic: CIC, e_p: List[Dual], tau: Dual,
         kperp: float, kpar: float) -> None:
    """p <- p + tau kappa E for the inside particles (map M2)."""
    sel = cic.sel
    for name, comp, kap in (("px", 0, kperp), ("py", 1, kperp), ("d", 2, kpar)):
        dp = tau * (e_p[comp] * kap)
        a = st[name].a.copy()
        a[sel] += dp.a
        st[name] = Dual(a)


# ---------------------------------------------------------------------------
# moments and emittance
# ---------------------------------------------------------------------------
def moments(st: Dict[str, Dual]) -> np.ndarray:
    """[plane][m][channel]: m = <u^2>, <u p>, <p^2>, <u>, <p> over all particles."""
    n = st["x"].v.shape[0]
    out = []
    for u, p in (("x", "px"), ("y", "py"), ("z", "d")):
        U, P = st[u], st[p]
        out.append([((U * U).sum() / n).a, ((U * P).sum() / n).a, ((P * P).sum() / n).a,
                    (U.sum() / n).a, (P.sum() / n).a])
    return np.asarray(out)


def emittance(mom: np.ndarray, centred: bool = False) -> np.ndarray:
    """[plane][channel]: sqrt(<u^2><p^2> - <u p>^2) as duals (raw by default)."""
    out = []
    for pl in range(3):
        uu, up, pp, u, p = (Dual(mom[pl, m]) for m in range(5))
        if centred:
            uu = uu - u * u
            up = up - u * p
            pp = pp - p * p
        out.append((uu * pp - up * up).sqrt().a)
    return np.asarray(out)


# ---------------------------------------------------------------------------
# full run
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Result:
    particles: np.ndarray      # (N, 6, 1+ntan)
    moments: np.ndarray        # (3, 5, 1+ntan)
    emittance: np.ndarray      # (3, 1+ntan) raw
    out_of_box: int            # particle-steps found outside the box at deposit
    max_extent: np.ndarray     # (3,) max |u| over particles and steps at deposit
    steps: int


def simulate(xi, sigma, sigma_seed, params, param_seed, lat, grid_n, lo, hi,
             kinetic_eV, rest_eV, charge_e, bunch_charge_C, ntan: int,
             nsteps: Optional[int] = None, history=None) -> Result:
    """Run nsteps (default: the whole lattice schedule) from the initial beam."""
    gamma0, _ = physics.gamma_beta(kinetic_eV, rest_eV)
    kperp, kpar = physics.kick_coefficients(kinetic_eV, rest_eV, charge_e)
    param_seed = np.asarray(param_seed, dtype=np.float64).reshape(len(params), ntan)
    maps = lattice.build_maps(lat, params, param_seed, gamma0)
    sched = lattice.schedule(lat)
    if nsteps is None:
        nsteps = len(sched)
    if nsteps > len(sched):
        raise ValueError("more steps than the lattice schedule holds")
    grid = Grid(grid_n, lo, hi)
    G = green.green_offsets(grid.n, grid.h, gamma0)
    n_part = xi.shape[0]
    q_macro = bunch_charge_C / n_part
    st = initial_state(xi, sigma, sigma_seed, ntan)
    outside = 0
    extent = np.zeros(3)
    for s in range(nsteps):
        em = maps[sched[s]]
        half_map(st, em)
        for dim, name in enumerate(("x", "y", "z")):
            extent[dim] = max(extent[dim], float(np.max(np.abs(st[name].v))))
        cic = cic_weights(st, grid)
        outside += cic.n_outside
        if q_macro != 0.0:
            rho = deposit(cic, grid, q_macro, ntan)
            phi = solve(rho, G)
            E = field(phi, grid, gamma0)
            e_p = gather(E, cic)
            kick(st, cic, e_p, em.tau, kperp, kpar)
        half_map(st, em)
        if history is not None:
            history.append(moments(st))
    mom = moments(st)
    return Result(particles=state_array(st), moments=mom, emittance=emittance(mom),
                  out_of_box=outside, max_extent=extent, steps=nsteps)


def simulate_workload(w, nsteps: Optional[int] = None, params=None, history=None,
                      xi=None) -> Result:
    """Convenience wrapper taking a workload description (plain data)."""
    p = tuple(w.params if params is None else params)
    return simulate(
        xi=w.xi() if xi is None else xi, sigma=w.sigma, sigma_seed=w.sigma_seed(),
        params=p, param_seed=w.param_seed(), lat=w.lattice, grid_n=w.grid, lo=w.lo,
        hi=w.hi, kinetic_eV=w.kinetic_eV, rest_eV=w.rest_eV, charge_e=w.charge_e,
        bunch_charge_C=w.bunch_charge_C, ntan=w.ntan, nsteps=nsteps, history=history)
