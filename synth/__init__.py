"""Seeded synthetic workloads for the differentiable 3D PIC space-charge step.

This module only *describes* inputs: beam, lattice, grid box, parameter
vector and the standard-normal draws that seed the initial particle cloud.
It holds none of the method's arithmetic (no maps, deposition, field solve
or moments), so both the CPU oracle and the HIP library can be fed from it
without sharing any computation.

Input recipe (the paper's FODO example, extended to 3D, see the method
description in Sec. 4 and the lattice description in Sec. 3):

* protons at 1 GeV kinetic energy;
* an uncorrelated 6D Gaussian in (x, px/p0, y, py/p0, z, delta) with
  sigma = (1 mm, 1e-3, 1 mm, 1e-3, 2 mm, 1e-3); every draw is a standard
  normal truncated at |xi| <= 4 by resampling (numpy PCG64, seeded);
* one FODO cell drift-QF-drift-QD-drift with hard-edge quadrupoles of
  normalised strength +-22 m^-2 (the value the paper prints); the element
  lengths (0.1, 0.1, 0.2, 0.1, 0.1 m) are not printed in the paper and are
  this build's choice;
* 7 parameters in the paper's order: D1 L, Q1 L, Q1 k, D2 L, Q2 L, Q2 k,
  D3 L;
* the bunch charge follows from a peak current of a Gaussian bunch,
  Q = I * sqrt(2 pi) * sigma_z / (beta0 c).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "truncated_normals",
    "Lattice",
    "Workload",
    "fodo_lattice",
    "bunch_charge_from_peak_current",
    "peak_current_for_tune_depression",
    "NOMINAL_PARAMS",
    "PARAM_NAMES",
    "c1",
    "c2",
    "c4",
    "c5_inputs",
    "c5_base",
    "c5_batch",
    "tiny",
    "Batch",
    "perturbed_batch",
    "PipeWorkload",
    "pipe2d",
    "Matching",
    "matching",
]

# Recipe constants (CODATA 2018); used only to turn a peak current into a
# bunch charge for the workload description.
_E = 1.602176634e-19
_C = 299792458.0
_EPS0 = 8.8541878128e-12
PROTON_REST_EV = 938.27208816e6

PARAM_NAMES = ("D1 L", "Q1 L", "Q1 k", "D2 L", "Q2 L", "Q2 k", "D3 L")
NOMINAL_PARAMS = (0.1, 0.1, 22.0, 0.2, 0.1, -22.0, 0.1)
SIGMA_NOMINAL = (1e-3, 1e-3, 1e-3, 1e-3, 2e-3, 1e-3)

DRIFT = 0
QUAD = 1


def truncated_normals(n: int, seed: int, cut: float = 4.0, ncoord: int = 6) -> np.ndarray:
    """Standard normals of shape (n, ncoord), every entry with |xi| <= cut.

    Entries outside the cut are redrawn from the same PCG64 stream until none
    remain, so the array is a deterministic function of (n, seed, cut).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.standard_normal((n, ncoord))
    bad = np.abs(xi) > cut
    while bad.any():
        xi[bad] = rng.standard_normal(int(bad.sum()))
        bad = np.abs(xi) > cut
    return np.ascontiguousarray(xi, dtype=np.float64)


@dataclasses.dataclass
class Lattice:
    """Element list of one period; the period is repeated n_periods times.

    kind: 0 drift, 1 quadrupole. L and k are the fixed values used when the
    element's length / strength is not bound to a parameter (L_param or
    k_param = -1). Bound parameters are shared by every period.
    """

    kind: List[int]
    n_steps: List[int]
    L: List[float]
    k: List[float]
    L_param: List[int]
    k_param: List[int]
    n_periods: int = 1

    @property
    def n_elem(self) -> int:
        return len(self.kind)

    def total_steps(self) -> int:
        return int(sum(self.n_steps)) * int(self.n_periods)


def fodo_lattice(steps_per_element: int, n_periods: int,
                 params: Sequence[float] = NOMINAL_PARAMS) -> Lattice:
    """drift-QF-drift-QD-drift, every length and strength bound to a parameter."""
    p = list(params)
    return Lattice(
        kind=[DRIFT, QUAD, DRIFT, QUAD, DRIFT],
        n_steps=[steps_per_element] * 5,
        L=[p[0], p[1], p[3], p[4], p[6]],
        k=[0.0, p[2], 0.0, p[5], 0.0],
        L_param=[0, 1, 3, 4, 6],
        k_param=[-1, 2, -1, 5, -1],
        n_periods=n_periods,
    )


def _beta_gamma(kinetic_eV: float, rest_eV: float) -> Tuple[float, float]:
    g = 1.0 + kinetic_eV / rest_eV
    return math.sqrt(1.0 - 1.0 / (g * g)), g


def bunch_charge_from_peak_current(I_peak: float, sigma_z: float,
                                   kinetic_eV: float = 1e9,
                                   rest_eV: float = PROTON_REST_EV) -> float:
    """Charge of a Gaussian bunch with peak current I_peak and rms length sigma_z."""
    b, _ = _beta_gamma(kinetic_eV, rest_eV)
    return I_peak * math.sqrt(2.0 * math.pi) * sigma_z / (b * _C)


def peak_current_for_tune_depression(eta: float, sigma: float, emit: float,
                                     kinetic_eV: float = 1e9,
                                     rest_eV: float = PROTON_REST_EV) -> float:
    """Peak current giving tune ratio eta = nu/nu0 in the smooth-focusing rms
    envelope relation eta^2 = 1 / (1 + K sigma^2 / (4 emit^2)), with the
    generalised perveance K = 2 I / (I0 (beta gamma)^3), I0 = 4 pi eps0 m c^3 / e.
    """
    b, g = _beta_gamma(kinetic_eV, rest_eV)
    K = (1.0 / (eta * eta) - 1.0) * 4.0 * emit * emit / (sigma * sigma)
    I0 = 4.0 * math.pi * _EPS0 * (rest_eV * _E) * _C / _E  # m c^3 / e with m c^2 in J
    return 0.5 * K * I0 * (b * g) ** 3


@dataclasses.dataclass
class Workload:
    """Everything needed to run one differentiable PIC simulation."""

    name: str
    n_particles: int
    seed: int
    grid: Tuple[int, int, int]
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    lattice: Lattice
    params: Tuple[float, ...] = NOMINAL_PARAMS
    sigma: Tuple[float, ...] = SIGMA_NOMINAL
    ntan: int = 7
    sigma_tangents: bool = False  # tangents 7..12 are d/d sigma_j (13-tangent mode)
    kinetic_eV: float = 1e9
    rest_eV: float = PROTON_REST_EV
    charge_e: float = 1.0
    bunch_charge_C: float = 0.0

    # -- derived inputs (no method arithmetic) ---------------------------
    def xi(self) -> np.ndarray:
        return truncated_normals(self.n_particles, self.seed)

    def param_seed(self) -> np.ndarray:
        """[n_params][ntan]: parameter j carries tangent j (identity seeding)."""
        s = np.zeros((len(self.params), self.ntan))
        for j in range(min(len(self.params), self.ntan)):
            s[j, j] = 1.0
        return s

    def sigma_seed(self) -> Optional[np.ndarray]:
        """[6][ntan]: sigma_j carries tangent 7+j in 13-tangent mode, else None."""
        if not self.sigma_tangents:
            return None
        s = np.zeros((6, self.ntan))
        for j in range(6):
            s[j, len(self.params) + j] = 1.0
        return s

    def total_steps(self) -> int:
        return self.lattice.total_steps()

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# Boxes are fixed per run and symmetric about the origin. They contain every
# particle at every step of the nominal run (the out-of-box counters stay at
# zero): synth/box_prepass.py iterates value-only runs, box <- 1.1 x extent.
# c1 settles at extents (3.81, 6.63, 7.61) mm, recorded with extra margin for
# the +-5% parameter perturbations used elsewhere; c2 (strong space charge
# lengthens the bunch) settles at half-widths (13.87, 15.86, 29.62) mm.
C1_HALF = (4.6e-3, 8.0e-3, 9.2e-3)
C2_HALF = (14.0e-3, 16.0e-3, 30.0e-3)
# Batched workloads, from the batched pre-pass over all their settings:
# c4's 64 settings settle at half-widths (18.48, 21.91, 14.72) mm; 1024
# settings spanning the surrogate's +-5% input box at (4.79, 8.96, 9.48) mm,
# recorded with 5% more so that other draws from that box stay inside.
C4_HALF = (18.5e-3, 22.0e-3, 14.8e-3)
C5_HALF = (5.0e-3, 9.4e-3, 10.0e-3)


def c1(ntan: int = 7, **kw) -> Workload:
    """1e4 protons, 32^3 grid (64^3 doubled), one FODO cell, 100 steps, 100 A peak."""
    w = Workload(
        name="c1: 1e4 protons, 32^3 grid, 1 FODO cell, 100 steps, 100 A",
        n_particles=10_000,
        seed=20251121,
        grid=(32, 32, 32),
        lo=tuple(-h for h in C1_HALF),
        hi=C1_HALF,
        lattice=fodo_lattice(20, 1),
        ntan=ntan,
        bunch_charge_C=bunch_charge_from_peak_current(100.0, SIGMA_NOMINAL[4]),
    )
    return w.with_(**kw) if kw else w


def c2(**kw) -> Workload:
    """1e6 protons, 64^3 grid (128^3 doubled), 10 FODO cells, 2000 steps, tune ratio 0.3."""
    I = peak_current_for_tune_depression(0.3, 1e-3, 1e-6)
    w = Workload(
        name="c2: 1e6 protons, 64^3 grid, 10 FODO cells, 2000 steps, eta=0.3",
        n_particles=1_000_000,
        seed=20251122,
        grid=(64, 64, 64),
        lo=tuple(-h for h in C2_HALF),
        hi=C2_HALF,
        lattice=fodo_lattice(40, 10),
        ntan=7,
        bunch_charge_C=bunch_charge_from_peak_current(I, SIGMA_NOMINAL[4]),
    )
    return w.with_(**kw) if kw else w


def tiny(n_particles: int = 3001, grid: int = 16, steps_per_element: int = 4,
         ntan: int = 7, seed: int = 7, **kw) -> Workload:
    """Small case for fast parity: ragged particle count, coarse grid."""
    w = Workload(
        name=f"tiny: {n_particles} protons, {grid}^3 grid, {5 * steps_per_element} steps",
        n_particles=n_particles,
        seed=seed,
        grid=(grid, grid, grid),
        lo=tuple(-h for h in C1_HALF),
        hi=C1_HALF,
        lattice=fodo_lattice(steps_per_element, 1),
        ntan=ntan,
        bunch_charge_C=bunch_charge_from_peak_current(100.0, SIGMA_NOMINAL[4]),
    )
    return w.with_(**kw) if kw else w


# ---------------------------------------------------------------- batches
@dataclasses.dataclass
class Batch:
    """Settings that share grid, beam energy, bunch charge and lattice
    structure, each with its own parameters, beam sizes, particle count and
    normals (drawn with its own seed)."""

    base: Workload
    params: np.ndarray   # [B][7]
    sigma: np.ndarray    # [B][6]
    ns: np.ndarray       # [B] particles per setting
    seeds: np.ndarray    # [B] normal-draw seeds

    @property
    def nbatch(self) -> int:
        return len(self.ns)

    def setting(self, b: int) -> Workload:
        """Setting b as a single-run workload (same inputs)."""
        return self.base.with_(params=tuple(float(v) for v in self.params[b]),
                               sigma=tuple(float(v) for v in self.sigma[b]),
                               n_particles=int(self.ns[b]), seed=int(self.seeds[b]))

    def xi(self) -> np.ndarray:
        """Packed normals [sum ns][6]: setting b's rows follow those of 0..b-1."""
        parts = [truncated_normals(int(n), int(s)) for n, s in zip(self.ns, self.seeds)]
        return np.concatenate(parts, axis=0) if parts else np.zeros((0, 6))


def perturbed_batch(base: Workload, ns: Sequence[int], seed: int, rel: float = 0.05,
                    perturb_sigma: bool = False) -> Batch:
    """Parameters (and optionally beam sizes) uniform within +-rel of the
    base workload's, one seeded draw per setting."""
    rng = np.random.default_rng(seed)
    B = len(ns)
    p = np.asarray(base.params, dtype=np.float64)[None, :] * (1.0 + rng.uniform(-rel, rel, size=(B, len(base.params))))
    s = np.tile(np.asarray(base.sigma, dtype=np.float64), (B, 1))
    if perturb_sigma:
        s = s * (1.0 + rng.uniform(-rel, rel, size=(B, 6)))
    seeds = base.seed + 1000 + np.arange(B)
    return Batch(base=base, params=p, sigma=s, ns=np.asarray(ns, dtype=np.int64), seeds=seeds)


def c4(nbatch: int = 64, seed: int = 20251124, **kw) -> Batch:
    """64 settings of the 64^3-grid beam (tune ratio 0.3 bunch charge) over 5
    FODO cells (500 steps), parameters uniform within +-5% of nominal,
    particle counts log-uniform in [1e5, 1e6]."""
    rng = np.random.default_rng(seed)
    ns = np.rint(10.0 ** rng.uniform(5.0, 6.0, size=nbatch)).astype(np.int64)
    I = peak_current_for_tune_depression(0.3, 1e-3, 1e-6)
    base = Workload(
        name=f"c4: {nbatch} settings, 1e5-1e6 protons each, 64^3 grid, 5 FODO cells, 500 steps, eta=0.3",
        n_particles=int(ns.max()),
        seed=seed,
        grid=(64, 64, 64),
        lo=tuple(-h for h in C4_HALF),
        hi=C4_HALF,
        lattice=fodo_lattice(20, 5),
        ntan=7,
        bunch_charge_C=bunch_charge_from_peak_current(I, SIGMA_NOMINAL[4]),
    )
    base = base.with_(**kw) if kw else base
    return perturbed_batch(base, ns, seed + 1)


def c5_base(ntan: int = 13) -> Workload:
    """The surrogate's training run: the 1e4-particle, 32^3, 100-step
    workload on a box that holds every input of the +-5% box, with the 13
    inputs (7 lattice parameters, 6 beam sizes) as tangents."""
    return c1(ntan=ntan, sigma_tangents=ntan == 13, lo=tuple(-h for h in C5_HALF), hi=C5_HALF,
              name="c5: 1e4 protons, 32^3 grid, 1 FODO cell, 100 steps, 100 A, inputs +-5%")


def c5_batch(n_runs: int, seed: int = 20251125, ntan: int = 13) -> Batch:
    """n_runs settings of c5_base at inputs c5_inputs(n_runs, seed). Every
    run uses the same normals (common random numbers): the emittance is then
    one smooth function of the 13 inputs, whose PIC gradient is the exact
    derivative of the PIC values the surrogate fits."""
    base = c5_base(ntan)
    x = c5_inputs(n_runs, seed)
    return Batch(base=base, params=x[:, :7], sigma=x[:, 7:], ns=np.full(n_runs, base.n_particles, dtype=np.int64),
                 seeds=np.full(n_runs, base.seed, dtype=np.int64))


def c5_inputs(n_runs: int, seed: int = 20251125, rel: float = 0.05) -> np.ndarray:
    """[n_runs][13]: the 7 lattice parameters and 6 beam sizes, each uniform
    within +-rel of nominal (the surrogate's training and test inputs)."""
    rng = np.random.default_rng(seed)
    nominal = np.concatenate([NOMINAL_PARAMS, SIGMA_NOMINAL])
    return nominal[None, :] * (1.0 + rng.uniform(-rel, rel, size=(n_runs, 13)))


# ---------------------------------------------------------------- 2D pipe and matching
@dataclasses.dataclass
class PipeWorkload:
    """The paper's own PIC instance: a 2D beam in a rectangular conducting pipe."""
    name: str
    n_particles: int
    seed: int
    a: float
    b: float
    nx: int            # cells
    ny: int
    lattice: Lattice
    params: Tuple[float, ...] = NOMINAL_PARAMS
    sigma: Tuple[float, ...] = (1e-3, 1e-3, 1e-3, 1e-3)
    ntan: int = 7
    kinetic_eV: float = 1e9
    rest_eV: float = PROTON_REST_EV
    charge_e: float = 1.0
    current_A: float = 100.0

    def xi(self) -> np.ndarray:
        return truncated_normals(self.n_particles, self.seed, ncoord=4)

    def param_seed(self) -> np.ndarray:
        s = np.zeros((len(self.params), self.ntan))
        for j in range(min(len(self.params), self.ntan)):
            s[j, j] = 1.0
        return s

    def total_steps(self) -> int:
        return self.lattice.total_steps()

    def with_(self, **kw) -> "PipeWorkload":
        return dataclasses.replace(self, **kw)


def pipe2d(n_particles: int = 10_000, cells: int = 64, steps_per_element: int = 20, **kw) -> PipeWorkload:
    """1 GeV protons, 100 A, one FODO cell in a 20 mm x 20 mm pipe (the
    sensitivity study of the paper's PIC section)."""
    w = PipeWorkload(name=f"pipe2d: {n_particles} protons, {cells}^2 cells, 20 mm pipe, one FODO cell, 100 A",
                     n_particles=n_particles, seed=20251126, a=0.02, b=0.02, nx=cells, ny=cells,
                     lattice=fodo_lattice(steps_per_element, 1))
    return w.with_(**kw) if kw else w


@dataclasses.dataclass
class Matching:
    """Four-quadrupole matching section between two periodic FODO lattices
    (the paper's third example): start from the first lattice's matched
    Twiss, reach the second's. Lattice lengths and strengths are this
    build's choice (the paper prints only the +-22 m^-2 cell)."""
    kind: Tuple[int, ...]
    L: Tuple[float, ...]
    k_param: Tuple[int, ...]
    cell_from: Tuple[float, float]   # quad strengths of the first FODO
    cell_to: Tuple[float, float]     # and of the second
    k0: Tuple[float, ...]            # starting strengths of the four matching quads


def matching() -> Matching:
    return Matching(kind=(DRIFT, QUAD, DRIFT, QUAD, DRIFT, QUAD, DRIFT, QUAD, DRIFT),
                    L=(0.1, 0.1, 0.2, 0.1, 0.2, 0.1, 0.2, 0.1, 0.1),
                    k_param=(-1, 0, -1, 1, -1, 2, -1, 3, -1),
                    cell_from=(22.0, -22.0), cell_to=(16.0, -16.0), k0=(20.0, -20.0, 20.0, -20.0))
