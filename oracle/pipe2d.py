"""2D particle-in-cell step in a rectangular perfectly conducting pipe, with
the sine-series Poisson solver (Sec. 4: the paper's own PIC instance),
every quantity a dual number.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Pipe [0, a] x [0, b] with phi = 0 on its walls, Nx x Ny cells, nodes
(i h_x, j h_y), i = 0..Nx, j = 0..Ny. The beam's transverse coordinates are
measured from the pipe centre (X = x + a/2, Y = y + b/2). Per step:

  M1(tau/2)  drift / quadrupole maps of (x, px) and (y, py) (Sec. 4);
  deposit    bilinear weights; a macroparticle carries lambda / N of the
             beam's line charge lambda = I / (beta0 c); node density
             rho_ij = (node charge per length) / (h_x h_y);
  solve      rho^lm = 4/(Nx Ny) sum_ij rho_ij sin(l pi i/Nx) sin(m pi j/Ny)
             over the interior nodes (the paper's projection integral by the
             trapezoid rule, wall terms vanish), phi^lm = rho^lm /
             (eps0 (alpha_l^2 + beta_m^2)), alpha_l = l pi / a,
             beta_m = m pi / b, and phi_ij = sum_lm phi^lm sin sin;
  field      central differences on every node; beyond a wall the sine
             series is odd, phi_{-1} = -phi_1 and phi_{N+1} = -phi_{N-1};
  gather     the deposit's weights;
  kick       Delta(px/p0) = tau q E_x / (m c^2 beta0^2 gamma0^3), likewise y:
             the lab field of a long beam with the magnetic force folded in
             (1 - beta0^2 = 1/gamma0^2). For a uniform round beam of radius
             r0 this is x'' = K x / r0^2 with the paper's perveance
             K = q I / (2 pi eps0 p0 v0^2 gamma0^2);
  M1(tau/2).

A particle is inside iff 0 <= X/h_x < Nx and 0 <= Y/h_y < Ny; others
deposit nothing, feel no kick and are counted.

Pins (tests/test_oracle_pipe2d.py): a single sine mode is solved exactly;
the explicit sine sums against scipy's type-I discrete sine transform;
zero current against the closed-form transfer matrices; a uniform round
beam's field against the perveance kick; mirror symmetry; the run's
derivatives against central differences.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

from . import lattice, physics
from .dual import Dual

COORDS4 = ("x", "px", "y", "py")


@dataclasses.dataclass
class Pipe:
    a: float
    b: float
    nx: int   # cells
    ny: int

    @property
    def hx(self):
        return self.a / self.nx

    @property
    def hy(self):
        return self.b / self.ny


def sine_matrix(n: int) -> np.ndarray:
    """S[l-1][i-1] = sin(l pi i / n) for l, i = 1..n-1."""
    k = np.arange(1, n)
    return np.sin(np.pi * np.outer(k, k) / n)


def solve(rho: np.ndarray, pipe: Pipe) -> np.ndarray:
    """rho [Nx+1][Ny+1][ch] node densities -> phi [Nx+1][Ny+1][ch] (walls 0)."""
    Sx, Sy = sine_matrix(pipe.nx), sine_matrix(pipe.ny)
    inner = rho[1:-1, 1:-1, :]
    # the double sums as matrix products (the library's contraction order)
    coef = 4.0 / (pipe.nx * pipe.ny) * np.einsum("li,ijc,mj->lmc", Sx, inner, Sy, optimize=True)
    al = np.arange(1, pipe.nx) * np.pi / pipe.a
    be = np.arange(1, pipe.ny) * np.pi / pipe.b
    g2 = al[:, None] ** 2 + be[None, :] ** 2
    phic = coef / (physics.EPS0 * g2[:, :, None])
    phi = np.zeros_like(rho)
    phi[1:-1, 1:-1, :] = np.einsum("li,lmc,mj->ijc", Sx, phic, Sy, optimize=True)
    return phi


def field(phi: np.ndarray, pipe: Pipe) -> np.ndarray:
    """E [2][Nx+1][Ny+1][ch] by central differences with odd reflection at the walls."""
    ext = np.zeros((phi.shape[0] + 2, phi.shape[1] + 2, phi.shape[2]))
    ext[1:-1, 1:-1] = phi
    ext[0, 1:-1] = -phi[1]
    ext[-1, 1:-1] = -phi[-2]
    ext[1:-1, 0] = -phi[:, 1]
    ext[1:-1, -1] = -phi[:, -2]
    Ex = -(ext[2:, 1:-1] - ext[:-2, 1:-1]) / (2 * pipe.hx)
    Ey = -(ext[1:-1, 2:] - ext[1:-1, :-2]) / (2 * pipe.hy)
    return np.stack([Ex, Ey])


@dataclasses.dataclass
class Weights:
    sel: np.ndarray
    ix: np.ndarray
    iy: np.ndarray
    wx: tuple
    wy: tuple
    n_outside: int


def weights(st, pipe: Pipe) -> Weights:
    sx = (st["x"].v + 0.5 * pipe.a) / pipe.hx
    sy = (st["y"].v + 0.5 * pipe.b) / pipe.hy
    inside = (sx >= 0) & (sx < pipe.nx) & (sy >= 0) & (sy < pipe.ny)
    sel = np.nonzero(inside)[0]
    ix, iy = np.floor(sx[sel]), np.floor(sy[sel])
    fx = (st["x"][sel] + 0.5 * pipe.a) / pipe.hx - ix
    fy = (st["y"][sel] + 0.5 * pipe.b) / pipe.hy - iy
    return Weights(sel, ix.astype(np.int64), iy.astype(np.int64), (1.0 - fx, fx), (1.0 - fy, fy),
                   int((~inside).sum()))


def deposit(w: Weights, pipe: Pipe, q_line: float, ntan: int) -> np.ndarray:
    rho = np.zeros((pipe.nx + 1, pipe.ny + 1, 1 + ntan))
    for a, wx in ((0, w.wx[0]), (1, w.wx[1])):
        for b, wy in ((0, w.wy[0]), (1, w.wy[1])):
            np.add.at(rho, (w.ix + a, w.iy + b), (wx * wy * q_line).a)
    return rho / (pipe.hx * pipe.hy)


def gather(E: np.ndarray, w: Weights):
    out = []
    for comp in range(2):
        acc = None
        for a, wx in ((0, w.wx[0]), (1, w.wx[1])):
            for b, wy in ((0, w.wy[0]), (1, w.wy[1])):
                t = wx * wy * Dual(E[comp][w.ix + a, w.iy + b])
                acc = t if acc is None else acc + t
        out.append(acc)
    return out


def kick_coefficient(kinetic_eV: float, rest_eV: float, charge_e: float) -> float:
    gamma0, beta0 = physics.gamma_beta(kinetic_eV, rest_eV)
    return (charge_e / rest_eV) / (beta0 * beta0 * gamma0 ** 3)


def half_map(st, em: lattice.ElementMap) -> None:
    (a, b), (c, d) = em.ax
    x, px = st["x"], st["px"]
    st["x"], st["px"] = a * x + b * px, c * x + d * px
    (a, b), (c, d) = em.ay
    y, py = st["y"], st["py"]
    st["y"], st["py"] = a * y + b * py, c * y + d * py


def moments(st) -> np.ndarray:
    """[2][3][1+ntan]: <u^2>, <u p>, <p^2> per plane (raw 1/N sums, Sec. 4)."""
    n = st["x"].v.shape[0]
    out = []
    for u, p in (("x", "px"), ("y", "py")):
        U, P = st[u], st[p]
        out.append([(U * U).sum() * (1.0 / n), (U * P).sum() * (1.0 / n), (P * P).sum() * (1.0 / n)])
    return np.array([[m.a for m in row] for row in out])


def emittance(mom: np.ndarray) -> np.ndarray:
    res = []
    for pl in range(2):
        uu, up, pp = (Dual(mom[pl, k]) for k in range(3))
        res.append((uu * pp - up * up).sqrt().a)
    return np.array(res)


@dataclasses.dataclass
class Result2:
    particles: np.ndarray   # [N][4][1+ntan]
    emittance: np.ndarray   # [2][1+ntan]
    lost: int               # particle-steps outside the pipe at deposit


def simulate(xi, sigma, sigma_seed, params, param_seed, lat, pipe: Pipe, kinetic_eV, rest_eV, charge_e,
             current_A: float, ntan: int, nsteps: Optional[int] = None) -> Result2:
    gamma0, beta0 = physics.gamma_beta(kinetic_eV, rest_eV)
    kap = kick_coefficient(kinetic_eV, rest_eV, charge_e)
    param_seed = np.asarray(param_seed, dtype=np.float64).reshape(len(params), ntan)
    maps = lattice.build_maps(lat, params, param_seed, gamma0)
    sched = lattice.schedule(lat)
    nsteps = len(sched) if nsteps is None else nsteps
    n = xi.shape[0]
    q_line = current_A / (beta0 * physics.C_LIGHT) / n
    st = {}
    for j, name in enumerate(COORDS4):
        row = sigma_seed[j] if sigma_seed is not None else np.zeros(ntan)
        st[name] = Dual.seeded(sigma[j], row) * xi[:, j]
    lost = 0
    for s in range(nsteps):
        em = maps[sched[s]]
        half_map(st, em)
        w = weights(st, pipe)
        lost += w.n_outside
        if current_A != 0.0:
            rho = deposit(w, pipe, q_line, ntan)
            E = field(solve(rho, pipe), pipe)
            ex, ey = gather(E, w)
            for name, e in (("px", ex), ("py", ey)):
                cur = st[name]
                upd = cur[w.sel] + em.tau * (e * kap)
                a = cur.a.copy()
                a[w.sel] = upd.a
                st[name] = Dual(a)
        half_map(st, em)
    parts = np.stack([st[c].a for c in COORDS4], axis=1)
    return Result2(particles=parts, emittance=emittance(moments(st)), lost=lost)
