"""Single-particle linear optics: transfer matrices of a lattice, Twiss
parameters and their derivatives with respect to lattice parameters, and
the matching objective of the paper's third example (Sec. 3), minimised by
BFGS.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Twiss transport from 0 to s with the plane's transfer matrix m (Sec. 3):
    beta1  =  m11^2 beta0 - 2 m11 m12 alpha0 + m12^2 gamma0
    alpha1 = -m11 m21 beta0 + (m11 m22 + m12 m21) alpha0 - m12 m22 gamma0
    gamma  = (1 + alpha^2) / beta.
A periodic cell's matched Twiss follow from its one-cell matrix M:
cos mu = (M11 + M22)/2, beta = M12 / sin mu, alpha = (M11 - M22) / (2 sin mu).
Each element's matrix is its exact map over its full length (Sec. 4 maps).

Matching objective (Sec. 3):
    f(k) = (beta_x - beta_xt)^2 / beta_xt^2 + (alpha_x - alpha_xt)^2
         + (beta_y - beta_yt)^2 / beta_yt^2 + (alpha_y - alpha_yt)^2.

The optimiser is textbook BFGS with the inverse-Hessian update
H <- (I - r s y^T) H (I - r y s^T) + r s s^T, r = 1/(y^T s), and a
backtracking Armijo line search.

Pins (tests/test_oracle_twiss.py): Twiss transport against sigma-matrix
transport M Sigma M^T (a different route); the matched Twiss are invariant
over one cell; derivatives against central differences; BFGS on a quadratic
and on the Rosenbrock function.
"""
from __future__ import annotations

from typing import Callable, List, Sequence, Tuple

import numpy as np

from .dual import Dual
from . import lattice


def element_matrices(kind: int, L: Dual, k: Dual):
    """Full-length maps of one element for x and y."""
    one = Dual.const(1.0, L.n)
    zero = Dual.const(0.0, L.n)
    if kind == lattice.DRIFT:
        m = ((one, L), (zero, one))
        return m, m
    return lattice.plane_map(k, L), lattice.plane_map(-k, L)


def matmul2(A, B):
    return ((A[0][0] * B[0][0] + A[0][1] * B[1][0], A[0][0] * B[0][1] + A[0][1] * B[1][1]),
            (A[1][0] * B[0][0] + A[1][1] * B[1][0], A[1][0] * B[0][1] + A[1][1] * B[1][1]))


def line_matrices(kind, L_fixed, k_fixed, L_param, k_param, params, seed):
    """Transfer matrices (x, y) of a line of elements traversed in order."""
    n = seed.shape[1]
    one = Dual.const(1.0, n)
    zero = Dual.const(0.0, n)
    Mx = ((one, zero), (zero, one))
    My = Mx
    for e in range(len(kind)):
        L, k = lattice.element_strengths(kind[e], L_fixed[e], k_fixed[e], L_param[e], k_param[e], params, seed)
        ex, ey = element_matrices(kind[e], L, k)
        Mx = matmul2(ex, Mx)
        My = matmul2(ey, My)
    return Mx, My


def transport(m, beta0, alpha0):
    gamma0 = (1.0 + alpha0 * alpha0) / beta0
    (m11, m12), (m21, m22) = m
    beta1 = m11 * m11 * beta0 - m11 * m12 * alpha0 * 2.0 + m12 * m12 * gamma0
    alpha1 = -(m11 * m21 * beta0) + (m11 * m22 + m12 * m21) * alpha0 - m12 * m22 * gamma0
    return beta1, alpha1


def periodic(m):
    """Matched (beta, alpha) of a stable cell with one-cell matrix m."""
    (m11, m12), (m21, m22) = m
    cmu = (m11 + m22) * 0.5
    smu = (1.0 - cmu * cmu).sqrt()
    if float(m12.v) < 0:
        smu = -smu
    return m12 / smu, (m11 - m22) / (smu * 2.0)


def matching_objective(tw, target) -> Dual:
    bx, ax, by, ay = tw
    bxt, axt, byt, ayt = target
    return ((bx - bxt) * (bx - bxt) * (1.0 / bxt ** 2) + (ax - axt) * (ax - axt)
            + (by - byt) * (by - byt) * (1.0 / byt ** 2) + (ay - ayt) * (ay - ayt))


def bfgs(fg: Callable[[np.ndarray], Tuple[float, np.ndarray]], x0, tol=1e-12, max_iter=200):
    """Returns (x, f, evaluations, history of f per evaluation)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    n = x.size
    f, g = fg(x)
    hist = [f]
    H = np.eye(n)
    for _ in range(max_iter):
        if np.linalg.norm(g) < tol:
            break
        d = -H @ g
        if g @ d >= 0:  # not a descent direction: restart from steepest descent
            H = np.eye(n)
            d = -g
        t = 1.0
        while True:
            xn = x + t * d
            fn, gn = fg(xn)
            hist.append(fn)
            if fn <= f + 1e-4 * t * (g @ d) or t < 1e-12:
                break
            t *= 0.5
        s, y = xn - x, gn - g
        ys = y @ s
        if ys > 1e-300:
            r = 1.0 / ys
            I = np.eye(n)
            H = (I - r * np.outer(s, y)) @ H @ (I - r * np.outer(y, s)) + r * np.outer(s, s)
        x, f, g = xn, fn, gn
        if f < tol:
            break
    return x, f, len(hist), hist
