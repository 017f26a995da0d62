"""Pins of the oracle's external maps (Sec. 4 quadrupole and drift maps).

At zero beam current every step is linear, so tracking the whole cell with
2 n half-step dual maps per element must equal the product of the
closed-form full-element matrices; the derivatives with respect to the seven
lattice parameters must equal complex-step derivatives of that product, which
uses complex arithmetic only and no dual numbers. The emittance is invariant
(det M = 1), so its lattice derivatives vanish.
"""
import cmath
import math

import numpy as np
import pytest

import synth
from oracle import lattice, physics, pic
from oracle.dual import Dual


def _plane(kind, L, k):
    """Closed-form 2x2 map of a full element (complex-safe for complex step)."""
    if kind == 0 or k == 0:
        return np.array([[1, L], [0, 1]], dtype=complex)
    if k.real > 0:
        r = cmath.sqrt(k)
        return np.array([[cmath.cos(r * L), cmath.sin(r * L) / r],
                         [-r * cmath.sin(r * L), cmath.cos(r * L)]])
    r = cmath.sqrt(-k)
    return np.array([[cmath.cosh(r * L), cmath.sinh(r * L) / r],
                     [r * cmath.sinh(r * L), cmath.cosh(r * L)]])


def _cell_maps(p, periods=1):
    """(Mx, My, total length) of the FODO cell for parameter vector p."""
    D1, Q1L, Q1k, D2, Q2L, Q2k, D3 = p
    elems = [(0, D1, 0), (1, Q1L, Q1k), (0, D2, 0), (1, Q2L, Q2k), (0, D3, 0)]
    Mx = np.eye(2, dtype=complex)
    My = np.eye(2, dtype=complex)
    for _ in range(periods):
        for kind, L, k in elems:
            Mx = _plane(kind, L, k) @ Mx
            My = _plane(kind, L, -k) @ My
    total = periods * (D1 + Q1L + D2 + Q2L + D3)
    return Mx, My, total


def _zero_current(w):
    return pic.simulate_workload(w.with_(bunch_charge_C=0.0))


@pytest.mark.parametrize("periods,steps", [(1, 7), (2, 3)])
def test_zero_current_tracking_equals_closed_form(periods, steps):
    w = synth.tiny(n_particles=64, steps_per_element=steps)
    w = w.with_(lattice=synth.fodo_lattice(steps, periods))
    r = _zero_current(w)
    xi = w.xi()
    z0 = np.asarray(w.sigma)[None, :] * xi
    p = np.asarray(w.params, dtype=complex)
    Mx, My, total = _cell_maps(p, periods)
    g0, _ = physics.gamma_beta(w.kinetic_eV, w.rest_eV)
    fx = z0[:, 0:2] @ Mx.real.T
    fy = z0[:, 2:4] @ My.real.T
    fz = z0[:, 4] + total / g0 ** 2 * z0[:, 5]
    P = r.particles
    np.testing.assert_allclose(P[:, 0:2, 0], fx, rtol=1e-12, atol=1e-12 * np.abs(fx).max())
    np.testing.assert_allclose(P[:, 2:4, 0], fy, rtol=1e-12, atol=1e-12 * np.abs(fy).max())
    np.testing.assert_allclose(P[:, 4, 0], fz, rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(P[:, 5, 0], z0[:, 5])
    # derivatives: complex step on each parameter of the closed-form product
    h = 1e-30
    for j in range(7):
        pj = p.copy()
        pj[j] += 1j * h
        Mxj, Myj, totj = _cell_maps(pj, periods)
        dx = z0[:, 0:2] @ (Mxj.imag / h).T
        dy = z0[:, 2:4] @ (Myj.imag / h).T
        dz = (totj.imag / h) / g0 ** 2 * z0[:, 5]
        scale = max(np.abs(dx).max(), np.abs(dy).max(), 1e-30)
        np.testing.assert_allclose(P[:, 0:2, 1 + j], dx, atol=1e-11 * scale)
        np.testing.assert_allclose(P[:, 2:4, 1 + j], dy, atol=1e-11 * scale)
        np.testing.assert_allclose(P[:, 4, 1 + j], dz, atol=1e-13 * max(np.abs(dz).max(), 1e-30))


def test_zero_current_emittance_invariant_and_sigma_derivatives():
    w = synth.tiny(n_particles=500, steps_per_element=5, ntan=13, sigma_tangents=True)
    r = _zero_current(w)
    xi = w.xi()
    z0 = np.asarray(w.sigma)[None, :] * xi
    for pl in range(3):
        u, q = z0[:, 2 * pl], z0[:, 2 * pl + 1]
        e0 = math.sqrt(np.mean(u * u) * np.mean(q * q) - np.mean(u * q) ** 2)
        e = r.emittance[pl]
        assert e[0] == pytest.approx(e0, rel=1e-12)
        # lattice derivatives vanish (relative to eps / p)
        for j in range(7):
            assert abs(e[1 + j] * w.params[j]) < 1e-11 * e0
        # sigma derivatives: eps is proportional to sigma_u * sigma_p of its plane
        for j in range(6):
            expect = e0 / w.sigma[j] if j in (2 * pl, 2 * pl + 1) else 0.0
            assert e[8 + j] == pytest.approx(expect, rel=1e-11, abs=1e-12 * e0 / w.sigma[j])


def test_half_maps_have_unit_determinant():
    g0 = 2.0
    seed = np.eye(7)
    for kind, L, k in ((0, 0.2, 0.0), (1, 0.1, 22.0), (1, 0.1, -22.0)):
        Ld = Dual.seeded(L, seed[1])
        kd = Dual.seeded(k, seed[2])
        em = lattice.element_map(kind, Ld, kd, 13, g0)
        for m in (em.ax, em.ay):
            det = m[0][0] * m[1][1] - m[0][1] * m[1][0]
            assert det.v == pytest.approx(1.0, abs=1e-15)
            np.testing.assert_allclose(det.d, 0.0, atol=1e-13)


def test_series_branch_matches_trigonometric_form():
    s_val, kk_val = 0.005, 2e-4  # u = kk s^2 = 5e-9, below the series threshold
    s = Dual.seeded(s_val, [1.0, 0.0])
    kk = Dual.seeded(kk_val, [0.0, 1.0])
    m = lattice.plane_map(kk, s)

    def trig(sv, kv):
        r = cmath.sqrt(kv)
        return np.array([[cmath.cos(r * sv), cmath.sin(r * sv) / r],
                         [-r * cmath.sin(r * sv), cmath.cos(r * sv)]])

    ref = trig(complex(s_val), complex(kk_val)).real
    ds = trig(complex(s_val, 1e-30), complex(kk_val)).imag / 1e-30
    dk = trig(complex(s_val), complex(kk_val, 1e-30)).imag / 1e-30
    for i in range(2):
        for j in range(2):
            assert m[i][j].v == pytest.approx(ref[i, j], rel=1e-15, abs=1e-18)
            assert m[i][j].d[0] == pytest.approx(ds[i, j], rel=1e-12, abs=1e-15)
            assert m[i][j].d[1] == pytest.approx(dk[i, j], rel=1e-9, abs=1e-15)
