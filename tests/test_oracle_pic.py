"""Pins of the oracle's PIC stages: deposit, solve, field, gather (the kick as
the step applies it is pinned in test_oracle_kick.py).

Every check below is fixed by mathematics independent of the code under test:
brute-force sums, exactness of linear interpolation and of central
differences on polynomials, conservation laws and symmetry.
"""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import green, physics, pic
from oracle.dual import Dual
from oracle.physics import EPS0


def _grid(n=(6, 7, 5), half=(3e-3, 4e-3, 5e-3)):
    return pic.Grid(n, [-h for h in half], list(half))


def _state(pos, ntan=3, seed=0):
    """Particles at given (x, y, z) with random position tangents."""
    rng = np.random.default_rng(seed)
    n = pos.shape[0]
    st = {}
    for j, name in enumerate(pic.COORDS):
        a = np.zeros((n, 1 + ntan))
        if name in ("x", "y", "z"):
            a[:, 0] = pos[:, "xyz".index(name)]
            a[:, 1:] = rng.normal(size=(n, ntan)) * 1e-3
        st[name] = Dual(a)
    return st


def test_solve_equals_brute_force_sum():
    rng = np.random.default_rng(1)
    n, h, g0 = (4, 5, 3), (1e-4, 1.5e-4, 2e-4), 1.7
    rho = rng.normal(size=n + (3,))
    G = green.green_offsets(n, h, g0)
    phi = pic.solve(rho, G)
    assert phi.shape == (6, 7, 5, 3)
    ref = np.zeros_like(phi)
    for i in itertools.product(*(range(-1, m + 1) for m in n)):
        acc = np.zeros(3)
        for j in itertools.product(*(range(m) for m in n)):
            o = tuple(i[d] - j[d] + n[d] for d in range(3))
            acc += rho[j] * G[o]
        ref[i[0] + 1, i[1] + 1, i[2] + 1] = acc
    np.testing.assert_allclose(phi, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_single_node_charge_gives_green_function():
    n, h, g0 = (5, 4, 6), (1e-4, 1e-4, 1e-4), 2.0
    G = green.green_offsets(n, h, g0)
    rho = np.zeros(n + (1,))
    rho[2, 1, 3, 0] = 1e-12
    phi = pic.solve(rho, G)
    for i in itertools.product(*(range(-1, m + 1) for m in n)):
        o = (i[0] - 2 + n[0], i[1] - 1 + n[1], i[2] - 3 + n[2])
        assert phi[i[0] + 1, i[1] + 1, i[2] + 1, 0] == pytest.approx(1e-12 * G[o], rel=1e-10)


def test_cic_weights_reproduce_position_and_charge():
    grid = _grid()
    rng = np.random.default_rng(2)
    pos = rng.uniform(-2.5e-3, 2.5e-3, size=(40, 3))
    st = _state(pos)
    cic = pic.cic_weights(st, grid)
    assert cic.n_outside == 0
    rho = pic.deposit(cic, grid, 1.0, 3)
    # total charge and zero total derivative charge
    assert rho[..., 0].sum() == pytest.approx(40.0, rel=1e-14)
    np.testing.assert_allclose(rho[..., 1:].sum(axis=(0, 1, 2)), 0.0, atol=1e-12)
    # first moment of the node charges equals the sum of positions (value and tangents)
    for d, name in enumerate("xyz"):
        coord = grid.lo[d] + grid.h[d] * np.arange(grid.n[d])
        shape = [1, 1, 1]
        shape[d] = -1
        m1 = (rho * coord.reshape(shape)[..., None]).sum(axis=(0, 1, 2))
        np.testing.assert_allclose(m1, st[name].a.sum(axis=0), rtol=1e-12, atol=1e-15)


def test_gather_interpolates_linear_fields_exactly():
    grid = _grid()
    rng = np.random.default_rng(3)
    pos = rng.uniform(-2.5e-3, 2.5e-3, size=(30, 3))
    st = _state(pos)
    cic = pic.cic_weights(st, grid)
    coords = np.meshgrid(*[grid.lo[d] + grid.h[d] * np.arange(grid.n[d]) for d in range(3)],
                         indexing="ij")
    E = np.zeros((3,) + grid.n + (4,))
    coef = rng.normal(size=(3, 4))
    for c in range(3):
        E[c, ..., 0] = coef[c, 0] + sum(coef[c, 1 + d] * coords[d] for d in range(3))
    e_p = pic.gather(E, cic)
    for c in range(3):
        want_v = coef[c, 0] + sum(coef[c, 1 + d] * pos[:, d] for d in range(3))
        want_d = sum(coef[c, 1 + d] * st["xyz"[d]].d for d in range(3))
        np.testing.assert_allclose(e_p[c].v, want_v, rtol=1e-12)
        np.testing.assert_allclose(e_p[c].d, want_d, rtol=1e-10, atol=1e-14)


def test_field_of_quadratic_potential_is_exact():
    grid = _grid()
    g0 = 1.9
    idx = [np.arange(-1, m + 1) for m in grid.n]
    X, Y, Z = np.meshgrid(*[grid.lo[d] + grid.h[d] * idx[d] for d in range(3)], indexing="ij")
    phi = np.stack([X * X + 3 * Y, Y * Y - Z, Z * Z + X * Y], axis=-1)
    E = pic.field(phi, grid, g0)
    c = (slice(1, -1),) * 3
    np.testing.assert_allclose(E[0][..., 0], -2 * X[c], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(E[1][..., 0], -3.0, rtol=1e-9)
    np.testing.assert_allclose(E[2][..., 0], 0.0, atol=1e-12)
    np.testing.assert_allclose(E[1][..., 1], -2 * Y[c], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(E[2][..., 1], 1.0 / g0, rtol=1e-9)
    np.testing.assert_allclose(E[2][..., 2], -2 * Z[c] / g0, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(E[0][..., 2], -Y[c], rtol=1e-9, atol=1e-12)


def _fields_at_particles(st, grid, g0, q=1e-12):
    cic = pic.cic_weights(st, grid)
    rho = pic.deposit(cic, grid, q, st["x"].n)
    G = green.green_offsets(grid.n, grid.h, g0)
    E = pic.field(pic.solve(rho, G), grid, g0)
    return cic, pic.gather(E, cic)


def test_total_space_charge_force_vanishes_for_value_and_tangents():
    grid = _grid((10, 9, 8))
    rng = np.random.default_rng(4)
    pos = rng.normal(size=(300, 3)) * 1e-3
    pos = np.clip(pos, -2.5e-3, 2.5e-3)
    st = _state(pos, ntan=4)
    _, e_p = _fields_at_particles(st, grid, 2.0)
    for c in range(3):
        tot = e_p[c].a.sum(axis=0)
        scale = np.abs(e_p[c].a).sum(axis=0)
        np.testing.assert_array_less(np.abs(tot), 1e-12 * scale + 1e-300)


def test_lone_particle_feels_no_self_force():
    grid = _grid((8, 8, 8))
    st = _state(np.array([[3.1e-4, -7.7e-4, 1.3e-3]]), ntan=3)
    _, e_p = _fields_at_particles(st, grid, 2.0)
    # compare against the field a neighbour one cell away would produce
    scale = 1e-12 / (4 * math.pi * EPS0 * grid.h.min() ** 2)
    for c in range(3):
        np.testing.assert_allclose(e_p[c].a, 0.0, atol=1e-12 * scale)


def test_mirror_symmetric_beam_gives_antisymmetric_field():
    grid = _grid((9, 9, 9), (3e-3, 3e-3, 3e-3))
    rng = np.random.default_rng(5)
    half = np.abs(rng.normal(size=(50, 3)) * 8e-4)
    half = np.clip(half, 1e-5, 2.5e-3)
    mirror = half * np.array([-1, 1, 1])
    st = _state(np.concatenate([half, mirror]), ntan=1)
    # tangents mirrored too: d(-x) = -dx
    st["x"].a[50:, 1:] = -st["x"].a[:50, 1:]
    st["y"].a[50:, 1:] = st["y"].a[:50, 1:]
    st["z"].a[50:, 1:] = st["z"].a[:50, 1:]
    _, e_p = _fields_at_particles(st, grid, 2.0)
    scale = np.abs(e_p[0].v).max()
    np.testing.assert_allclose(e_p[0].v[:50], -e_p[0].v[50:], atol=1e-12 * scale)
    np.testing.assert_allclose(e_p[1].v[:50], e_p[1].v[50:], atol=1e-12 * scale)
    np.testing.assert_allclose(e_p[2].v[:50], e_p[2].v[50:], atol=1e-12 * scale)


def test_sparse_particles_feel_pairwise_coulomb_fields():
    # three particles many cells apart: the PIC field approaches the direct
    # rest-frame Coulomb sum (self excluded); CIC smoothing sets the ~1% level
    g0 = 2.0
    grid = _grid((33, 33, 33), (8e-3, 8e-3, 8e-3))
    pos = np.array([[-4.0e-3, 0.3e-3, 0.2e-3], [3.5e-3, -0.4e-3, 0.1e-3], [0.2e-3, 4.5e-3, -3.0e-3]])
    st = _state(pos, ntan=0)
    q = 1e-12
    _, e_p = _fields_at_particles(st, grid, g0, q)
    for i in range(3):
        ref = np.zeros(3)
        for j in range(3):
            if i == j:
                continue
            d = pos[i] - pos[j]
            rr = np.array([d[0], d[1], g0 * d[2]])
            ref += q * rr / (4 * math.pi * EPS0 * np.linalg.norm(rr) ** 3)
        got = np.array([e_p[c].v[i] for c in range(3)])
        np.testing.assert_allclose(got, ref, atol=0.02 * np.linalg.norm(ref))


def test_particles_outside_box_are_counted_and_skipped():
    grid = _grid((6, 6, 6))
    pos = np.array([[0.0, 0.0, 0.0], [3.0e-3, 0.0, 0.0], [0.0, -4.1e-3, 0.0], [1e-3, 1e-3, 1e-3]])
    st = _state(pos, ntan=1)
    cic = pic.cic_weights(st, grid)
    # x = hi lies on the last node: (u-lo)/h = n-1 is outside by the half-open rule
    assert cic.n_outside == 2
    np.testing.assert_array_equal(cic.sel, [0, 3])
