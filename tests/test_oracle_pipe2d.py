"""Pins of the 2D conducting-pipe oracle (oracle/pipe2d.py). No GPU."""
import numpy as np
import pytest
import scipy.fft

import synth
from oracle import physics, pipe2d, twiss
from oracle.dual import Dual

PIPE = pipe2d.Pipe(a=0.02, b=0.016, nx=32, ny=24)


def test_single_sine_mode_is_solved_exactly():
    i = np.arange(PIPE.nx + 1)[:, None]
    j = np.arange(PIPE.ny + 1)[None, :]
    for l, m in ((1, 1), (3, 5), (PIPE.nx - 1, 2)):
        rho = (np.sin(l * np.pi * i / PIPE.nx) * np.sin(m * np.pi * j / PIPE.ny))[:, :, None]
        phi = pipe2d.solve(rho, PIPE)
        g2 = (l * np.pi / PIPE.a) ** 2 + (m * np.pi / PIPE.b) ** 2
        np.testing.assert_allclose(phi, rho / (physics.EPS0 * g2), atol=1e-12 * np.abs(rho).max() / (physics.EPS0 * g2))
    # the walls stay at zero potential
    rho = np.random.default_rng(0).normal(size=(PIPE.nx + 1, PIPE.ny + 1, 3))
    phi = pipe2d.solve(rho, PIPE)
    assert np.all(phi[0] == 0) and np.all(phi[-1] == 0) and np.all(phi[:, 0] == 0) and np.all(phi[:, -1] == 0)


def test_sine_sums_match_scipy_type_one_dst():
    rho = np.random.default_rng(1).normal(size=(PIPE.nx + 1, PIPE.ny + 1, 2))
    phi = pipe2d.solve(rho, PIPE)
    # scipy's DST-I carries a factor 2 per axis: coefficients = dstn / (Nx Ny)
    coef = scipy.fft.dstn(rho[1:-1, 1:-1], type=1, axes=(0, 1)) / (PIPE.nx * PIPE.ny)
    al = np.arange(1, PIPE.nx) * np.pi / PIPE.a
    be = np.arange(1, PIPE.ny) * np.pi / PIPE.b
    phic = coef / (physics.EPS0 * (al[:, None] ** 2 + be[None, :] ** 2))[:, :, None]
    want = scipy.fft.dstn(phic, type=1, axes=(0, 1)) / 4.0
    np.testing.assert_allclose(phi[1:-1, 1:-1], want, rtol=1e-11, atol=1e-12 * np.abs(want).max())


def test_uniform_round_beam_feels_the_perveance_kick():
    pipe = pipe2d.Pipe(a=0.08, b=0.08, nx=128, ny=128)
    r0 = 0.006
    rng = np.random.default_rng(2)
    n = 400_000
    r = r0 * np.sqrt(rng.uniform(size=n))
    th = rng.uniform(0, 2 * np.pi, size=n)
    st = {"x": Dual(np.stack([r * np.cos(th)], -1)), "y": Dual(np.stack([r * np.sin(th)], -1))}
    I = 100.0
    g0, b0 = physics.gamma_beta(1e9, physics.PROTON_REST_EV)
    lam = I / (b0 * physics.C_LIGHT)
    w = pipe2d.weights(st, pipe)
    E = pipe2d.field(pipe2d.solve(pipe2d.deposit(w, pipe, lam / n, 0), pipe), pipe)
    ex, _ = pipe2d.gather(E, w)
    x = st["x"].v[w.sel]
    inner = np.abs(x) < 0.6 * r0
    inner &= np.abs(st["y"].v[w.sel]) < 0.3 * r0
    slope = np.polyfit(x[inner], ex.v[inner], 1)[0]
    want = lam / (2 * np.pi * physics.EPS0 * r0 ** 2)
    assert slope == pytest.approx(want, rel=0.03)
    # the kick coefficient turns it into the paper's perveance: x'' = K x / r0^2
    kap = pipe2d.kick_coefficient(1e9, physics.PROTON_REST_EV, 1.0)
    K = physics.E_CHARGE * I / (2 * np.pi * physics.EPS0 * physics.PROTON_REST_EV * physics.E_CHARGE
                                * physics.C_LIGHT * b0 ** 3 * g0 ** 3)
    assert kap * want == pytest.approx(K / r0 ** 2, rel=1e-12)


def test_mirror_symmetric_beam_gives_antisymmetric_field():
    pipe = pipe2d.Pipe(a=0.02, b=0.02, nx=32, ny=32)
    rng = np.random.default_rng(3)
    x = rng.normal(scale=2e-3, size=5000)
    y = rng.normal(scale=1e-3, size=5000)
    xs = np.concatenate([x, -x])
    ys = np.concatenate([y, y])
    st = {"x": Dual(xs[:, None]), "y": Dual(ys[:, None])}
    w = pipe2d.weights(st, pipe)
    E = pipe2d.field(pipe2d.solve(pipe2d.deposit(w, pipe, 1e-12, 0), pipe), pipe)
    np.testing.assert_allclose(E[0], -E[0][::-1], atol=1e-9 * np.abs(E[0]).max())
    np.testing.assert_allclose(E[1], E[1][::-1], atol=1e-9 * np.abs(E[1]).max())


def _run(params, current=100.0, n=3000, ntan=7, steps=3):
    lat = synth.fodo_lattice(steps, 1)
    xi = synth.truncated_normals(n, 5, ncoord=4)
    seed = np.eye(7)[:, :ntan]
    return pipe2d.simulate(xi, (1e-3, 1e-3, 1e-3, 1e-3), None, params, seed, lat, PIPE, 1e9,
                           physics.PROTON_REST_EV, 1.0, current, ntan)


def test_zero_current_matches_the_transfer_matrices():
    lat = synth.fodo_lattice(3, 1)
    p = synth.NOMINAL_PARAMS
    res = _run(p, current=0.0, ntan=0)
    Mx, My = twiss.line_matrices(lat.kind, lat.L, lat.k, lat.L_param, lat.k_param, p, np.zeros((7, 0)))
    xi = synth.truncated_normals(3000, 5, ncoord=4) * 1e-3
    for (M, u, q) in ((Mx, 0, 1), (My, 2, 3)):
        m = np.array([[M[0][0].v, M[0][1].v], [M[1][0].v, M[1][1].v]], dtype=float)
        want = xi[:, [u, q]] @ m.T
        np.testing.assert_allclose(res.particles[:, [u, q], 0], want, rtol=1e-12, atol=1e-15)


def test_run_derivatives_match_central_differences():
    p0 = np.asarray(synth.NOMINAL_PARAMS, dtype=float)
    res = _run(p0, current=400.0)
    fd = np.zeros((2, 7))
    for j in range(7):
        h = 1e-6 * abs(p0[j])
        up, dn = p0.copy(), p0.copy()
        up[j] += h
        dn[j] -= h
        fd[:, j] = (_run(up, 400.0, ntan=0).emittance[:, 0] - _run(dn, 400.0, ntan=0).emittance[:, 0]) / (2 * h)
    for pl in range(2):
        assert np.abs(res.emittance[pl, 1:] - fd[pl]).max() <= 1e-5 * np.abs(fd[pl]).max()
