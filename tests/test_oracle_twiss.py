"""Pins of the Twiss oracle and its optimisers (oracle/twiss.py). No GPU."""
import numpy as np
import pytest

import synth
from oracle import twiss
from oracle.dual import Dual


def _fodo_matrices(params, ntan=7):
    lat = synth.fodo_lattice(1, 1)
    seed = np.eye(7)[:, :ntan]
    return twiss.line_matrices(lat.kind, lat.L, lat.k, lat.L_param, lat.k_param, params, seed)


def _num(m):
    return np.array([[m[0][0].v, m[0][1].v], [m[1][0].v, m[1][1].v]], dtype=float)


def test_transport_matches_sigma_matrix_transport():
    Mx, My = _fodo_matrices(synth.NOMINAL_PARAMS, ntan=0)
    for M in (Mx, My):
        m = _num(M)
        assert np.linalg.det(m) == pytest.approx(1.0, abs=1e-13)
        b0, a0 = 1.7, -0.4
        g0 = (1 + a0 ** 2) / b0
        S1 = m @ np.array([[b0, -a0], [-a0, g0]]) @ m.T
        b1, a1 = twiss.transport(M, Dual.const(b0, 0), Dual.const(a0, 0))
        assert float(b1.v) == pytest.approx(S1[0, 0], rel=1e-13)
        assert float(a1.v) == pytest.approx(-S1[0, 1], rel=1e-12)


def test_matched_twiss_are_periodic_and_match_the_cell_tune():
    Mx, My = _fodo_matrices(synth.NOMINAL_PARAMS, ntan=0)
    for M in (Mx, My):
        b, a = twiss.periodic(M)
        b1, a1 = twiss.transport(M, b, a)
        assert float(b1.v) == pytest.approx(float(b.v), rel=1e-12)
        assert float(a1.v) == pytest.approx(float(a.v), abs=1e-12)
        m = _num(M)
        # the proposed FODO: cos mu = 0.830668 in both planes, beta = 1.0365 m at the entry
        assert (m[0, 0] + m[1, 1]) / 2 == pytest.approx(0.830668, abs=2e-6)
        assert float(b.v) == pytest.approx(1.0365, abs=2e-4)


def test_twiss_derivatives_match_central_differences():
    p0 = np.asarray(synth.NOMINAL_PARAMS, dtype=float)
    Mx, My = _fodo_matrices(p0)
    tw = [*twiss.periodic(Mx), *twiss.periodic(My)]
    for j in range(7):
        h = 1e-6 * abs(p0[j])
        up, dn = p0.copy(), p0.copy()
        up[j] += h
        dn[j] -= h
        Mu, Nu = _fodo_matrices(up, ntan=0)
        Md, Nd = _fodo_matrices(dn, ntan=0)
        tu = [*twiss.periodic(Mu), *twiss.periodic(Nu)]
        td = [*twiss.periodic(Md), *twiss.periodic(Nd)]
        for q in range(4):
            fd = (float(tu[q].v) - float(td[q].v)) / (2 * h)
            assert float(tw[q].d[j]) == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_bfgs_on_textbook_functions():
    A = np.array([[3.0, 1.0], [1.0, 2.0]])
    b = np.array([1.0, -2.0])
    fq = lambda x: (0.5 * x @ A @ x - b @ x + 0.5 * b @ np.linalg.solve(A, b), A @ x - b)
    x, f, ne, _ = twiss.bfgs(fq, [4.0, -3.0], tol=1e-14)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), atol=1e-6)

    def rosen_g(x):
        f = (1 - x[0]) ** 2 + 100 * (x[1] - x[0] ** 2) ** 2
        return f, np.array([-2 * (1 - x[0]) - 400 * x[0] * (x[1] - x[0] ** 2), 200 * (x[1] - x[0] ** 2)])

    x, f, ne_b, _ = twiss.bfgs(rosen_g, [-1.2, 1.0], tol=1e-14, max_iter=500)
    assert f < 1e-10
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-5)
