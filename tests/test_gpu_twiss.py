"""Twiss parameters, their lattice derivatives and the matching optimisers
on the GPU (include/dtwiss.h) against the oracle (oracle/twiss.py)."""
import numpy as np
import pytest

import synth
from oracle import twiss
from oracle.dual import Dual

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _fodo():
    from paper_2511_21839_amd import pipe2d as p2

    lat = synth.fodo_lattice(1, 1)
    return lat, p2.Twiss(lat.kind, lat.L, lat.k, lat.L_param, lat.k_param, nmax=64)


def _oracle_periodic(lat, p, ntan=7):
    Mx, My = twiss.line_matrices(lat.kind, lat.L, lat.k, lat.L_param, lat.k_param, p, np.eye(7)[:, :ntan])
    return np.array([t.a for t in (*twiss.periodic(Mx), *twiss.periodic(My))])


def test_periodic_twiss_and_derivatives_match_oracle():
    lat, tw = _fodo()
    rng = np.random.default_rng(1)
    P = np.asarray(synth.NOMINAL_PARAMS) * (1 + rng.uniform(-0.05, 0.05, size=(20, 7)))
    got = tw.eval(P)
    for s in range(20):
        want = _oracle_periodic(lat, P[s])
        np.testing.assert_allclose(got[s], want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_relative_sensitivities_match_central_differences():
    # the paper's Fig. 5 quantity x dT / (T dx) from one evaluation, against
    # central differences with 14 evaluations
    lat, tw = _fodo()
    p0 = np.asarray(synth.NOMINAL_PARAMS, dtype=float)
    t = tw.eval(p0[None])[0]
    rel = t[:, 1:] * p0[None, :] / t[:, :1]
    fd = np.zeros((4, 7))
    for j in range(7):
        h = 1e-6 * abs(p0[j])
        up, dn = p0.copy(), p0.copy()
        up[j] += h
        dn[j] -= h
        tu, td = tw.eval(up[None])[0][:, 0], tw.eval(dn[None])[0][:, 0]
        fd[:, j] = (tu - td) / (2 * h) * p0[j] / t[:, 0]
    np.testing.assert_allclose(rel, fd, rtol=1e-6, atol=1e-8)


def _matching():
    m = synth.matching()
    lat_from, lat_to = synth.fodo_lattice(1, 1), synth.fodo_lattice(1, 1)
    nz = np.zeros((7, 0))

    def periodic(kq):
        kk = [0.0, kq[0], 0.0, kq[1], 0.0]
        Mx, My = twiss.line_matrices(lat_from.kind, [0.1, 0.1, 0.2, 0.1, 0.1], kk, [-1] * 5, [-1] * 5, [], np.zeros((0, 0)))
        return [float(v.v) for v in (*twiss.periodic(Mx), *twiss.periodic(My))]

    return m, periodic(m.cell_from), periodic(m.cell_to)


def test_matching_objective_and_gradient_match_oracle():
    from paper_2511_21839_amd import pipe2d as p2

    m, t0, tt = _matching()
    tw = p2.Twiss(m.kind, m.L, [0.0] * len(m.kind), [-1] * len(m.kind), m.k_param, nmax=8)
    K = np.asarray(m.k0) * (1 + np.random.default_rng(2).uniform(-0.2, 0.2, size=(8, 4)))
    _, f = tw.eval(K, twiss0=t0, target=tt)
    for s in range(8):
        Mx, My = twiss.line_matrices(m.kind, m.L, [0.0] * len(m.kind), [-1] * len(m.kind), m.k_param, K[s], np.eye(4))
        bx, ax = twiss.transport(Mx, Dual.const(t0[0], 4), Dual.const(t0[1], 4))
        by, ay = twiss.transport(My, Dual.const(t0[2], 4), Dual.const(t0[3], 4))
        want = twiss.matching_objective((bx, ax, by, ay), tt).a
        np.testing.assert_allclose(f[s], want, rtol=1e-11, atol=1e-12 * np.abs(want).max())


def test_bfgs_matching_reaches_the_target_and_the_oracle_optimum():
    from paper_2511_21839_amd import pipe2d as p2

    m, t0, tt = _matching()
    tw = p2.Twiss(m.kind, m.L, [0.0] * len(m.kind), [-1] * len(m.kind), m.k_param, nmax=1)
    kb, fb, nb, hb = tw.match(m.k0, t0, tt, tol=1e-14, max_eval=500)
    assert fb < 1e-12 and nb < 500
    assert hb[-1] == fb and hb[0] > 1e3 * fb
    # the oracle's BFGS reaches the same strengths
    def fg(kv):
        Mx, My = twiss.line_matrices(m.kind, m.L, [0.0] * len(m.kind), [-1] * len(m.kind), m.k_param, kv, np.eye(4))
        bx, ax = twiss.transport(Mx, Dual.const(t0[0], 4), Dual.const(t0[1], 4))
        by, ay = twiss.transport(My, Dual.const(t0[2], 4), Dual.const(t0[3], 4))
        f = twiss.matching_objective((bx, ax, by, ay), tt)
        return float(f.v), np.asarray(f.d, dtype=float)
    ko, fo, _, _ = twiss.bfgs(fg, m.k0, tol=1e-14, max_iter=300)
    np.testing.assert_allclose(kb, ko, rtol=1e-7)
