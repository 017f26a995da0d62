"""Pins of the space-charge map M2(tau) as the oracle's step applies it
(Sec. 4: the split step M1(tau/2) M2(tau) M1(tau/2), with M2 leaving the
positions fixed and moving the momenta by the space-charge force over the
full step tau).

Each test runs the oracle's whole step (pic.simulate) on a beam whose momenta
start at zero, through one short drift taken in a single step. The first
half map then leaves the positions unchanged, the kick fills the momenta,
and the closing half map moves only the positions. So the final momenta are
the kick alone, and they are compared with momentum changes computed here by
a route that shares nothing with the oracle's kick:

  * the lab-frame fields of uniformly moving charges (the textbook field of a
    charge moving at v0 along z, E = Q gamma d / (4 pi eps0
    (dx^2 + dy^2 + gamma^2 dz^2)^(3/2)) at equal lab time, B = v x E / c^2);
  * the Lorentz force F = q (E + v x B) on a test proton moving at v0, held
    for the transit time tau / v0 of the step, divided by p0.

A kick scaled by a wrong coefficient (the transverse kappa on the
longitudinal momentum, a factor gamma0), applied over half the step, or with
a flipped sign fails these tests by tens of percent; the tolerances are a
few percent (cloud-in-cell smoothing and the finite grid).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special
from scipy.stats import qmc

import synth
from oracle import pic

E_CH = 1.602176634e-19
C0 = 299792458.0
EPS_0 = 8.8541878128e-12
REST_EV = 938.27208816e6
T_EV = 1e9


def _kinematics():
    g = 1.0 + T_EV / REST_EV
    b = math.sqrt(1.0 - 1.0 / g ** 2)
    m = REST_EV * E_CH / C0 ** 2
    return g, b, m * g * b * C0  # gamma0, beta0, p0


def _lorentz_dp(E_lab, tau):
    """Normalised momentum change (dpx/p0, dpy/p0, d delta) of a proton
    moving at v0 along z through lab field E_lab (of sources moving with it)
    over the path length tau."""
    g, b, p0 = _kinematics()
    v = np.array([0.0, 0.0, b * C0])
    B = np.cross(v, E_lab) / C0 ** 2
    F = E_CH * (E_lab + np.cross(v, B))
    return F * (tau / (b * C0)) / p0


def _one_drift(L):
    return synth.Lattice(kind=[synth.DRIFT], n_steps=[1], L=[L], k=[0.0], L_param=[0], k_param=[-1],
                         n_periods=1)


def _run_one_step(pos, bunch_charge, grid_n, half, L=0.01):
    """One oracle step of a beam at rest in the transverse and longitudinal
    momenta; tangent 0 is d/dL of the drift's length."""
    n = pos.shape[0]
    xi = np.zeros((n, 6))
    xi[:, 0], xi[:, 2], xi[:, 4] = pos[:, 0], pos[:, 1], pos[:, 2]
    return pic.simulate(xi=xi, sigma=(1.0,) * 6, sigma_seed=None, params=(L,), param_seed=np.ones((1, 1)),
                        lat=_one_drift(L), grid_n=grid_n, lo=[-h for h in half], hi=list(half),
                        kinetic_eV=T_EV, rest_eV=REST_EV, charge_e=1.0, bunch_charge_C=bunch_charge,
                        ntan=1)


# sparse macroparticles, every pair at least 11 cells apart
SPARSE = np.array([
    [0.0, 0.0, -4.5e-3],
    [0.3e-3, -0.2e-3, 4.2e-3],
    [4.6e-3, 0.4e-3, 0.3e-3],
    [-0.5e-3, -4.4e-3, -0.6e-3],
    [-4.1e-3, 4.3e-3, 4.0e-3],
])


def _sparse_reference(pos, q_macro, tau):
    g, _, _ = _kinematics()
    out = np.zeros((pos.shape[0], 3))
    for i in range(pos.shape[0]):
        E = np.zeros(3)
        for j in range(pos.shape[0]):
            if i == j:
                continue
            d = pos[i] - pos[j]
            den = (d[0] ** 2 + d[1] ** 2 + (g * d[2]) ** 2) ** 1.5
            E += q_macro * g * d / (4 * math.pi * EPS_0 * den)
        out[i] = _lorentz_dp(E, tau)
    return out


def test_one_step_kick_of_sparse_charges_equals_lorentz_force():
    L, q_macro = 0.01, 1e-12
    r = _run_one_step(SPARSE, q_macro * len(SPARSE), (64, 64, 64), (8e-3, 8e-3, 8e-3), L=L)
    assert r.out_of_box == 0
    got = r.particles[:, [1, 3, 5], 0]
    want = _sparse_reference(SPARSE, q_macro, L)
    for i in range(len(SPARSE)):
        scale = np.linalg.norm(want[i])
        np.testing.assert_allclose(got[i], want[i], atol=0.02 * scale, err_msg=f"particle {i}")
    # the longitudinal momentum change dominates for the two particles on the
    # z axis, so a wrong longitudinal coefficient cannot hide in the norm
    for i in (0, 1):
        assert abs(want[i, 2]) > 0.5 * np.linalg.norm(want[i])
        assert got[i, 2] == pytest.approx(want[i, 2], rel=0.03)
    # tau = L in one step, and the kick is tau times a field that does not
    # depend on L here (the momenta are zero at the first half map), so the
    # tangent of every momentum is the kick divided by L
    np.testing.assert_allclose(r.particles[:, [1, 3, 5], 1], got / L, rtol=1e-12,
                               atol=1e-12 * np.abs(got).max() / L)


def _gaussian_rest_field(x, y, zr, sx, sy, szr, Q):
    """Rest-frame field of a Gaussian charge Q with rms sizes (sx, sy, szr),
    from 1/r = (2/sqrt(pi)) int_0^inf exp(-r^2 t^2) dt: the potential is
    Q/(4 pi eps0) (2/sqrt(pi)) int prod_i exp(-x_i^2 t^2 / (1 + 2 s_i^2 t^2)) / sqrt(1 + 2 s_i^2 t^2) dt,
    and E_i is minus its derivative in x_i."""
    def f(t, comp):
        a = [1.0 + 2.0 * s * s * t * t for s in (sx, sy, szr)]
        u = [x, y, zr]
        w = math.exp(-sum(u[i] ** 2 * t * t / a[i] for i in range(3))) / math.sqrt(a[0] * a[1] * a[2])
        return w * 2.0 * u[comp] * t * t / a[comp]

    pref = Q / (4 * math.pi * EPS_0) * 2.0 / math.sqrt(math.pi)
    return np.array([pref * integrate.quad(f, 0.0, np.inf, args=(c,), epsabs=0, epsrel=1e-10, limit=200)[0]
                     for c in range(3)])


def test_gaussian_field_formula_has_the_paper_perveance_long_beam_limit():
    """The reference field used below reduces, for a long bunch, to the
    paper's generalised-perveance kick x'' = K x / a^2 of a uniform round
    beam (Sec. 4, K = q I / (2 pi eps0 p0 v0^2 gamma0^2)); a round Gaussian
    has the central focusing of a uniform beam of radius a = sqrt(2) sigma."""
    g, b, p0 = _kinematics()
    sig, sz, Q = 1e-3, 0.4, 1e-9  # lab bunch length 400 sigma
    lam_lab = Q / (math.sqrt(2 * math.pi) * sz)
    I = lam_lab * b * C0
    K = E_CH * I / (2 * math.pi * EPS_0 * p0 * (b * C0) ** 2 * g ** 2)
    x = 0.05 * sig
    Er = _gaussian_rest_field(x, 0.0, 0.0, sig, sig, g * sz, Q)
    dp = _lorentz_dp(g * np.array([Er[0], 0.0, Er[2]]), 1.0)  # lab E_perp = gamma E_rest_perp
    assert dp[0] == pytest.approx(K * x / (2 * sig ** 2), rel=2e-3)


def test_one_step_kick_of_gaussian_bunch_equals_closed_form_field():
    """A quiet-start Gaussian bunch (scrambled Sobol points through the normal
    quantile), one step: the kick of particles in the core equals the
    Lorentz force of the continuous bunch's field, transverse and
    longitudinal, to 2% (grid smoothing and sampling; measured below 1%).
    The bunch is 1.5 sigma_x long in the lab, so that the rest-frame cells
    (gamma0 h_z against h_x) stay within an aspect of about 3: with point
    charges on much longer cells the potential of the discrete grid departs
    from the continuous one at the few-percent level."""
    g, _, _ = _kinematics()
    sx, sy, sz = 1.0e-3, 1.0e-3, 1.5e-3
    n = 2 ** 16
    u = qmc.Sobol(d=3, scramble=True, seed=11).random(n)
    xi = special.ndtri(np.clip(u, 1e-12, 1 - 1e-12))
    keep = np.all(np.abs(xi) < 4.2, axis=1)
    pos = xi[keep] * np.array([sx, sy, sz])
    Q, L = 2e-9, 0.01
    half = (4.3 * sx, 4.3 * sy, 4.3 * sz)
    r = _run_one_step(pos, Q * keep.mean(), (64, 64, 64), half, L=L)
    assert r.out_of_box == 0
    dp = r.particles[:, [1, 3, 5], 0]
    rr = np.hypot(pos[:, 0] / sx, pos[:, 1] / sy)
    core = np.nonzero((rr < 1.5) & (np.abs(pos[:, 2]) < 1.5 * sz))[0]
    pick = core[np.linspace(0, len(core) - 1, 60).astype(int)]
    want = np.zeros((len(pick), 3))
    for k, i in enumerate(pick):
        x, y, z = pos[i]
        Er = _gaussian_rest_field(x, y, g * z, sx, sy, g * sz, Q * keep.mean())
        # lab field of the moving bunch: E_perp,lab = gamma E_perp,rest, E_z,lab = E_z,rest
        want[k] = _lorentz_dp(np.array([g * Er[0], g * Er[1], Er[2]]), L)
    got = dp[pick]
    for c in range(3):
        scale = np.abs(want[:, c]).max()
        err = np.abs(got[:, c] - want[:, c]).max() / scale
        assert err <= 0.02, (c, err)
    # the sample spans both signs of every component
    assert all((want[:, c] > 0).any() and (want[:, c] < 0).any() for c in range(3))


# ---------------------------------------------------------------------------
# centred emittance (the optional variant of the Sec. 4 emittance)
# ---------------------------------------------------------------------------
def _random_state(n=500, ntan=3, seed=0, shift=0.0):
    rng = np.random.default_rng(seed)
    st = {}
    A = rng.normal(size=(6, 6)) * 0.3 + np.eye(6)
    base = rng.normal(size=(n, 6)) @ A.T
    for j, name in enumerate(pic.COORDS):
        a = np.zeros((n, 1 + ntan))
        a[:, 0] = base[:, j] * 1e-3 + shift * (j + 1) * 1e-4
        a[:, 1:] = rng.normal(size=(n, ntan)) * 1e-4
        st[name] = pic.Dual(a)
    return st


def _cov_emittance(u, p):
    """sqrt(det) of the 1/N covariance matrix of (u, p), numpy's own routine."""
    return math.sqrt(np.linalg.det(np.cov(np.stack([u, p]), bias=True)))


def test_centred_emittance_equals_covariance_determinant_and_its_derivatives():
    st = _random_state(shift=3.0)
    eps = pic.emittance(pic.moments(st), centred=True)
    for pl, (un, pn) in enumerate((("x", "px"), ("y", "py"), ("z", "d"))):
        U, P = st[un].a, st[pn].a
        assert eps[pl, 0] == pytest.approx(_cov_emittance(U[:, 0], P[:, 0]), rel=1e-12)
        for t in range(U.shape[1] - 1):
            h = 1e-4  # tangent rows are ~1e-4 against values ~1e-3
            fd = (_cov_emittance(U[:, 0] + h * U[:, 1 + t], P[:, 0] + h * P[:, 1 + t])
                  - _cov_emittance(U[:, 0] - h * U[:, 1 + t], P[:, 0] - h * P[:, 1 + t])) / (2 * h)
            assert eps[pl, 1 + t] == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(eps[pl, 0])), (pl, t)


def test_centred_emittance_is_shift_invariant_and_equals_raw_for_zero_mean():
    st = _random_state(seed=1)
    eps = pic.emittance(pic.moments(st), centred=True)
    # shift every coordinate by a dual constant (value and tangents)
    rng = np.random.default_rng(2)
    shifted = {}
    for name in pic.COORDS:
        c = rng.normal(size=st[name].a.shape[1]) * 1e-3
        shifted[name] = pic.Dual(st[name].a + c[None, :])
    eps_s = pic.emittance(pic.moments(shifted), centred=True)
    np.testing.assert_allclose(eps_s, eps, rtol=1e-9, atol=1e-9 * np.abs(eps).max())
    # a beam and its point reflection have zero mean: centred equals raw
    sym = {name: pic.Dual(np.concatenate([st[name].a, -st[name].a])) for name in pic.COORDS}
    mom = pic.moments(sym)
    np.testing.assert_allclose(pic.emittance(mom, centred=True), pic.emittance(mom), rtol=1e-13)
    # and raw differs from centred once the beam is off centre
    off = _random_state(seed=1, shift=3.0)
    mo = pic.moments(off)
    assert np.abs(pic.emittance(mo)[:, 0] - pic.emittance(mo, centred=True)[:, 0]).min() > 1e-3 * eps[:, 0].min()
