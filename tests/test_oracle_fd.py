"""Central finite differences of the full space-charge run (the paper's own
check, Sec. 3 and Sec. 4: central differences with two runs per parameter).

The dual-number derivatives of the final emittances must agree with
(eps(p + h) - eps(p - h)) / 2h, h = 1e-6 |p|, from value-only runs. Agreement is
limited by truncation and rounding of the difference quotient, so the bound
is 1e-5 normwise over the parameters (per emittance).
"""
import numpy as np
import pytest

import synth
from oracle import pic


def _fd_emittance(w, j, rel=1e-6):
    p = np.asarray(w.params, dtype=np.float64)
    h = rel * abs(p[j])
    out = []
    for sgn in (1.0, -1.0):
        q = p.copy()
        q[j] += sgn * h
        r = pic.simulate_workload(w.with_(ntan=0), params=tuple(q))
        out.append(r.emittance[:, 0])
    return (out[0] - out[1]) / (2 * h)


def test_emittance_derivatives_match_central_differences():
    w = synth.tiny(n_particles=1500, grid=16, steps_per_element=4)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 10)  # strong space charge
    r = pic.simulate_workload(w)
    assert r.out_of_box == 0
    fd = np.stack([_fd_emittance(w, j) for j in range(7)], axis=1)  # [plane][param]
    ad = r.emittance[:, 1:8]
    for pl in range(2):
        err = np.abs(ad[pl] - fd[pl]).max()
        assert err <= 1e-5 * np.abs(ad[pl]).max(), (pl, ad[pl], fd[pl])
    # space charge makes the lattice derivatives non-zero (unlike zero current)
    assert np.abs(ad[0]).max() > 1e-3 * r.emittance[0, 0]


def test_sigma_derivatives_match_central_differences():
    w = synth.tiny(n_particles=1000, grid=16, steps_per_element=3, ntan=13,
                   sigma_tangents=True)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 10)
    r = pic.simulate_workload(w)
    for j in (0, 3, 4):
        s = np.asarray(w.sigma, dtype=np.float64)
        h = 1e-6 * s[j]
        e = []
        for sgn in (1.0, -1.0):
            t = s.copy()
            t[j] += sgn * h
            e.append(pic.simulate_workload(w.with_(ntan=0, sigma_tangents=False,
                                                   sigma=tuple(t))).emittance[:, 0])
        fd = (e[0] - e[1]) / (2 * h)
        ad = r.emittance[:, 8 + j]
        np.testing.assert_allclose(ad[:2], fd[:2], rtol=1e-5,
                                   atol=1e-5 * np.abs(r.emittance[:2, 8:]).max())
