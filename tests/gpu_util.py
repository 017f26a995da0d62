"""Helpers shared by the GPU tests: build a Simulation from a workload and
compare dual arrays at the stated tolerances.

Tolerances (FP64 GPU path against the FP64 oracle):
  * values: 1e-10 relative (per scalar for emittances and moments,
    normwise over particles for a particle coordinate);
  * derivatives: normwise over the tangent components of one output,
    ||g - g_ref||_inf <= 1e-9 ||g_ref||_inf;
  * single-stage grid arrays (one deposit, one solve, one field): 1e-12
    normwise per channel, since only one stage's rounding separates them.
"""
import numpy as np

VALUE_RTOL = 1e-10
DERIV_RTOL = 1e-9


def make_sim(w, capacity=None, sort_every=5, n_particles=None, xi=None):
    """sort_every 5 (the default here) is the benchmark's tiled configuration,
    which the library's automatic default takes only for larger beams; 0
    selects the storage-order kernel with global atomics; None keeps the
    library default (-1, automatic)."""
    from paper_2511_21839_amd import dpic

    sim = dpic.Simulation(capacity or w.n_particles, w.ntan, w.grid)
    sim.set_beam(w.kinetic_eV, w.rest_eV, w.charge_e, w.bunch_charge_C)
    sim.set_grid(w.lo, w.hi)
    L = w.lattice
    sim.set_lattice(L.kind, L.n_steps, L.L, L.k, L.L_param, L.k_param, L.n_periods)
    sim.set_params(w.params, w.param_seed())
    if sort_every is not None:  # before the beam, which init_beam stores sorted when the cadence tiles
        sim.set_option(dpic.OPT_SORT_EVERY, sort_every)
    sim.init_beam(w.xi() if xi is None else xi, w.sigma, w.sigma_seed())
    return sim


def normwise_err(got, want, axis=None):
    got, want = np.asarray(got), np.asarray(want)
    den = np.abs(want).max(axis=axis)
    num = np.abs(got - want).max(axis=axis)
    return num / np.where(den > 0, den, 1.0)


def assert_particles_close(got, want, vtol=VALUE_RTOL, dtol=DERIV_RTOL):
    """got/want: (N, 6, 1+ntan)."""
    assert got.shape == want.shape, (got.shape, want.shape)
    for j in range(6):
        ev = normwise_err(got[:, j, 0], want[:, j, 0])
        assert ev <= vtol, f"coordinate {j} value error {ev:.3e}"
        if got.shape[2] > 1:
            ed = normwise_err(got[:, j, 1:], want[:, j, 1:])
            assert ed <= dtol, f"coordinate {j} derivative error {ed:.3e}"


def moment_term_scales(particles):
    """Mean magnitude of the summed terms of every moment, (3, 5, 2): value, derivatives.

    A moment is a sum over particles; when the terms cancel (the mean
    momentum's derivatives vanish by momentum conservation) the rounding error
    of either side is relative to the sum of |terms|, not to the sum itself.
    """
    P = np.asarray(particles)
    out = np.zeros((3, 5, 2))
    for pl in range(3):
        u, p = P[:, 2 * pl], P[:, 2 * pl + 1]
        terms = []
        for a, b in ((u, u), (u, p), (p, p)):
            v = a[:, 0] * b[:, 0]
            d = a[:, :1] * b[:, 1:] + a[:, 1:] * b[:, :1]
            terms.append((v, d))
        terms.append((u[:, 0], u[:, 1:]))
        terms.append((p[:, 0], p[:, 1:]))
        for m, (v, d) in enumerate(terms):
            out[pl, m, 0] = np.abs(v).mean()
            out[pl, m, 1] = np.abs(d).max(axis=1).mean() if d.shape[1] else 0.0
    return out


def assert_moments_close(got, want, ref_particles, vtol=VALUE_RTOL, dtol=DERIV_RTOL):
    got, want = np.asarray(got), np.asarray(want)
    sc = moment_term_scales(ref_particles)
    for pl in range(3):
        for m in range(5):
            g, w = got[pl, m], want[pl, m]
            sv = max(abs(w[0]), sc[pl, m, 0])
            assert abs(g[0] - w[0]) <= vtol * sv, (pl, m, g[0], w[0])
            if g.shape[0] > 1:
                sd = max(np.abs(w[1:]).max(), sc[pl, m, 1])
                assert np.abs(g[1:] - w[1:]).max() <= dtol * sd, (pl, m, g[1:], w[1:])


def assert_outputs_close(got, want, vtol=VALUE_RTOL, dtol=DERIV_RTOL, what="output"):
    """got/want: (..., 1+ntan); value per scalar, derivatives normwise per output."""
    got, want = np.asarray(got), np.asarray(want)
    assert got.shape == want.shape
    g = got.reshape(-1, got.shape[-1])
    w = want.reshape(-1, want.shape[-1])
    for i in range(g.shape[0]):
        rv = abs(g[i, 0] - w[i, 0]) / max(abs(w[i, 0]), 1e-300)
        assert rv <= vtol, f"{what}[{i}] value {g[i, 0]!r} vs {w[i, 0]!r} (rel {rv:.3e})"
        if g.shape[1] > 1:
            rd = normwise_err(g[i, 1:], w[i, 1:])
            assert rd <= dtol, f"{what}[{i}] derivatives rel {rd:.3e}: {g[i, 1:]} vs {w[i, 1:]}"
