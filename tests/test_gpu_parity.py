"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every case feeds both sides the same seeded inputs and compares element by
element at the tolerances stated in gpu_util. Stage tests isolate one kernel
group each (deposit, solve, field); run tests compare the particle state,
the moments and the emittances after whole schedules.
"""
import math

import numpy as np
import pytest

import synth
from oracle import green, physics, pic
from gpu_util import (assert_moments_close, assert_outputs_close, assert_particles_close, make_sim,
                      normwise_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_21839_amd import dpic

    dpic.lib()
    yield


def _oracle(w, **kw):
    return pic.simulate_workload(w, **kw)


def _to_gpu_grid(a):
    """oracle [ix, iy, iz, ch] -> library [iz, iy, ix, ch]"""
    return np.ascontiguousarray(np.transpose(a, (2, 1, 0, 3)))


def _field_to_gpu(E):
    """oracle [comp, ix, iy, iz, ch] -> library [iz, iy, ix, comp, ch]"""
    return np.ascontiguousarray(np.transpose(E, (3, 2, 1, 0, 4)))


def _compare_run(w, sim, ref):
    assert_particles_close(sim.particles(), ref.particles)
    assert_moments_close(sim.moments(), ref.moments, ref.particles)
    assert_outputs_close(sim.emittance(), ref.emittance, what="emittance")
    assert_outputs_close(sim.emittance(centred=True), pic.emittance(ref.moments, centred=True),
                         what="centred emittance")
    oob, steps, ext = sim.counters()
    assert oob == ref.out_of_box
    assert steps == ref.steps
    np.testing.assert_allclose(ext, ref.max_extent, rtol=1e-10)


# ---------------------------------------------------------------- stages
def test_stage_deposit_matches_oracle():
    from paper_2511_21839_amd import dpic

    w = synth.tiny(n_particles=2999, grid=16)
    sim = make_sim(w)
    sim.stage(dpic.STAGE_DEPOSIT)
    got = sim.read_grid(dpic.GRID_RHO)
    st = pic.initial_state(w.xi(), w.sigma, w.sigma_seed(), w.ntan)
    grid = pic.Grid(w.grid, w.lo, w.hi)
    want = _to_gpu_grid(pic.deposit(pic.cic_weights(st, grid), grid, w.bunch_charge_C / w.n_particles, w.ntan))
    for ch in range(w.ntan + 1):
        assert normwise_err(got[..., ch], want[..., ch]) <= 1e-12, ch


# 64 or 32 nodes in both y and z take the fused y-z pass (passes 2-4 in one kernel)
@pytest.mark.parametrize("grid,ntan", [((16, 16, 16), 7), ((32, 16, 8), 7), ((8, 64, 16), 7), ((16, 64, 64), 7),
                                       ((16, 64, 64), 0), ((16, 64, 64), 13), ((64, 64, 64), 7), ((32, 32, 32), 7),
                                       ((16, 32, 32), 13), ((64, 32, 32), 0)])
def test_stage_solve_matches_oracle(grid, ntan):
    from paper_2511_21839_amd import dpic

    w = synth.tiny(n_particles=10, grid=16, ntan=ntan).with_(grid=grid)
    sim = make_sim(w)
    rng = np.random.default_rng(11)
    rho = rng.normal(size=tuple(grid) + (w.ntan + 1,)) * 1e-15
    if w.ntan >= 3:
        rho[..., 3] *= 1e-6  # channels of very different size stay separate
    sim.write_grid(dpic.GRID_RHO, _to_gpu_grid(rho))
    sim.stage(dpic.STAGE_SOLVE)
    got = sim.read_grid(dpic.GRID_PHI)
    g0, _ = physics.gamma_beta(w.kinetic_eV, w.rest_eV)
    pg = pic.Grid(grid, w.lo, w.hi)
    want = _to_gpu_grid(pic.solve(rho, green.green_offsets(pg.n, pg.h, g0)))
    for ch in range(w.ntan + 1):
        e = normwise_err(got[..., ch], want[..., ch])
        assert e <= 1e-12 or (ch == 3 and e <= 1e-9), (ch, e)
    # the solve consumes rho
    assert not np.any(sim.read_grid(dpic.GRID_RHO))


def test_stage_field_matches_oracle():
    from paper_2511_21839_amd import dpic

    w = synth.tiny(n_particles=10, grid=16).with_(grid=(16, 8, 32))
    sim = make_sim(w)
    rng = np.random.default_rng(12)
    phi = rng.normal(size=(18, 10, 34, w.ntan + 1))
    sim.write_grid(dpic.GRID_PHI, _to_gpu_grid(phi))
    sim.stage(dpic.STAGE_FIELD)
    got = sim.read_grid(dpic.GRID_E)
    g0, _ = physics.gamma_beta(w.kinetic_eV, w.rest_eV)
    want = _field_to_gpu(pic.field(phi, pic.Grid(w.grid, w.lo, w.hi), g0))
    assert normwise_err(got, want) <= 1e-13


# ---------------------------------------------------------------- whole runs
def test_zero_current_run_matches_oracle():
    w = synth.tiny(n_particles=777, steps_per_element=6).with_(bunch_charge_C=0.0)
    sim = make_sim(w)
    sim.step(w.total_steps())
    ref = _oracle(w)
    assert_particles_close(sim.particles(), ref.particles)
    assert_moments_close(sim.moments(), ref.moments, ref.particles)
    # the emittance is invariant under the linear maps, so its lattice
    # derivatives vanish: both sides hold rounding noise, checked on the
    # scale eps / p of a relative sensitivity
    got = sim.emittance()
    for pl in range(3):
        assert abs(got[pl, 0] - ref.emittance[pl, 0]) <= 1e-10 * ref.emittance[pl, 0]
        assert np.all(np.abs(got[pl, 1:] * np.asarray(w.params)) <= 1e-11 * ref.emittance[pl, 0])
    oob, steps, ext = sim.counters()
    assert (oob, steps) == (ref.out_of_box, ref.steps)
    np.testing.assert_allclose(ext, ref.max_extent, rtol=1e-10)


@pytest.mark.parametrize("sort_every", [0, 1, 3, 50])
def test_tiny_space_charge_run_matches_oracle(sort_every):
    w = synth.tiny(n_particles=3001, grid=16, steps_per_element=4)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 10)
    sim = make_sim(w, sort_every=sort_every)
    sim.step(w.total_steps())
    _compare_run(w, sim, _oracle(w))


def test_automatic_sort_choice_follows_the_beam_size():
    """The default cadence (-1) tiles and re-sorts only from 32768 particles
    up; either way the run matches the oracle."""
    from paper_2511_21839_amd import dpic

    for n, sorted_run in ((3000, False), (40000, True)):
        w = synth.tiny(n_particles=n, grid=16, steps_per_element=3)
        sim = make_sim(w, sort_every=None)
        assert sim.get_option(dpic.OPT_SORT_EVERY) == -1
        sim.set_option(dpic.OPT_STAGE_TIMING, 1)
        sim.stage_times()
        sim.step(w.total_steps())
        _, launches = sim.stage_times()
        assert (launches[3] > 0) == sorted_run, (n, launches)
        sim.set_option(dpic.OPT_STAGE_TIMING, 0)
        _compare_run(w, sim, _oracle(w))


def test_tiled_deposit_with_drift_beyond_the_halo():
    # large momentum spread and a single sort: many particles leave their
    # tile's LDS window and take the global-atomic path of the tiled kernel
    w = synth.tiny(n_particles=3000, grid=32, steps_per_element=4)
    w = w.with_(sigma=(1e-3, 6e-3, 1e-3, 6e-3, 2e-3, 1e-3), bunch_charge_C=w.bunch_charge_C * 5)
    sim = make_sim(w, sort_every=1000)
    sim.step(w.total_steps())
    _compare_run(w, sim, _oracle(w))


def test_split_calls_match_one_schedule():
    w = synth.tiny(n_particles=1500, grid=16, steps_per_element=4)
    sim = make_sim(w)
    for n in (1, 6, 13):
        sim.step(n)
    _compare_run(w, sim, _oracle(w))


def test_thirteen_tangents_with_sigma_seeds():
    w = synth.tiny(n_particles=2000, grid=16, steps_per_element=3, ntan=13, sigma_tangents=True)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 10)
    sim = make_sim(w)
    sim.step(w.total_steps())
    _compare_run(w, sim, _oracle(w))


def test_value_only_run():
    w = synth.tiny(n_particles=2500, grid=32, steps_per_element=4, ntan=0)
    sim = make_sim(w)
    sim.step(w.total_steps())
    _compare_run(w, sim, _oracle(w))


def test_non_cubic_grid_run():
    w = synth.tiny(n_particles=2048, grid=16, steps_per_element=3).with_(grid=(16, 32, 8))
    sim = make_sim(w)
    sim.step(w.total_steps())
    _compare_run(w, sim, _oracle(w))


def test_particles_outside_box_are_counted_and_skipped():
    # a box narrower than the beam in x: the outer particles are lost to the
    # field but keep being pushed by the lattice
    w = synth.tiny(n_particles=1200, grid=16, steps_per_element=3)
    w = w.with_(lo=(-2.0e-3, -8e-3, -9.2e-3), hi=(2.0e-3, 8e-3, 9.2e-3))
    sim = make_sim(w)
    sim.step(w.total_steps())
    ref = _oracle(w)
    assert ref.out_of_box > 0
    _compare_run(w, sim, ref)


def test_empty_beam_and_schedule_end():
    from paper_2511_21839_amd import dpic

    w = synth.tiny(n_particles=64, grid=16, steps_per_element=2)
    sim = make_sim(w)
    sim.init_beam(np.zeros((0, 6)), w.sigma)
    sim.step(3)
    oob, steps, _ = sim.counters()
    assert (oob, steps) == (0, 3)
    with pytest.raises(dpic.DpicError):
        sim.step(w.total_steps())  # past the end of the schedule


def test_capacity_larger_than_beam():
    w = synth.tiny(n_particles=1000, grid=16, steps_per_element=3)
    sim = make_sim(w, capacity=5000)
    sim.step(w.total_steps())
    _compare_run(w, sim, _oracle(w))


def test_checkpoint_round_trip():
    import torch
    from paper_2511_21839_amd import dpic

    w = synth.tiny(n_particles=1000, grid=16, steps_per_element=4)
    sim = make_sim(w, sort_every=2)
    sim.step(7)
    buf = torch.empty(dpic.dpic_state_bytes(sim.ctx), dtype=torch.uint8, device="cuda")
    dpic.dpic_save_state(sim.ctx, buf.data_ptr())
    sim.step(13)
    a = sim.particles()
    dpic.dpic_load_state(sim.ctx, buf.data_ptr())
    assert sim.counters()[1] == 7
    sim.step(13)
    b = sim.particles()
    assert normwise_err(b, a) <= 1e-12
    _compare_run(w, sim, _oracle(w))


def test_c1_full_run_matches_oracle():
    w = synth.c1()
    sim = make_sim(w, sort_every=10)
    sim.step(w.total_steps())
    _compare_run(w, sim, _oracle(w))


def test_off_centre_beam_centred_emittance():
    """A beam displaced by half a sigma in x and y (and by 0.2 sigma in the
    momenta): the centred emittance differs from the raw one, and both
    match the oracle."""
    w = synth.tiny(n_particles=2500, grid=16, steps_per_element=4)
    w = w.with_(bunch_charge_C=w.bunch_charge_C * 5)
    xi = w.xi()
    xi[:, 0] += 0.5
    xi[:, 2] -= 0.5
    xi[:, 1] += 0.2
    xi[:, 3] += 0.2
    sim = make_sim(w, xi=xi)
    sim.step(w.total_steps())
    ref = pic.simulate_workload(w, xi=xi)
    _compare_run(w, sim, ref)
    raw, cen = pic.emittance(ref.moments), pic.emittance(ref.moments, centred=True)
    assert np.abs(raw[:2, 0] - cen[:2, 0]).min() > 1e-2 * cen[:2, 0].min()
